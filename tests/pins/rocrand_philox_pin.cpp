// Pin helper: evaluates one Philox4x32-10 block with ROCm's rocRAND engine
// (host build of its header-only generator) for every "k0 k1 c0 c1 c2 c3"
// line read from stdin, printing the 4 output words.  rocRAND maps the
// 64-bit seed to the key (low word, high word), the subsequence to counter
// words 2..3 and offset/4 to counter words 0..1.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(k0 | (k1 << 32), c2 | (c3 << 32), 0ull, &st);
        skipahead(4ull * c0, &st);
        // counter word 1 advances by c1 via four skips of 4*(c1 << 30) draws
        for (int i = 0; i < 4; i++) skipahead(c1 << 32, &st);
        unsigned int o[4];
        for (int i = 0; i < 4; i++) o[i] = rocrand(&st);
        std::printf("%u %u %u %u\n", o[0], o[1], o[2], o[3]);
    }
    return 0;
}
