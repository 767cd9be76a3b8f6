"""Build libamber.so (the gfx950 HIP kernels and the C ABI) in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libamber.so")

SOURCES = ["amber_device.hip", "amber_batch.hip", "amber_tiled.hip", "amber_views.hip",
           "amber_async.hip", "amber_env.hip", "amber_cont.hip", "amber_noalloc.hip",
           "amber_host.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result", "-fvisibility=hidden",
    # keep the compiler from emitting packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


# host code only: the device code of a sanitized build is the ordinary one
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host",
                 "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize_host: bool = False, out: str = None) -> str:
    """libamber.so in-tree; with sanitize_host, a build whose host code has
    AddressSanitizer and UndefinedBehaviorSanitizer (load it with the
    compiler's ASan runtime preloaded) at `out`."""
    lib = out or LIB
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    cmd = [hipcc(), *HIP_FLAGS, *(SANITIZE_HOST if sanitize_host else []), "-I", INCLUDE,
           "-I", CSRC, *srcs, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out_text = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                         if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        sys.stderr.write(out_text + "\n")
        raise RuntimeError("hipcc failed building libamber.so")
    if verbose and out_text:
        print(out_text)
    os.replace(lib + ".tmp", lib)
    return lib


def asan_runtime() -> str:
    """The ASan runtime of the compiler behind hipcc (to preload for a
    sanitized build)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    hits = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")) +
                  glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found")
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose=True))
