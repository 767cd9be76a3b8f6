"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU.

  * the oracle (plain C) built with gcc's sanitizers, under its own pin tests
    (models, invariants, views, thresholds);
  * the host code of the library (the big-integer threshold tables, the
    descriptor checks and sizing, the workspace layout, argument checks of
    every entry point before any device call) built with hipcc's host-only
    sanitizers, under the CPU tests of the boundary, the autotuner's host
    logic and the serving loop.

Each runs as a child process with the sanitizer runtime preloaded; any
report ends that process with a failure (no recovery)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_OPTS = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(env_extra, tests, timeout=900):
    env = dict(os.environ, **ENV_OPTS, **env_extra)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *tests]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    from oracle import build_oracle
    lib = build_oracle.build(sanitize=True, out=str(tmp_path / "liboracle_asan.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    out = _run({"LD_PRELOAD": asan, "AMBER_ORACLE_LIB": lib},
               ["tests/test_oracle_models.py", "tests/test_oracle_invariants.py",
                "tests/test_oracle_views.py", "tests/test_oracle_thresholds.py",
                "tests/test_oracle_async_log.py", "tests/test_oracle_environments.py",
                "tests/test_oracle_continuous.py"])
    assert " passed" in out


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    from paper_2601_16292_amd import build
    lib = build.build(sanitize_host=True, out=str(tmp_path / "libamber_asan.so"))
    out = _run({"LD_PRELOAD": build.asan_runtime(), "AMBER_LIB_PATH": lib},
               ["tests/test_abi.py", "tests/test_autotune.py", "tests/test_serve_logic.py",
                "tests/test_bench_pricing.py"])
    assert " passed" in out
