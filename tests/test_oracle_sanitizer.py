"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle's own CPU tests (all but the long evolutions) run in a child process
that loads the sanitizer build of the library, with every finding fatal."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FILES = ["test_oracle_ppm.py", "test_oracle_state_flux.py", "test_oracle_status.py",
         "test_oracle_invariants.py", "test_oracle_variants.py", "test_oracle_subgrid16.py",
         "test_oracle_cw84.py"]
# the multi-step evolutions (Sod tubes, the advected contact) only repeat
# the calls the others make, at a hundred times the cost under the sanitizer
DESELECT = "not sod and not advected"


def _runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_tests_pass_under_the_sanitizers():
    asan = _runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    for n in oracle.SUBGRID_SIZES:
        oracle.build(force=True, n=n, san=True)
    env = dict(os.environ, HYDRO_REF_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = subprocess.run(
        [sys.executable, "-c", "import oracle; print(oracle.lib()._name); print(oracle.lib(16)._name)"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    names = probe.stdout.split()
    assert names and all(n.endswith("_san.so") for n in names), probe.stdout
    run = subprocess.run(
        [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
         "-k", DESELECT, *[os.path.join(HERE, f) for f in FILES]],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (run.stdout + run.stderr)[-3000:]
    assert run.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert " passed" in run.stdout, tail
