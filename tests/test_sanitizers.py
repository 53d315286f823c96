"""Host AddressSanitizer / UndefinedBehaviorSanitizer runs (CPU only, no device work).

* The oracle (oracle/pt_oracle.c), built with gcc -fsanitize=address,undefined into a driver that
  tracks particles through small random and degenerate grids in every mode (endpoint, snapshots,
  pathline records with small capacities, transient steps, a quadtree with split faces).
* libpt's host code (argument validation, handle bookkeeping, shutdown), built by hipcc with the
  sanitizers on the host side only, called from a driver whose every call fails validation,
  finds no device or is a no-op -- so the host checks read exactly sized arrays under ASan.

Both drivers exit 0 only if every call returned the expected code; any sanitizer report (a
non-zero exit through halt_on_error, or its message) fails the test.  The paper's explicit
data-sharing declarations (Methods "Multiprocessing") are the CPU analogue of what these check:
no access outside what each routine owns."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe, env):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    bad = ("AddressSanitizer" in r.stderr) or ("runtime error" in r.stderr) or ("LeakSanitizer" in r.stderr)
    assert r.returncode == 0 and not bad, r.stderr[-3000:]
    return r.stdout


def test_oracle_under_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-o", exe,
               os.path.join(HERE, "native", "oracle_sanitize.c"), "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        assert "oracle sanitize run ok" in _run(exe, ENV)


def test_library_host_validation_under_sanitizers():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang not available")
    import torch
    if torch.cuda.is_available():
        pytest.skip("runs where no device is present: every call must stop before device work")
    csrc = os.path.join(ROOT, "paper_2302_13590_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "libpt_asan.so")
        # sanitizers on the host code only: each -fsanitize= follows -Xarch_host; the device code,
        # which this driver never launches, is built without optimisation to save time
        build = [HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-std=c++17", "-fPIC", "-shared",
                 "-ffp-contract=off", "-Xarch_host", "-g",
                 "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-I", inc, "-o", lib,
                 os.path.join(csrc, "pt_kernels.hip"), os.path.join(csrc, "pt_api.hip")]
        subprocess.check_call(build, stderr=subprocess.DEVNULL)
        exe = os.path.join(d, "abi_sanitize")
        subprocess.check_call([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                               "-I", inc, "-o", exe, os.path.join(HERE, "native", "abi_sanitize.c"), "-L", d,
                               "-lpt_asan", "-Wl,-rpath," + d])
        # the HIP runtime itself is not instrumented and keeps allocations until exit
        env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
        assert "libpt sanitize run ok" in _run(exe, env)
