"""Host-side memory and undefined-behaviour checks (no GPU).

The oracle (gcc, AddressSanitizer + UndefinedBehaviorSanitizer) and the host
code of the HIP library (clang, the same sanitizers on the host pass only;
the device code is built as usual) are built into a temporary directory, and
the CPU tests that drive them run in a child process with the sanitizer
runtime preloaded:
* the oracle's pins of the heat bath, margins, lattice, wave function,
  sampler and the learned correction;
* the C-ABI tests (every declared symbol, argument validation before any
  device work, spacing choice) and the host helpers.
A sanitizer report anywhere fails the test; the reports go to files so that
the child's own output capture cannot hide them.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.slow


def _runtime(kind):
    if kind == "gcc":
        out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
        return out if os.path.isabs(out) and os.path.exists(out) else None
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return rts[-1] if rts else None


def _run_tests(tmp, preload, env_extra, tests, tag):
    log = os.path.join(tmp, f"{tag}-report")
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS=f"detect_leaks=0:log_path={log}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={log}", **env_extra)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join(ROOT, "tests", t) for t in tests]]
    res = subprocess.run(cmd, cwd=tmp, env=env, capture_output=True, text=True, timeout=900)
    reports = glob.glob(log + "*")
    text = "".join(open(r).read() for r in reports)
    assert not reports, f"{tag}: sanitizer report\n{text[:4000]}"
    assert res.returncode == 0, f"{tag}: child tests failed\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    rt = _runtime("gcc")
    if rt is None or shutil.which("gcc") is None:
        pytest.skip("gcc AddressSanitizer runtime not available")
    lib = os.path.join(tmp_path, "liblrdmc_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
                    os.path.join(ROOT, "oracle", "lrdmc_oracle.c"), "-o", lib, "-lm"], check=True)
    out = _run_tests(str(tmp_path), rt, {"LRDMC_ORACLE_LIB": lib},
                     ["test_oracle_margins.py", "test_oracle_lattice.py", "test_oracle_wavefunction.py",
                      "test_oracle_sampler.py", "test_oracle_neural.py", "test_oracle_vmc.py",
                      "test_oracle_modes.py", "test_oracle_jastrow_grad.py", "test_oracle_drop.py",
                      "test_oracle_rng.py"], "oracle")
    assert "passed" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    rt = _runtime("clang")
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or the clang AddressSanitizer runtime not available")
    lib = os.path.join(tmp_path, "liblrdmc_san.so")
    src = os.path.join(ROOT, "paper_1909_01589_amd", "csrc", "lrdmc.hip")
    host_san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer", "-shared-libsan"):
        host_san += ["-Xarch_host", flag]
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-shared", "-std=c++17",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(src), src, "-o", lib],
                   check=True, capture_output=True)
    out = _run_tests(str(tmp_path), rt, {"LRDMC_LIB": lib}, ["test_abi.py", "test_host_helpers.py"], "library")
    assert "passed" in out
