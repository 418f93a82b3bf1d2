"""Host-side checks of what the kernels and the server rely on, run on the CPU
from the library's own code:

* the device index arithmetic (cooling lane ownership, XCD region order,
  launch-slot mapping, the reduction butterfly), compiled for the host from
  the kernels' headers (tests/hostcheck/index_checks.hip);
* the server's admission rule and first-fit arena allocator on a fake clock
  (tests/hostcheck/sched_checks.cpp, g++ only);
* the oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1311_1056_amd", "csrc")
HC = os.path.join(ROOT, "tests", "hostcheck")
BUILD = os.path.join(ROOT, "tests", "_build")


def _stale(exe, deps):
    return not os.path.exists(exe) or any(os.path.getmtime(d) > os.path.getmtime(exe) for d in deps)


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout
    return r.stdout


def test_device_index_arithmetic_on_host():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "index_checks")
    src = os.path.join(HC, "index_checks.hip")
    deps = [src] + [os.path.join(CSRC, f) for f in ("lattice.hpp", "engine.hpp", "reduce.hpp", "su3.hpp")]
    if _stale(exe, deps):
        subprocess.check_call([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-I", CSRC,
                               "-I", os.path.join(ROOT, "include"), src, "-o", exe])
    out = _run(exe)
    assert out.count("ok cooling lanes own every link once") >= 10
    assert out.count("ok omega blocks cover every chunk once") >= 10


def test_server_admission_and_allocator_on_a_fake_clock():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "sched_checks")
    src = os.path.join(HC, "sched_checks.cpp")
    if _stale(exe, [src, os.path.join(CSRC, "sched.hpp")]):
        subprocess.check_call([gxx, "-O2", "-std=c++17", "-Wall", "-I", CSRC, src, "-o", exe])
    _run(exe)


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_under_address_and_ub_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    env = dict(os.environ)
    env.update(CLGC_ORACLE_SANITIZE="1", LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    # build the sanitized oracle in a process without the preload (gcc itself)
    subprocess.check_call([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT,
                          env={**os.environ, "CLGC_ORACLE_SANITIZE": "1"})
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_observables.py", "test_oracle_dynamics.py", "test_oracle_chain.py", "test_oracle_philox.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=1200)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert " passed" in r.stdout
