"""The planner and the C ABI's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): plan.cpp and fcc_api.cpp are rebuilt
with g++ -fsanitize=address,undefined, linked with the library's device
objects as built, and tests/host/sanitize_driver.cpp drives every planner
refusal, the host queries and the basis export for every precision, the
argument errors of the device calls, the batch refusals and layout, and the
FCC_FAULT failure injection.  Nothing reaches the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_13622_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2204_13622_amd", "_build")


def _device_objects():
    from paper_2204_13622_amd import build as B
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s.endswith(".hip")]
    return objs if all(os.path.exists(o) for o in objs) else None


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("g++ or the HIP headers are missing")
    objs = _device_objects()
    if objs is None:
        from paper_2204_13622_amd import build as B
        B.build()
        objs = _device_objects()
    out = tmp_path_factory.mktemp("asan")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host = []
    for src in ("plan.cpp", "fcc_api.cpp"):
        o = str(out / (src + ".o"))
        subprocess.run([gxx] + flags + ["-c", os.path.join(CSRC, src), "-o", o], check=True)
        host.append(o)
    drv = str(out / "driver.o")
    subprocess.run([gxx] + flags + ["-c", os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"), "-o", drv],
                   check=True)
    exe = str(out / "sanitize_driver")
    subprocess.run([gxx, "-fsanitize=address,undefined", "-o", exe, drv] + host + objs +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    return exe


def test_host_code_under_sanitizers(driver):
    env = dict(os.environ)
    env.pop("FCC_FAULT", None)
    # leaks inside the HIP runtime's own start-up are not ours; every plan and
    # batch the driver creates is destroyed, which the exit code checks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([driver], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-4000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "OK: 0 failed checks" in r.stdout
