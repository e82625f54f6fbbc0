"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): every source is compiled with the sanitizers on its host side only
(the gfx950 device code is built as usual, without them), linked with
host_sanitized_checks.cpp, and run.  That program exercises descriptor and
wave validation, the footprint estimate, the NULL refusals, context
creation without a usable device and the server's admission pass under a
fake executor; the test fails on any unexpected status or any sanitizer
report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0704_2344_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not installed")
def test_host_code_is_clean_under_sanitizers(tmp_path):
    common = ["-O1", "-g", "-fPIC", "-std=c++17", f"-I{ROOT}/include", f"-I{CSRC}"]
    objs = []
    procs = []
    for name in sorted(os.listdir(CSRC)):
        if not name.endswith((".hip", ".cpp")):
            continue
        obj = str(tmp_path / (name + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, "-x", "hip"] + DEVICE + common + SAN +
                                      ["-c", os.path.join(CSRC, name), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    drv = str(tmp_path / "checks.o")
    r = subprocess.run([CLANG] + common + ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-c",
                        os.path.join(ROOT, "tests", "host_sanitized_checks.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "host_checks")
    r = subprocess.run([CLANG, "-fsanitize=address,undefined", drv] + objs +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ)
    # leaks inside the HIP runtime's own start-up are not this library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "runtime error" not in r.stderr, r.stderr
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 unexpected" in r.stdout
