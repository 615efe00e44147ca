"""Host code of the library under AddressSanitizer and UndefinedBehavior-
Sanitizer: the library's sources compiled with both sanitizers on their host
pass only, linked with a C driver (`host_sanitize_driver.c`) that makes the
host-only calls (bank, length classes, bank metric, lattice placement) with
valid and invalid arguments.  The run must end cleanly, with every
documented return code and no sanitizer report.  No GPU is used: none of
these calls touches a device."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1006_4644_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
# sanitizers on the host pass only (the device pass gets none)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


def test_host_calls_under_sanitizers(tmp_path):
    from paper_1006_4644_amd.build import hipcc
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    hip = hipcc()
    out = str(tmp_path)
    drv = os.path.join(out, "driver.o")
    r = subprocess.run([gcc, "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", INCLUDE, "-c",
                        os.path.join(ROOT, "tests", "host_sanitize_driver.c"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # the three sources in parallel; the device pass unoptimised (nothing runs on it)
    objs, procs = [], []
    for src in ("api", "bank", "kernels"):
        obj = os.path.join(out, src + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen(
            [hip, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xarch_device", "-O0",
             *SAN, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE,
             "-c", os.path.join(CSRC, src + ".hip"), "-o", obj],
            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err
    exe = os.path.join(out, "hostsan")
    r = subprocess.run([hip, "--offload-arch=gfx950", *SAN[:4], "-o", exe, drv, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "host calls ok" in r.stdout
    assert "AddressSanitizer" not in report and "runtime error" not in report, report
