"""Host code of the library under the sanitizers: the library's sources
compiled with them on their host pass only, linked with a C driver
(`host_sanitize_driver.c`) that makes the host-only calls (bank, length
classes, bank metric, lattice placement) with valid and invalid arguments.
Two builds: AddressSanitizer with UndefinedBehaviorSanitizer, and
ThreadSanitizer (the metric samples and lattice rows are placed on several
host threads).  Each run must end cleanly, with every documented return code
and no sanitizer report.  No GPU is used: none of these calls touches a
device."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1006_4644_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
# sanitizer options per build: for gcc (the driver), and for hipcc on the
# host pass only (the device pass gets none)
KINDS = {
    "asan_ubsan": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                   ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined"]),
    "tsan": (["-fsanitize=thread"], ["-Xarch_host", "-fsanitize=thread"]),
}
LINK = {"asan_ubsan": KINDS["asan_ubsan"][1][:4], "tsan": KINDS["tsan"][1]}


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    """Both instrumented executables, their compiles run side by side."""
    from paper_1006_4644_amd.build import hipcc
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    hip = hipcc()
    out = str(tmp_path_factory.mktemp("hostsan"))
    procs, objs = [], {}
    for kind, (gflags, hflags) in KINDS.items():
        drv = os.path.join(out, kind + "_driver.o")
        objs[kind] = [drv]
        procs.append(subprocess.Popen(
            [gcc, "-O1", "-g", *gflags, "-I", INCLUDE, "-c",
             os.path.join(ROOT, "tests", "host_sanitize_driver.c"), "-o", drv],
            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        # the device pass unoptimised: nothing runs on it
        for src in ("api", "bank", "kernels"):
            obj = os.path.join(out, f"{kind}_{src}.o")
            objs[kind].append(obj)
            procs.append(subprocess.Popen(
                [hip, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xarch_device", "-O0",
                 *hflags, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-I", INCLUDE, "-c", os.path.join(CSRC, src + ".hip"), "-o", obj],
                stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err
    exes = {}
    for kind in KINDS:
        exe = os.path.join(out, kind)
        r = subprocess.run([hip, "--offload-arch=gfx950", *LINK[kind], "-o", exe, *objs[kind]],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        exes[kind] = exe
    return exes


def _run(exe, env_extra):
    r = subprocess.run([exe], capture_output=True, text=True,
                       env=dict(os.environ, **env_extra), timeout=600)
    return r, r.stdout + r.stderr


def test_host_calls_under_asan_ubsan(builds):
    r, report = _run(builds["asan_ubsan"],
                     {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, report
    assert "host calls ok" in r.stdout
    assert "AddressSanitizer" not in report and "runtime error" not in report, report


def test_host_calls_under_tsan(builds):
    r, report = _run(builds["tsan"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert r.returncode == 0, report
    assert "host calls ok" in r.stdout
    assert "ThreadSanitizer" not in report, report
