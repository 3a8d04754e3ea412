"""The C oracle and the library's host code built under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): a driver program exercises every
oracle entry point on small images, another the library's host-side
argument validation (the dwt_fuse_check_* entry points and
dwt_fuse_status_str, valid and invalid arguments).  Any memory error or
undefined behaviour aborts the program; the test wants exit status 0 and no
sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]


def _have(cc):
    if shutil.which(cc) is None:
        return False
    r = subprocess.run([cc, "-print-file-name=libasan.so"], capture_output=True, text=True)
    return r.returncode == 0 and os.path.sep in r.stdout.strip()


def _run(exe, leaks):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=%d:abort_on_error=0:exitcode=23" % (1 if leaks else 0)
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report


@pytest.mark.skipif(not _have("gcc"), reason="gcc with AddressSanitizer not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11"] + SAN + ["-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_driver.c"),
                                       os.path.join(ROOT, "oracle", "dwt_oracle.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    _run(exe, leaks=True)


@pytest.mark.skipif(not _have("g++") or not os.path.exists(os.path.join(ROCM, "include", "hip")),
                    reason="g++ with AddressSanitizer or the HIP headers not available")
def test_host_validation_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1803_00737_amd", "csrc")
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "driver.o")
    exe = str(tmp_path / "abi_check_driver")
    steps = [
        ["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-DDWT_FUSE_BUILD_ID=\"sanitizer\"",
                                       "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
                                       "-I", csrc, "-c", os.path.join(csrc, "dwt_fuse_api.cpp"), "-o", api],
        ["gcc", "-std=c11"] + SAN + ["-I", os.path.join(ROOT, "include"), "-c",
                                     os.path.join(HERE, "abi_check_driver.c"), "-o", drv],
        # The kernels' launchers live in the device sources, which this host
        # build leaves out; the validation entry points never reach them.
        ["g++"] + SAN + [drv, api, "-o", exe, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                         "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-Wl,--unresolved-symbols=ignore-in-object-files"],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout + r.stderr
    _run(exe, leaks=False)
