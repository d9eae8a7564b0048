"""The host side of the C-ABI library under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU, no GPU).

Every library source is compiled with the sanitizers on its host code only
(device code for gfx950 is built as usual) and linked with
tests/host_sanitize_driver.cpp, which calls every entry point that works on
the host (mixture set-up and lattice-unit constants for each cubic and N up
to the maximum, buffer sizes) and every argument check that returns before
the first device call (invalid descriptors, unphysical initial fields
scanned site by site, stepping and read-out argument errors, the batch
size limit of the allocation-free step).  An out-of-bounds access or
undefined arithmetic aborts the driver; a wrong status fails it.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2306_10652_amd", "csrc")
SOURCES = ["kernels_generic.hip", "kernels_fused2d.hip", "kernels_fused2d_ws.hip",
           "fuglbm_host.cpp"]
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not available")
    out = tmp_path_factory.mktemp("hostsan")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + HOST_SAN
    procs, objs = [], []
    for src in SOURCES:
        obj = str(out / (os.path.splitext(src)[0] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC] + common + ["-x", "hip", "-c",
                                       os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    drv = str(out / "driver.o")
    objs.append(drv)
    procs.append(subprocess.Popen([CLANG, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                   "-I" + os.path.join(ROOT, "include"), "-c",
                                   os.path.join(HERE, "host_sanitize_driver.cpp"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            pytest.fail("sanitizer build failed:\n" + err[-3000:])
    exe = str(out / "host_san")
    r = subprocess.run([CLANG, "-fsanitize=address,undefined"] + objs +
                       ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
                        "-lrocprofiler-sdk-roctx", "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("sanitizer link failed:\n" + r.stderr[-3000:])
    return exe


def test_host_library_clean_under_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    assert r.stdout.strip().endswith("OK")
