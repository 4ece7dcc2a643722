"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (CPU
only): the library's host side (topology building, the coloring orders, every
host query, argument errors) through tests/sanitize/host_driver.cpp, and the
FP64 oracle through tests/sanitize/oracle_driver.c (every entry point, with
contacts, friction, damping, acceleration, the adjoint and the complex-step
build).  Device code is built without sanitizers and never launched."""
import os
import subprocess

import pytest

from paper_2403_06321_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:])
    return r


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    odir = os.path.join(ROOT, "oracle")
    flags = ["-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", *SAN]
    objs = []
    for src, extra in (("oracle_core.c", ["-DOR_COMPLEX=0"]), ("oracle_core.c", ["-DOR_COMPLEX=1"]),
                       ("oracle_prep.c", [])):
        out = str(tmp_path / f"{src}{len(objs)}.o")
        _run(["gcc", *flags, *extra, "-c", os.path.join(odir, src), "-o", out])
        objs.append(out)
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", *flags, os.path.join(HERE, "sanitize", "oracle_driver.c"), *objs, "-o", exe, "-lm"])
    r = _run([exe], env=ENV)
    assert "oracle driver:" in r.stdout


@pytest.mark.slow
def test_host_library_under_address_and_undefined_sanitizers(tmp_path):
    # -fno-gpu-sanitize: the sanitizers apply to the host code only
    flags = ["-O1", "-g", "-std=c++17", *SAN, "-fno-gpu-sanitize", "-I", os.path.join(ROOT, "include")]
    arch = f"--offload-arch={B.ARCH}"
    objs = []
    for src in B.SOURCES:
        out = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([B.HIPCC, *flags, "-fPIC", arch, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              *lang, "-c", os.path.join(B.CSRC, src), "-o", out])
        objs.append(out)
    drv = str(tmp_path / "driver.o")
    _run([B.HIPCC, *flags, "-c", os.path.join(HERE, "sanitize", "host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "host_driver")
    _run([B.HIPCC, arch, *SAN, "-fno-gpu-sanitize", drv, *objs, *B.LIBS, "-o", exe])
    r = _run([exe], env=ENV)
    assert "all calls behaved" in r.stdout
