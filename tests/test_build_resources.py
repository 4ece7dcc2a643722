"""Every gfx950 kernel of the library compiles without private-memory
(scratch) spills: a spill turns the register-resident per-lane element sums
into memory traffic.  Uses the compiler's resource-usage remarks (CPU only)."""
import os
import re
import subprocess

import pytest

from paper_2403_06321_amd import build as B


@pytest.mark.parametrize("src", [s for s in B.SOURCES if s.endswith(".hip")])
def test_no_scratch_in_any_kernel(src, tmp_path):
    cmd = [B.HIPCC, *B.COMMON, "-x", "hip", "-c", os.path.join(B.CSRC, src),
           "-o", str(tmp_path / "k.o"), "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    has_kernels = "__global__" in open(os.path.join(B.CSRC, src)).read()
    assert bool(names) == has_kernels and len(names) == len(scratch)
    spilled = [n for n, s in zip(names, scratch) if s != 0]
    assert not spilled, f"kernels with scratch: {spilled[:5]}"


def test_persistent_kernels_fit_the_grid_residency(tmp_path):
    """The persistent kernel's grid barrier needs every block resident.  The
    host fills kPersistentWavesPerSimd waves per SIMD; every k_persistent
    instantiation must be compiled for at least that occupancy (the
    compiler's own figure, which counts the SGPR and VGPR limits that the
    runtime's occupancy query can miss)."""
    src = os.path.join(B.CSRC, "vbd_kernels.hip")
    hdr = open(os.path.join(B.CSRC, "vbd_internal.h")).read()
    want = int(re.search(r"constexpr int kPersistentWavesPerSimd = (\d+);", hdr).group(1))
    cmd = [B.HIPCC, *B.COMMON, "-x", "hip", "-c", src, "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    blocks = re.split(r"remark: Function Name: ", r.stderr)[1:]
    occ = {}
    for blk in blocks:
        name = blk.split()[0]
        m = re.search(r"Occupancy \[waves/SIMD\]: (\d+)", blk)
        if "k_persistent" in name and m:
            occ[name] = int(m.group(1))
    assert len(occ) >= 10, f"persistent instantiations found: {len(occ)}"
    low = {n: o for n, o in occ.items() if o < want}
    assert not low, f"persistent kernels below {want} waves/SIMD: {low}"
