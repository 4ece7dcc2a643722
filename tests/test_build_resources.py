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
