"""Build-level check of the device code (CPU only, needs hipcc).

No kernel may use scratch (private) memory.  A dynamically indexed local array
in a kernel lives in scratch, and one such array (vertex coordinates indexed
by a runtime vertex count) was miscompiled for gfx950 into a load at an
undefined scratch offset on one branch; every kernel therefore keeps its local
arrays compile-time indexed, which this test enforces.
"""
import os
import re
import subprocess

import pytest

from paper_1507_02557_amd import build as B

SOURCES = [s for s in B.SOURCES if s.endswith(".hip")]


@pytest.mark.parametrize("src", SOURCES)
def test_kernels_use_no_scratch(src, tmp_path):
    hipcc = B._hipcc()
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    cmd = [hipcc, *B.FLAGS, "-c", os.path.join(B.CSRC, src), "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    sizes = [int(m) for m in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert sizes, "no resource-usage remarks parsed"
    assert max(sizes) == 0, sizes
