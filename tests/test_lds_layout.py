"""The label permutations of the fused passes address LDS rows by XOR-ing a
byte offset below 4q into a row base, which assumes the kernel's dynamic LDS
array is its only LDS and so starts 4q-aligned.  Any static LDS in these
kernels (for instance from a library workgroup reduction) shifts the dynamic
array and silently corrupts the permutations for large q, so the assembly of
the GF(256) instance (the largest rows) is checked: every fused and
edge-parallel kernel reports no static LDS (group_segment_fixed_size 0)."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_1008_4370_amd import build


def test_fused_kernels_have_no_static_lds():
    try:
        cc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    src = os.path.join(build.CSRC, "kernels_q.hip")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "kq8.s")
        flags = [f for f in build.HIPCC_FLAGS if f != "-fPIC"]
        res = subprocess.run([cc, *flags, "-DLDPC_FD_LOGQ=8", "--cuda-device-only", "-S", "-o", out, src],
                             capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-2000:]
        text = open(out).read()
    meta = text[text.index("amdhsa.kernels:"):]
    seen = 0
    for entry in meta.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", entry).group(1)
        if "k_fused" not in name:
            continue
        seen += 1
        lds = int(re.search(r"\.group_segment_fixed_size:\s+(\d+)", entry).group(1))
        assert lds == 0, (name, lds)
    assert seen >= 40
