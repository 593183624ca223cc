"""Register and scratch budgets of the HIP kernels (built for gfx950 here, on the CPU).

The kernels' speed rests on how many wavefronts fit a SIMD: 512 VGPRs per lane
are shared by the wavefronts of a SIMD, so 128 VGPRs allow 4, 168 allow 3 and
256 allow 2. The compiler's choice can move a long way on a small code change
(the angular leaf once went from 106 to 226 VGPRs, halving its workgroups per
CU), so each kernel's device code is compiled with the library's flags and its
metadata checked against the budget its design assumes.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2301_12191_amd import build as B

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, kernel symbol pattern, max VGPRs, max scratch bytes per lane[, max LDS bytes])
BUDGETS = [
    ("mr_kernels.hip", r"leaf_kernelILb1ELb0E", 128, 0),   # angular leaf: 4 waves/SIMD
    # leaf: 8 waves/SIMD and 8 workgroups of 256 threads per CU (160 KB of LDS / 8)
    ("mr_kernels.hip", r"leaf_kernelILb0ELb0E", 64, 0, 20480),
    ("mr_kernels.hip", r"leaf_kernelILb0ELb1E", 64, 0, 20480),
    ("mr_kernels.hip", r"prep_kernel", 64, 0),
    ("mr_kernels.hip", r"search_kernel_d8", 256, 0),       # D = 8: 2 waves/SIMD
    ("mr_kernels.hip", r"search_kernelILi4E", 168, 0),     # D = 4: 3 waves/SIMD
    ("mr_kernels.hip", r"search_kernelILi2E", 128, 0),
    ("mr_refine.hip", r"refine_kernel_q2", 128, 0),         # 4 waves/SIMD
    ("mr_refine.hip", r"refine_kernel_q1", 128, 0),
    ("mr_refine.hip", r"pad_kernel", 64, 0),
    ("mr_subpel.hip", r"subpel_kernel", 168, 64),           # 3 waves/SIMD
]


def _metadata(src, tmp_path):
    out = tmp_path / (src + ".s")
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(B.ROOT, "include"),
           "-I", B.CSRC, os.path.join(B.CSRC, src), "-o", str(out)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    kernels = {}
    for block in out.read_text().split("\n  - "):
        name = re.search(r"\.name:\s+(\S+)", block)
        vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
        priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        lds = re.search(r"\.group_segment_fixed_size:\s+(\d+)", block)
        if name and vgpr and priv and lds:
            kernels[name.group(1)] = (int(vgpr.group(1)), int(priv.group(1)), int(lds.group(1)))
    return kernels


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
def test_kernel_register_budgets(tmp_path):
    meta = {}
    for src in sorted({b[0] for b in BUDGETS}):
        meta[src] = _metadata(src, tmp_path)
    failures = []
    for src, pat, max_vgpr, max_priv, *max_lds in BUDGETS:
        hits = [(k, v) for k, v in meta[src].items() if re.search(pat, k)]
        assert hits, f"{pat}: no kernel in {src}"
        for k, (vgpr, priv, lds) in hits:
            if vgpr > max_vgpr or priv > max_priv or (max_lds and lds > max_lds[0]):
                failures.append(f"{k}: {vgpr} VGPRs (budget {max_vgpr}), "
                                f"{priv} scratch bytes (budget {max_priv}), {lds} LDS bytes")
    assert not failures, "\n".join(failures)
