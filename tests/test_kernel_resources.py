"""Register use of the hot kernels (CPU only: hipcc's resource report for
gfx950, no GPU needed).  The occupancy each kernel was measured fastest at
depends on how many registers the compiler allocates; these checks keep a
source or compiler change from silently dropping a kernel to fewer waves
per SIMD or making it spill."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2406_19920_amd import build

pytestmark = pytest.mark.skipif(not shutil.which(build.hipcc()) and not os.path.exists(build.hipcc()),
                                reason="no hipcc")


def _resources(src, tmp_path):
    """kernel (mangled) -> {'occupancy', 'vgpr_spill', 'lds'} from hipcc's
    kernel-resource-usage remarks for one source file."""
    cmd = [build.hipcc(), *build.FLAGS, "--offload-device-only", "-Rpass-analysis=kernel-resource-usage", "-c",
           os.path.join(build.CSRC, src), "-o", str(tmp_path / (src + ".o"))]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark:\s+(Occupancy \[waves/SIMD\]|VGPRs Spill|LDS Size \[bytes/block\]): (\d+)", line)
        if m and name:
            key = {"Occupancy [waves/SIMD]": "occupancy", "VGPRs Spill": "vgpr_spill",
                   "LDS Size [bytes/block]": "lds"}[m.group(1)]
            out[name][key] = int(m.group(2))
    return out


def _pick(res, pattern):
    hits = {k: v for k, v in res.items() if re.search(pattern, k)}
    assert hits, f"no kernel matches {pattern}"
    return hits


# (source, mangled-name pattern, least waves per SIMD); none may spill
EXPECT = [
    # FP64 folded transforms: the 256^3 tiles (x 2x2, z 4x1) at three waves
    ("k_fold.hip", r"xfold_f64_kernelILi2ELi2ELb[01]ELb0E", 3),
    ("k_fold.hip", r"zfold_f64_kernelILi4ELi1ELb[01]ELb0E", 3),
    # plain FP64 z transform (walls in z): two waves
    ("k_xform.hip", r"zgemm_f64_kernelILi4ELi4E", 2),
    # multi-grid stage kernels
    ("k_multigrid.hip", r"mg_xgemm_kernelILi2E", 3),
    ("k_multigrid.hip", r"mg_zgemm_kernelILi2E", 3),
    ("k_multigrid.hip", r"mg_tridiag_kernelILb0E", 7),
    # FP32 pencils of the refined path at 256 rows: four waves, 16-wave blocks
    ("k_tridiag.hip", r"tridiag_kernelIffLi32ELi8ELi32ELb0ELb[01]E", 4),
    # split z transform of the 256^3 step: one 8-wave block per CU (LDS)
    ("k_split.hip", r"split_zfold_kernelILi8ELi1ELb[01]ELi1E", 2),
]


@pytest.mark.parametrize("src", sorted({e[0] for e in EXPECT}))
def test_hot_kernels_keep_their_occupancy(src, tmp_path):
    res = _resources(src, tmp_path)
    for s, pattern, waves in EXPECT:
        if s != src:
            continue
        for name, r in _pick(res, pattern).items():
            assert r.get("vgpr_spill", 0) == 0, (name, r)
            assert r.get("occupancy", 0) >= waves, (name, r)
