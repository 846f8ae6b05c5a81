"""The persistent-grid residency rule (dawn_api.hip, resident_per_cu) against
the compiler's own occupancy figure for every persistent kernel, on the CPU:
the kernels are compiled for gfx950 (device code only) with the compiler's
resource-usage remarks, and for each persistent kernel the rule's waves per
SIMD from its VGPR count must equal the occupancy the compiler reports (which
also accounts for SGPRs and LDS).  A kernel that the rule would over-count
fails here before it ever runs."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_07872_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _remarks(src, tmp_path):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
           "-fno-gpu-flush-denormals-to-zero", "-ffp-contract=off", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-c", os.path.join(CSRC, src),
           "-o", str(tmp_path / (src + ".o")), "-Rpass-analysis=kernel-resource-usage"]
    p = subprocess.run(cmd, capture_output=True, text=True, check=True)
    kernels, cur = {}, None
    for line in p.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark: .*?(VGPRs|AGPRs|Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]"
                      r"|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1)] = int(m.group(2))
    return kernels


def rule_waves_per_simd(vgprs: int) -> int:
    return min(8, 512 // max(8, (vgprs + 7) // 8 * 8))


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
@pytest.mark.parametrize("src", ["govm_sssp.hip", "govm_tile.hip"])
def test_rule_matches_compiler_occupancy(src, tmp_path):
    ks = _remarks(src, tmp_path)
    pers = {k: v for k, v in ks.items() if "persistent_kernel" in k}
    assert pers, "no persistent kernel found"
    for name, r in pers.items():
        assert r.get("AGPRs", 0) == 0, name
        assert rule_waves_per_simd(r["VGPRs"]) == r["Occupancy [waves/SIMD]"], (name, r)
        assert r["LDS Size [bytes/block]"] <= 160 * 1024
