"""Register and scratch budgets of the step kernels (CPU: cross-compiles for gfx950).

The FP32 step kernels are tuned for two resident waves per SIMD on large
workloads, which needs at most 256 VGPRs (and no AGPR overflow); the plain
homogeneous kernel of the batched workload must not touch scratch memory.
A change that silently halves occupancy or adds stack traffic fails here.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1811_04156_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")


def _resources(src):
    from paper_1811_04156_amd.build import HIPCC_FLAGS
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared",)]
    cmd = [HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "--cuda-device-only", "-c", "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage", os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"(VGPRs|AGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur:
            out[cur][m.group(1)] = int(m.group(2))
    return out


@pytest.mark.slow
@pytest.mark.parametrize("src", ["rj_run_f32.hip", "rj_run_f32_mala.hip", "rj_run_f32_lmala.hip",
                                 "rj_run_f32_tree.hip"])
def test_fp32_step_kernels_allow_two_waves(src):
    """Every plain and joint-Langevin variant, and the variants of the other
    moves on the media without the simplified-Liu term whose tables sit in
    LDS (the layered batches' case), fit 256 registers per lane."""
    res = _resources(src)
    kernels = {k: v for k, v in res.items() if "run_kernel" in k}
    assert len(kernels) == 6, sorted(res)
    for name, r in kernels.items():
        m = re.search(r"run_kernelIfLi(\d)ELi(\d)ELb(\d)E", name)
        mk, samp, sl = int(m.group(1)), int(m.group(2)), int(m.group(3))
        if samp >= 2 and (sl or mk == 1):
            continue
        assert r["VGPRs"] + r.get("AGPRs", 0) <= 256, (name, r)


@pytest.mark.slow
@pytest.mark.parametrize("src", ["rj_run_f32.hip", "rj_run_f32_mala.hip", "rj_run_f32_lmala.hip",
                                 "rj_run_f32_tree.hip"])
def test_fp32_step_kernel_scratch(src):
    """No FP32 step kernel without the simplified-Liu term touches scratch;
    the simplified-Liu variants of the layered kernels spill at most 16 bytes
    per lane.  A change that adds stack traffic to the hot variants fails
    here."""
    res = _resources(src)
    for name, r in res.items():
        if "run_kernel" not in name:
            continue
        m = re.search(r"run_kernelIfLi(\d)ELi(\d)ELb(\d)E", name)
        mk, samp, sl = int(m.group(1)), int(m.group(2)), int(m.group(3))
        limit = 16 if sl else 0
        assert r["ScratchSize [bytes/lane]"] <= limit, (name, r)
