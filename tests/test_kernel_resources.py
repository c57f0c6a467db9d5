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
@pytest.mark.parametrize("src", ["rj_run_f32.hip", "rj_run_f32_mala.hip"])
def test_fp32_step_kernels_allow_two_waves(src):
    res = _resources(src)
    kernels = {k: v for k, v in res.items() if "run_kernel" in k}
    assert len(kernels) == 6, sorted(res)
    for name, r in kernels.items():
        assert r["VGPRs"] + r.get("AGPRs", 0) <= 256, (name, r)


@pytest.mark.slow
def test_homogeneous_plain_kernel_has_no_scratch():
    res = _resources("rj_run_f32.hip")
    hom = [k for k in res if k.startswith("_ZN2rj10run_kernelIfLi0ELb0E")]
    assert len(hom) == 2, sorted(res)
    for name in hom:
        assert res[name]["ScratchSize [bytes/lane]"] == 0, (name, res[name])
