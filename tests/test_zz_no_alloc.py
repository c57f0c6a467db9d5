"""rjpath_intensity_noalloc (the entry point for callers that cannot
allocate) against rjpath_intensity on the same chains: two calls in a row,
the second with a smaller input, and the size limit of its static buffer."""
import numpy as np
import pytest

from paper_1811_04156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_04156_amd import rjpath
    rjpath.load()
    return rjpath


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(a)
    assert np.allclose(a[ok], b[ok], rtol=1e-12, atol=0), np.max(np.abs(a[ok] / b[ok] - 1))


def _check(s, groups, pass_anchor):
    ref = s.intensity(groups=groups)  # host finalisation, workspace in the handle
    anc = torch.as_tensor(ref["anchor"], device=s.dev) if pass_anchor else None
    out = s.intensity_noalloc(groups=groups, anchor=anc)
    torch.cuda.synchronize()
    for k in ("I", "se", "ess", "rhat"):
        _same(out[k].cpu().numpy(), ref[k])
    assert np.isfinite(ref["I"]).sum() > 0


def test_noalloc_intensity_matches_intensity(rj):
    # first call: 64 targets x 256 chains (layered, contiguous pairs), anchors on the device
    w = W.layered_pairs(pairs=64, chains=64 * 256, cap=64, n_layers=12, dz=6.0, dmin=5.0, dmax=20.0)
    w["burn_in"] = 100
    s = rj.Sampler(w, precision="f32")
    s.run(400)
    _check(s, 16, pass_anchor=False)
    # second call, smaller input: 8 homogeneous targets x 128 chains, caller's anchors
    w2 = W.homogeneous_groups(groups=8, per_group=128, cap=32)
    w2["burn_in"] = 50
    s2 = rj.Sampler(w2, precision="f32")
    s2.run(300)
    _check(s2, 8, pass_anchor=True)
    # and the first sampler again after more steps (the buffer keeps the last call's contents)
    s.run(100)
    _check(s, 16, pass_anchor=True)


def test_noalloc_rejects_inputs_beyond_its_buffer(rj):
    w = W.homogeneous_groups(groups=1400, per_group=1, cap=16)
    s = rj.Sampler(w, precision="f32")
    with pytest.raises(rj.RJPathError, match="exceeds its static buffer"):
        s.intensity_noalloc(groups=64)
