"""Energy and difference reductions on the GPU (the diagnostic reductions of
the primal-dual solve): the linearised energy of Eq. (10) against the FP64
oracle's, the per-iteration energy trace of the primal-dual iteration
against the oracle's trace, run-to-run determinism, and masked difference
statistics against numpy.  Inputs: the seeded level problems of the step
tests (C1 128x128, the ragged 200x136 rig, C2 level 0)."""
import numpy as np
import pytest

import oracle
from synth import configs
from tests.test_gpu_steps import _np, _pd_state, _t, f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vfs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_07545_amd as v
    return v


def _tpack(T, Iu):
    return np.concatenate([T, Iu[..., None]], -1).astype(np.float32)


@pytest.mark.parametrize("cid,reg", [("c1", "tgv"), ("r200", "tgv"), ("r200", "tv"), ("c2", "tgv")])
def test_energy_matches_oracle(vfs, cid, reg):
    """E of a state: FP32 per-pixel terms with FP64 accumulation against the
    FP64 oracle on the same float32 inputs, relative 1e-6; bitwise the same
    on a second call."""
    flags, T, Iu, rho, u, v, p, q = _pd_state(cid, 0, reg == "tgv")
    params = dict(configs.PAPER_PARAMS, levels=1, warps=1, iters=1, reg=reg)
    tv = _t(v) if reg == "tgv" else None
    e1 = vfs.step_energy(_t(_tpack(T, Iu)), _t(rho), _t(flags), _t(u), tv, params)
    e2 = vfs.step_energy(_t(_tpack(T, Iu)), _t(rho), _t(flags), _t(u), tv, params)
    eo = oracle.energy(params, f32(T), flags & 1, f32(Iu), f32(rho), f32(u), f32(v) if reg == "tgv" else None)
    assert e1 == e2
    assert abs(e1 - eo) <= 1e-6 * abs(eo), (e1, eo)


@pytest.mark.parametrize("cid,K,reg", [("c1", 30, "tgv"), ("r200", 25, "tv"), ("r200", 12, "tgv")])
def test_energy_trace_matches_oracle(vfs, cid, K, reg):
    """E(x^0) ... E(x^K) of K primal-dual iterations against the oracle's
    trace (relative 1e-5: the FP32 iterates drift ~1e-7 per iteration), and
    the final state against the two-iterations-per-launch path (2e-5)."""
    import torch
    tgv = reg == "tgv"
    flags, T, Iu, rho, u, v, p, q = _pd_state(cid, 0, tgv)
    params = dict(configs.PAPER_PARAMS, levels=1, warps=1, iters=K, reg=reg)
    tp = _t(_tpack(T, Iu))
    tu, tpp = _t(u), _t(p)
    tv, tq = (_t(v), _t(q)) if tgv else (None, None)
    trace = vfs.step_pd_energy(tp, _t(rho), _t(flags), tu, tv, tpp, tq, params, K)
    m = flags & 1
    sp, su, sv = oracle.steps(f32(T), m, params["alpha0"], params["alpha1"], reg)
    st = oracle.pd_iterations(params, f32(T), m, sp, su, sv, f32(Iu), f32(rho), f32(u), f32(v), f32(p), f32(q), K,
                              trace=True)
    eo = st["energy"]
    assert trace.shape == (K + 1,)
    assert np.max(np.abs(trace - eo) / np.abs(eo)) < 1e-5
    # the same iterations through vfs_step_pd (two per launch)
    tu2, tp2 = _t(u), _t(p)
    tv2, tq2 = (_t(v), _t(q)) if tgv else (None, None)
    vfs.step_pd(tp, _t(rho), _t(flags), tu2, tv2, tp2, tq2, params, K)
    torch.cuda.synchronize()
    assert np.max(np.abs(_np(tu) - _np(tu2))) < 2e-5
    assert np.max(np.abs(_np(tu) - st["u"])) < 2e-5


@pytest.mark.parametrize("H,W,masked", [(128, 128, True), (136, 200, True), (77, 301, False)])
def test_diff_stats(vfs, H, W, masked):
    """Mean, max and count of |a - b| over a mask (or everything) against
    numpy in float64."""
    rng = np.random.default_rng(H * W)
    a = rng.normal(size=(H, W)).astype(np.float32)
    b = (a + rng.normal(0, 1e-3, (H, W))).astype(np.float32)
    b[3, 5] += 7.0
    flags = (rng.random((H, W)) < 0.8).astype(np.uint8) if masked else None
    mean, mx, cnt = vfs.diff_stats(_t(a), _t(b), _t(flags) if masked else None)
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    sel = flags.astype(bool) if masked else np.ones((H, W), bool)
    assert cnt == int(sel.sum())
    assert mx == d[sel].max()
    assert abs(mean - d[sel].mean()) <= 1e-12 * d[sel].mean()
