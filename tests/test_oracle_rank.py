"""Pins of the oracle's rank-transform (a census variant) and gradient-magnitude
data terms (the paper allows any image in its data term, Sec. III-A).

- The transform against its definition written out in plain Python loops on
  small images, ties included.
- Exact invariance under strictly increasing intensity maps (gain, offset,
  a tanh curve) and under transposition of the image.
- The whole method on the 128x128 plane with an illumination change of I1
  (gain 1.25, offset 0.03, plus a tanh curve): the rank data term recovers
  the rendered correspondences about as well as without the change, the
  brightness data term does not.
"""
import numpy as np
import pytest

import oracle
from synth import configs
from tests.conftest import inputs


def _rank_by_definition(I, r):
    H, W = I.shape
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            darker = 0
            for di in range(-r, r + 1):
                for dj in range(-r, r + 1):
                    if di == 0 and dj == 0:
                        continue
                    y = min(max(i + di, 0), H - 1)
                    x = min(max(j + dj, 0), W - 1)
                    if I[y, x] < I[i, j]:
                        darker += 1
            out[i, j] = darker / ((2 * r + 1) ** 2 - 1)
    return out


@pytest.mark.parametrize("shape,r", [((7, 9), 2), ((5, 4), 1), ((11, 6), 3)])
def test_rank_transform_by_definition(shape, r):
    rng = np.random.default_rng(sum(shape) + r)
    for I in (rng.random(shape), np.round(rng.random(shape) * 4) / 4):   # the second has ties
        assert np.array_equal(oracle.rank_transform(I, r), _rank_by_definition(I, r))


def test_rank_transform_invariances():
    rng = np.random.default_rng(5)
    I = rng.random((40, 57))
    R = oracle.rank_transform(I, 2)
    for g in (lambda x: 1.7 * x + 0.2, lambda x: np.tanh(3.0 * x - 1.0), lambda x: x ** 3 - 5.0):
        assert np.array_equal(oracle.rank_transform(g(I), 2), R)
    assert np.array_equal(oracle.rank_transform(I.T.copy(), 2), R.T)
    # a constant image has no darker neighbours anywhere
    assert not oracle.rank_transform(np.full((9, 9), 0.3), 2).any()


def _illum(I):
    return 1.25 * I + 0.03 + 0.1 * np.tanh(3.0 * I)


def _errors(d, data_term, lam, changed):
    rig, cfg = d["rig"], d["cfg"]
    I0 = d["I0"][0].astype(np.float64)
    I1 = d["I1"][0].astype(np.float64)
    if changed:
        I1 = _illum(I1)
    params = configs.solver_params(cfg, data_term=data_term, **{"lambda": lam})
    o = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, I0, I1)
    gt = d["gt"][0]
    keep = oracle.mask0(rig["cam0"]).astype(bool) & gt["visible"] & (o["valid"] > 0)
    e = np.linalg.norm(o["w"] - gt["flow"], axis=-1)[keep]
    return float(np.mean(e > 1.0)), float(np.median(e))


def test_rank_data_term_survives_an_illumination_change():
    d = inputs("c1")
    tau_b, epe_b = _errors(d, "brightness", 50.0, False)
    tau_bc, epe_bc = _errors(d, "brightness", 50.0, True)
    tau_r, epe_r = _errors(d, "rank", 2.0, False)
    tau_rc, epe_rc = _errors(d, "rank", 2.0, True)
    print("brightness", tau_b, epe_b, "changed", tau_bc, epe_bc, "| rank", tau_r, epe_r, "changed", tau_rc, epe_rc)
    assert tau_b < 0.01 and tau_bc > 0.5             # brightness constancy broken by the change
    assert tau_r < 0.01 and tau_rc < 0.01            # the rank term does not see it
    assert abs(epe_rc - epe_r) <= 0.05 * epe_r and epe_r < 0.1


def _gradient_by_definition(I):
    H, W = I.shape
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            gx = 0.5 * (I[i, min(j + 1, W - 1)] - I[i, max(j - 1, 0)])
            gy = 0.5 * (I[min(i + 1, H - 1), j] - I[max(i - 1, 0), j])
            out[i, j] = np.sqrt(gx * gx + gy * gy)
    return out


def test_gradient_magnitude_pins():
    """Against the definition in plain loops; a linear ramp gives its slope
    exactly inside the image; an added constant changes nothing; transposing
    the image transposes the result."""
    rng = np.random.default_rng(21)
    for shape in ((7, 9), (1, 5), (4, 1), (13, 6)):
        I = rng.random(shape)
        assert np.max(np.abs(oracle.gradient_magnitude(I) - _gradient_by_definition(I))) < 1e-15
    jj, ii = np.meshgrid(np.arange(20.0), np.arange(15.0))
    G = oracle.gradient_magnitude(0.03 * jj - 0.04 * ii + 0.2)
    assert np.max(np.abs(G[1:-1, 1:-1] - 0.05)) < 1e-15
    I = rng.random((30, 41))
    assert np.max(np.abs(oracle.gradient_magnitude(I + 0.25) - oracle.gradient_magnitude(I))) < 1e-15
    assert np.array_equal(oracle.gradient_magnitude(I.T.copy()), oracle.gradient_magnitude(I).T)


def test_gradient_data_term_survives_an_offset():
    """The whole method on the 128x128 plane with I1 + 0.15: the gradient data
    term recovers the rendered correspondences as without the offset; the
    brightness data term does not."""
    d = inputs("c1")
    rig, cfg = d["rig"], d["cfg"]
    I0 = d["I0"][0].astype(np.float64)
    I1 = d["I1"][0].astype(np.float64)
    gt = d["gt"][0]
    res = {}
    for term, lam in (("brightness", 50.0), ("gradient", 50.0)):
        for off in (0.0, 0.15):
            params = configs.solver_params(cfg, data_term=term, **{"lambda": lam})
            o = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, I0, I1 + off)
            keep = oracle.mask0(rig["cam0"]).astype(bool) & gt["visible"] & (o["valid"] > 0)
            e = np.linalg.norm(o["w"] - gt["flow"], axis=-1)[keep]
            res[(term, off)] = (float(np.mean(e > 1.0)), float(np.median(e)))
    print(res)
    assert res[("brightness", 0.15)][0] > 0.5
    assert res[("gradient", 0.0)][0] < 0.05 and res[("gradient", 0.15)][0] < 0.05
    # the offset changes the pyramid only by the same constant: nothing moves
    assert abs(res[("gradient", 0.15)][1] - res[("gradient", 0.0)][1]) < 1e-9
