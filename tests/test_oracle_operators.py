"""Pins of the oracle's operators: masked grad / div (Sec. IV-B boundary
conditions), projections and resolvent (Eqs. (11), (13)), tensor (Eq. (12)),
preconditioned step sizes (Sec. III-D).

Checks are against definitions written out independently here (sparse
matrices built entry by entry, brute-force minimisation, eigen-decomposition).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle


def _random_mask(rng, H, W, p=0.85):
    return (rng.random((H, W)) < p).astype(np.uint8)


def _grad_matrix(mask):
    """Sparse forward-difference gradient with the mask condition, written
    from its definition: component x of pixel P is u(P+x) - u(P) if P and P+x
    are both inside the image and the mask, else 0 (likewise y)."""
    H, W = mask.shape
    rows, cols, vals = [], [], []
    for i in range(H):
        for j in range(W):
            P = i * W + j
            if mask[i, j] and j + 1 < W and mask[i, j + 1]:
                rows += [2 * P, 2 * P]
                cols += [P + 1, P]
                vals += [1.0, -1.0]
            if mask[i, j] and i + 1 < H and mask[i + 1, j]:
                rows += [2 * P + 1, 2 * P + 1]
                cols += [P + W, P]
                vals += [1.0, -1.0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * H * W, H * W))


@pytest.mark.parametrize("seed", range(3))
def test_grad_div_adjoint(seed):
    rng = np.random.default_rng(seed)
    H, W = 23, 31
    m = _random_mask(rng, H, W)
    u = rng.normal(size=(H, W))
    p = rng.normal(size=(H, W, 2))
    g = oracle.grad(u, m)
    d = oracle.div(p, m)
    lhs = np.sum(g * p)
    rhs = -np.sum(u * d)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)
    # and grad is exactly the matrix of the definition
    G = _grad_matrix(m)
    assert np.array_equal(g.reshape(-1), G @ u.reshape(-1))


def test_projections():
    rng = np.random.default_rng(7)
    for n in (2, 4):
        phi = rng.normal(size=(5000, n)) * rng.uniform(0.01, 3.0, (5000, 1))
        P = oracle.project_balls(phi, n).reshape(-1, n)
        nrm = np.linalg.norm(phi, axis=1)
        assert np.all(np.linalg.norm(P, axis=1) <= 1 + 1e-15)
        inside = nrm <= 1
        assert np.array_equal(P[inside], phi[inside])
        assert np.allclose(P[~inside], phi[~inside] / nrm[~inside, None], rtol=0, atol=1e-15)
        assert np.max(np.abs(oracle.project_balls(P, n).reshape(-1, n) - P)) <= 4e-16


def test_threshold_is_the_prox_of_the_linearised_l1_term():
    """Eq. (13) (third case read with the sign that zeroes rho_bar) equals the
    argmin of (u - uhat)^2 / (2 tau) + lambda |rho_c + u I_u|, found by a
    dense 1-D search refined by golden-section search."""
    rng = np.random.default_rng(8)
    n = 20000
    uhat = rng.normal(0, 2, n)
    rho = rng.normal(0, 0.2, n)
    Iu = rng.normal(0, 0.1, n)
    Iu[:500] = 0.0                                   # no data
    tau = rng.uniform(0.01, 1.0, n)
    lam = 50.0
    # cases on the tie boundaries |rho_bar| = tau lam Iu^2
    k = slice(500, 1000)
    s = np.where(rng.random(500) < 0.5, -1.0, 1.0)
    rho[k] = s * tau[k] * lam * Iu[k] ** 2 - uhat[k] * Iu[k]
    out = oracle.threshold(uhat, rho, Iu, tau, lam)

    def f(u):
        return (u - uhat[:, None]) ** 2 / (2 * tau[:, None]) + lam * np.abs(rho[:, None] + u * Iu[:, None])

    span = 2 * tau * lam * np.abs(Iu) + 1e-3
    grid = uhat[:, None] + span[:, None] * np.linspace(-1.5, 1.5, 3001)[None, :]
    best = grid[np.arange(n), np.argmin(f(grid), axis=1)]
    a = best - 3 * span / 3000
    b = best + 3 * span / 3000
    g = (np.sqrt(5) - 1) / 2
    for _ in range(120):
        c = b - g * (b - a)
        d = a + g * (b - a)
        left = f(c[:, None])[:, 0] < f(d[:, None])[:, 0]
        b = np.where(left, d, b)
        a = np.where(left, a, c)
    brute = 0.5 * (a + b)
    fo = f(out[:, None])[:, 0]
    fb = f(brute[:, None])[:, 0]
    assert np.all(fo <= fb + 1e-10 * (1 + np.abs(fb)))
    assert np.max(np.abs(out - brute) / (1 + np.abs(brute))) < 1e-6
    assert np.array_equal(out[:500], uhat[:500])


def test_tensor_eigen_structure():
    rng = np.random.default_rng(9)
    H, W = 40, 48
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    J = 0.5 + 0.2 * np.sin(0.3 * jj + 0.1 * ii) + 0.1 * np.cos(0.17 * ii - 0.05 * jj * jj / W)
    m = np.ones((H, W), np.uint8)
    beta, eta = 9.0, 0.85
    T = oracle.tensor(J, m, beta, eta)
    # interior gradient by central differences, written out here
    gx = 0.5 * (J[1:-1, 2:] - J[1:-1, :-2])
    gy = 0.5 * (J[2:, 1:-1] - J[:-2, 1:-1])
    Ti = T[1:-1, 1:-1]
    for t, x, y in zip(Ti.reshape(-1, 3), gx.reshape(-1), gy.reshape(-1)):
        M = np.array([[t[0], t[1]], [t[1], t[2]]])
        g = np.hypot(x, y)
        e = np.exp(-beta * g ** eta)
        n = np.array([x, y]) / g
        assert np.allclose(M @ n, e * n, atol=1e-14)
        nperp = np.array([-n[1], n[0]])
        assert np.allclose(M @ nperp, nperp, atol=1e-14)
    # constant image and masked-out pixels: identity
    Tc = oracle.tensor(np.full((H, W), 0.3), m, beta, eta)
    assert np.array_equal(Tc, np.broadcast_to([1.0, 0.0, 1.0], Tc.shape))
    m2 = _random_mask(rng, H, W, 0.5)
    T2 = oracle.tensor(J, m2, beta, eta)
    assert np.array_equal(T2[m2 == 0], np.broadcast_to([1.0, 0.0, 1.0], T2[m2 == 0].shape))


def test_tensor_one_sided_at_mask_border():
    J = np.arange(5 * 6, dtype=np.float64).reshape(5, 6) ** 1.5 / 10
    m = np.ones((5, 6), np.uint8)
    m[:, 4:] = 0
    T = oracle.tensor(J, m, 2.0, 1.0)
    i, j = 2, 3            # right neighbour is masked: backward difference in x
    gx = J[i, j] - J[i, j - 1]
    gy = 0.5 * (J[i + 1, j] - J[i - 1, j])
    g = np.hypot(gx, gy)
    M = np.array([[T[i, j, 0], T[i, j, 1]], [T[i, j, 1], T[i, j, 2]]])
    n = np.array([gx, gy]) / g
    assert np.allclose(M @ n, np.exp(-2.0 * g) * n, atol=1e-14)


@pytest.mark.parametrize("reg", ["tgv", "tv"])
def test_steps_are_reciprocal_abs_sums_of_K(reg):
    """Diagonal preconditioning with alpha = 1: sigma = 1 / (row abs-sum),
    tau = 1 / (column abs-sum) of K = [[a1 T grad, -a1 I], [0, a0 grad]]
    assembled explicitly (TV: K = [a1 T grad])."""
    rng = np.random.default_rng(10)
    H, W = 12, 12
    m = _random_mask(rng, H, W, 0.8)
    J = rng.random((H, W))
    T = oracle.tensor(J, m, 9.0, 0.85)
    a0, a1 = 17.0, 1.2
    n = H * W
    G = _grad_matrix(m).tocsr()
    Gx, Gy = G[0::2], G[1::2]
    t11 = sp.diags(T[..., 0].reshape(-1))
    t12 = sp.diags(T[..., 1].reshape(-1))
    t22 = sp.diags(T[..., 2].reshape(-1))
    TG = sp.vstack([t11 @ Gx + t12 @ Gy, t12 @ Gx + t22 @ Gy])          # rows p1, p2
    if reg == "tgv":
        I = sp.identity(n)
        K = sp.bmat([[a1 * TG[:n], -a1 * I, None],
                     [a1 * TG[n:], None, -a1 * I],
                     [None, a0 * Gx, None], [None, a0 * Gy, None],
                     [None, None, a0 * Gx], [None, None, a0 * Gy]]).tocsr()
    else:
        K = (a1 * TG).tocsr()
    A = abs(K)
    row = np.asarray(A.sum(axis=1)).reshape(-1)
    col = np.asarray(A.sum(axis=0)).reshape(-1)
    sp_, tu, tv = oracle.steps(T, m, a0, a1, reg)
    rp = np.maximum(row[:n], row[n:2 * n])
    ok = rp > 0
    assert np.allclose(sp_.reshape(-1)[ok], 1.0 / rp[ok], rtol=1e-14, atol=0)
    cu = col[:n]
    ok = cu > 0
    assert np.allclose(tu.reshape(-1)[ok], 1.0 / cu[ok], rtol=1e-14, atol=0)
    if reg == "tgv":
        assert np.allclose(tv.reshape(-1), 1.0 / col[n:2 * n], rtol=1e-14, atol=0)
        assert np.allclose(tv.reshape(-1), 1.0 / col[2 * n:], rtol=1e-14, atol=0)
        # every q row has abs-sum 2 a0 or 0: sigma_q = 1/(2 a0) is the smallest safe value
        assert np.max(row[2 * n:]) == 2 * a0


@pytest.mark.parametrize("reg", ["tgv", "tv"])
@pytest.mark.parametrize("seed", range(3))
def test_energy_is_eq10_written_with_explicit_operators(reg, seed):
    """The linearised energy of Eq. (10) written out here with the sparse
    gradient of the definition (entry by entry, not through the oracle):
    E = sum over the mask of lambda |rho_c + u I_u| + alpha1 |(T grad u - v)_P|_2
        + alpha0 |(grad v)_P|_F      (TV: v = 0, no last term),
    on random masked states with v, I_u and rho_c non-zero everywhere, so a
    dropped term, a sign, a swapped tensor entry or a missed mask changes the
    value."""
    rng = np.random.default_rng(20 + seed)
    H, W = 17, 13
    m = _random_mask(rng, H, W, 0.75)
    n = H * W
    J = rng.random((H, W))
    T = oracle.tensor(J, m, 9.0, 0.85)
    # perturb the tensor off its structured form so t11, t12, t22 are all
    # distinct and a swapped entry shows
    T = T + 0.1 * rng.normal(size=T.shape)
    u = rng.normal(size=(H, W))
    v = rng.normal(size=(H, W, 2)) if reg == "tgv" else None
    Iu = rng.normal(0, 0.3, (H, W))
    rho = rng.normal(0, 0.3, (H, W))
    params = dict(levels=1, warps=1, iters=1, reg=reg, alpha0=17.0, alpha1=1.2, beta=9.0, eta=0.85,
                  du_max=0.2, **{"lambda": 50.0})
    G = _grad_matrix(m).tocsr()
    Gx, Gy = G[0::2], G[1::2]
    ux, uy = Gx @ u.reshape(-1), Gy @ u.reshape(-1)
    t11, t12, t22 = (T[..., k].reshape(-1) for k in range(3))
    a1 = t11 * ux + t12 * uy
    a2 = t12 * ux + t22 * uy
    if reg == "tgv":
        a1 = a1 - v[..., 0].reshape(-1)
        a2 = a2 - v[..., 1].reshape(-1)
    inside = m.reshape(-1).astype(bool)
    E = np.sum((50.0 * np.abs(rho.reshape(-1) + u.reshape(-1) * Iu.reshape(-1)))[inside])
    E += np.sum((1.2 * np.hypot(a1, a2))[inside])
    if reg == "tgv":
        comps = [Gx @ v[..., 0].reshape(-1), Gy @ v[..., 0].reshape(-1),
                 Gx @ v[..., 1].reshape(-1), Gy @ v[..., 1].reshape(-1)]
        E += np.sum((17.0 * np.sqrt(sum(c * c for c in comps)))[inside])
    Eo = oracle.energy(params, T, m, Iu, rho, u, v)
    assert abs(Eo - E) <= 1e-12 * abs(E)
    # each term is large enough on these states that dropping it would show
    assert np.sum((1.2 * np.hypot(a1, a2))[inside]) > 1e-3 * E
    if reg == "tgv":
        assert np.sum((17.0 * np.sqrt(sum(c * c for c in comps)))[inside]) > 1e-3 * E


def test_upsample_closed_forms():
    """The x2 transfer of (u, w) between pyramid levels (Sec. IV-B; the
    coarse pixel j covers fine pixels 2j and 2j + 1 of the box pyramid, so
    its centre sits at fine coordinate 2j + 1/2), pinned by closed forms:
    (a) a linear ramp on a full mask comes back as twice the ramp sampled at
    the fine pixel's centre, x = (j_f + 1/2) / 2 - 1/2, wherever both coarse
    neighbours exist; (b) the box-filtered fine ramp comes back as twice the
    fine ramp; (c) only coarse pixels inside the mask contribute, with their
    bilinear weights renormalised: a constant inside the mask comes back as
    twice the constant wherever any of the four neighbours is inside, values
    outside the mask never leak, and a fine pixel with no neighbour inside
    gets 0."""
    rng = np.random.default_rng(21)
    Hc, Wc = 7, 9
    ic, jc = np.mgrid[0:Hc, 0:Wc].astype(np.float64)
    a, b, c = 0.37, -1.21, 2.5
    u = a * jc + b * ic + c
    w = np.stack([-0.8 * jc + 0.3 * ic, 0.45 * jc + 1.7 * ic - 4.0], -1)
    full = np.ones((Hc, Wc), np.uint8)
    uf, wf = oracle.upsample(full, u, w)
    assert uf.shape == (2 * Hc, 2 * Wc) and wf.shape == (2 * Hc, 2 * Wc, 2)
    i_f, j_f = np.mgrid[0:2 * Hc, 0:2 * Wc].astype(np.float64)
    x, y = (j_f + 0.5) / 2 - 0.5, (i_f + 0.5) / 2 - 0.5
    inner = (x >= 0) & (x <= Wc - 1) & (y >= 0) & (y <= Hc - 1)
    assert np.abs(uf - 2 * (a * x + b * y + c))[inner].max() < 1e-12
    assert np.abs(wf[..., 0] - 2 * (-0.8 * x + 0.3 * y))[inner].max() < 1e-12
    assert np.abs(wf[..., 1] - 2 * (0.45 * x + 1.7 * y - 4.0))[inner].max() < 1e-12
    # (b) down then up: the fine ramp, doubled, away from the clamped border
    ramp = a * j_f + b * i_f + c
    back, _ = oracle.upsample(full, oracle.downsample(ramp), np.zeros((Hc, Wc, 2)))
    assert np.abs(back - 2 * ramp)[1:-1, 1:-1].max() < 1e-12
    # (c) mask-awareness
    mask = (rng.random((Hc, Wc)) < 0.6).astype(np.uint8)
    mask[3, 4] = 0
    mask[2, 2] = 1
    uc = np.where(mask == 1, 3.0, 1e6)
    wc = np.where(mask[..., None] == 1, np.array([-1.5, 0.25]), 1e6)
    uf, wf = oracle.upsample(mask, uc, wc)
    for i in range(2 * Hc):
        for j in range(2 * Wc):
            x0, y0 = int(np.floor((j + 0.5) / 2 - 0.5)), int(np.floor((i + 0.5) / 2 - 0.5))
            nb = [(min(max(yy, 0), Hc - 1), min(max(xx, 0), Wc - 1)) for yy in (y0, y0 + 1) for xx in (x0, x0 + 1)]
            x, y = (j + 0.5) / 2 - 0.5, (i + 0.5) / 2 - 0.5
            wts = [(1 - abs(x - xx)) * (1 - abs(y - yy)) for yy in (y0, y0 + 1) for xx in (x0, x0 + 1)]
            inside = any(mask[p] and wt > 0 for p, wt in zip(nb, wts))
            if inside:
                assert abs(uf[i, j] - 6.0) < 1e-12 and np.abs(wf[i, j] - [-3.0, 0.5]).max() < 1e-12, (i, j)
            else:
                assert uf[i, j] == 0.0 and not wf[i, j].any(), (i, j)


def test_downsample_closed_forms():
    """The box pyramid (Sec. IV-B: 2x2 averages, scale 1/2), pinned by closed
    forms: a linear ramp comes back as the ramp at the coarse pixel's centre
    (fine coordinate 2j + 1/2), a +-1 checkerboard vanishes, the total is a
    quarter of the fine one, and an odd last row / column is dropped."""
    H, W = 9, 12
    i, j = np.mgrid[0:H, 0:W].astype(np.float64)
    a, b, c = 0.61, -0.29, 1.75
    d = oracle.downsample(a * j + b * i + c)
    assert d.shape == (H // 2, W // 2)
    ic, jc = np.mgrid[0:H // 2, 0:W // 2].astype(np.float64)
    assert np.abs(d - (a * (2 * jc + 0.5) + b * (2 * ic + 0.5) + c)).max() < 1e-12
    checker = np.where((i + j) % 2 == 0, 1.0, -1.0)
    assert np.abs(oracle.downsample(checker)).max() == 0.0
    rng = np.random.default_rng(3)
    x = rng.normal(size=(H, W))
    assert abs(oracle.downsample(x).sum() * 4 - x[:H - 1, :].sum()) < 1e-10
