"""Independent rectified 1-D TGV-L1 stereo solver (numpy, float64).

Test helper that pins the oracle's whole loop on the special case the method
reduces to: a pinhole camera pair translated along x, where the trajectory
field is (1, 0) everywhere, the epipolar curve is the image row and the search
is the conventional rectified one (Sec. III-B).  It is written vectorised,
from the textbook rectified formulation (straight warp x + u,
I_u = I1(x + u + 1) - I1(x + u)), and shares no code with the oracle.

Conventions (the same readings the method's implementation takes): 2x2 box
pyramid, nearest-neighbour masks, central-difference tensor one-sided at
mask / image borders, forward differences with the mask condition,
diagonal preconditioning, theta = 1, elementwise clip of the increment,
mask-aware bilinear x2 upsampling of u, v = p = q = 0 at every level.
"""
import numpy as np


def _box(J):
    return 0.25 * (J[0::2, 0::2] + J[0::2, 1::2] + J[1::2, 0::2] + J[1::2, 1::2])


def _inside(m):
    H, W = m.shape
    mx = np.zeros_like(m, dtype=bool)
    my = np.zeros_like(m, dtype=bool)
    mx[:, :-1] = m[:, :-1] & m[:, 1:]
    my[:-1, :] = m[:-1, :] & m[1:, :]
    return mx, my


def _grad(u, mx, my):
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gx[:, :-1] = u[:, 1:] - u[:, :-1]
    gy[:-1, :] = u[1:, :] - u[:-1, :]
    return gx * mx, gy * my


def _div(px, py, mx, my):
    ax, ay = px * mx, py * my
    d = ax + ay
    d[:, 1:] -= ax[:, :-1]
    d[1:, :] -= ay[:-1, :]
    return d


def _tensor(J, m, beta, eta):
    H, W = J.shape
    mb = m.astype(bool)
    left = np.zeros_like(mb)
    right = np.zeros_like(mb)
    up = np.zeros_like(mb)
    down = np.zeros_like(mb)
    left[:, 1:] = mb[:, :-1]
    right[:, :-1] = mb[:, 1:]
    up[1:, :] = mb[:-1, :]
    down[:-1, :] = mb[1:, :]
    Jl = np.zeros_like(J)
    Jr = np.zeros_like(J)
    Ju = np.zeros_like(J)
    Jd = np.zeros_like(J)
    Jl[:, 1:] = J[:, :-1]
    Jr[:, :-1] = J[:, 1:]
    Ju[1:, :] = J[:-1, :]
    Jd[:-1, :] = J[1:, :]
    gx = np.where(left & right, 0.5 * (Jr - Jl), np.where(right, Jr - J, np.where(left, J - Jl, 0.0)))
    gy = np.where(up & down, 0.5 * (Jd - Ju), np.where(down, Jd - J, np.where(up, J - Ju, 0.0)))
    g = np.hypot(gx, gy)
    ok = mb & (g >= 1e-12)
    gs = np.where(ok, g, 1.0)
    nx, ny = gx / gs, gy / gs
    e = np.exp(-beta * gs ** eta)
    t11 = np.where(ok, e * nx * nx + ny * ny, 1.0)
    t12 = np.where(ok, (e - 1.0) * nx * ny, 0.0)
    t22 = np.where(ok, e * ny * ny + nx * nx, 1.0)
    return t11, t12, t22


def _interp_row(J, x):
    """Linear interpolation of each row of J at abscissae x (clamp-to-edge)."""
    H, W = J.shape
    x0 = np.floor(x)
    a = x - x0
    i0 = np.clip(x0.astype(int), 0, W - 1)
    i1 = np.clip(x0.astype(int) + 1, 0, W - 1)
    rows = np.arange(H)[:, None]
    return (1 - a) * J[rows, i0] + a * J[rows, i1]


def _upsample(uc, mc):
    Hc, Wc = uc.shape
    Hf, Wf = 2 * Hc, 2 * Wc
    y = (np.arange(Hf) + 0.5) / 2 - 0.5
    x = (np.arange(Wf) + 0.5) / 2 - 0.5
    y0 = np.floor(y).astype(int)
    x0 = np.floor(x).astype(int)
    ay = (y - y0)[:, None]
    ax = (x - x0)[None, :]
    num = np.zeros((Hf, Wf))
    den = np.zeros((Hf, Wf))
    for dy, wy in ((0, 1 - ay), (1, ay)):
        yy = np.clip(y0 + dy, 0, Hc - 1)[:, None]
        for dx, wx in ((0, 1 - ax), (1, ax)):
            xx = np.clip(x0 + dx, 0, Wc - 1)[None, :]
            wgt = wy * wx * mc[yy, xx]
            num += wgt * uc[yy, xx]
            den += wgt
    return np.where(den > 0, 2 * num / np.where(den > 0, den, 1.0), 0.0)


def solve(I0, I1, mask0, levels, warps, iters, lam, alpha0, alpha1, beta, eta, du_max):
    I0 = np.asarray(I0, np.float64)
    I1 = np.asarray(I1, np.float64)
    J0, J1, M = [I0], [I1], [mask0.astype(bool)]
    for l in range(1, levels):
        J0.append(_box(J0[-1]))
        J1.append(_box(J1[-1]))
        o = 1 << (l - 1)
        M.append(mask0.astype(bool)[o::1 << l, o::1 << l])
    u = None
    for l in range(levels - 1, -1, -1):
        m = M[l]
        H, W = m.shape
        mx, my = _inside(m)
        t11, t12, t22 = _tensor(J0[l], m, beta, eta)
        mxl = np.zeros_like(mx)
        myu = np.zeros_like(my)
        mxl[:, 1:] = mx[:, :-1]
        myu[1:, :] = my[:-1, :]
        s1 = alpha1 * (np.abs(t11 * mx + t12 * my) + np.abs(t11) * mx + np.abs(t12) * my) + alpha1
        s2 = alpha1 * (np.abs(t12 * mx + t22 * my) + np.abs(t12) * mx + np.abs(t22) * my) + alpha1
        sig_p = 1.0 / np.maximum(s1, s2)
        sig_q = 1.0 / (2 * alpha0)
        cu = np.abs(t11 * mx + t12 * my) + np.abs(t12 * mx + t22 * my)
        cu[:, 1:] += ((np.abs(t11) + np.abs(t12)) * mx)[:, :-1]
        cu[1:, :] += ((np.abs(t12) + np.abs(t22)) * my)[:-1, :]
        tau_u = np.where(cu > 0, 1.0 / (alpha1 * np.where(cu > 0, cu, 1.0)), 1.0 / alpha1)
        cnt = mx.astype(np.float64) + my + mxl + myu
        tau_v = 1.0 / (alpha1 + alpha0 * cnt)
        u = np.zeros((H, W)) if u is None else _upsample(u, M[l + 1])
        v1, v2 = np.zeros((H, W)), np.zeros((H, W))
        p1, p2 = np.zeros((H, W)), np.zeros((H, W))
        q = [np.zeros((H, W)) for _ in range(4)]
        xs = np.arange(W, dtype=np.float64)[None, :]
        for _ in range(warps):
            u_w = u.copy()
            i1 = _interp_row(J1[l], xs + u)
            Iu = _interp_row(J1[l], xs + u + 1.0) - i1
            rho = i1 - J0[l] - u_w * Iu
            Iu = np.where(m, Iu, 0.0)
            rho = np.where(m, rho, 0.0)
            ub, vb1, vb2 = u.copy(), v1.copy(), v2.copy()
            for _ in range(iters):
                gx, gy = _grad(ub, mx, my)
                a1 = p1 + sig_p * alpha1 * (t11 * gx + t12 * gy - vb1)
                a2 = p2 + sig_p * alpha1 * (t12 * gx + t22 * gy - vb2)
                n = np.maximum(1.0, np.hypot(a1, a2))
                p1 = np.where(m, a1 / n, 0.0)
                p2 = np.where(m, a2 / n, 0.0)
                d11, d12 = _grad(vb1, mx, my)
                d21, d22 = _grad(vb2, mx, my)
                qq = [q[0] + sig_q * alpha0 * d11, q[1] + sig_q * alpha0 * d12,
                      q[2] + sig_q * alpha0 * d21, q[3] + sig_q * alpha0 * d22]
                n = np.maximum(1.0, np.sqrt(sum(c * c for c in qq)))
                q = [np.where(m, c / n, 0.0) for c in qq]
                tp1 = t11 * p1 + t12 * p2
                tp2 = t12 * p1 + t22 * p2
                uhat = u + tau_u * alpha1 * _div(tp1, tp2, mx, my)
                rb = rho + uhat * Iu
                a = tau_u * lam * Iu
                un = np.where(rb < -a * Iu, uhat + a,
                              np.where(rb > a * Iu, uhat - a,
                                       np.where(Iu != 0, uhat - rb / np.where(Iu != 0, Iu, 1.0), uhat)))
                un = np.where(m, un, u)
                vn1 = np.where(m, v1 + tau_v * (alpha1 * p1 + alpha0 * _div(q[0], q[1], mx, my)), v1)
                vn2 = np.where(m, v2 + tau_v * (alpha1 * p2 + alpha0 * _div(q[2], q[3], mx, my)), v2)
                ub = 2 * un - u
                vb1 = 2 * vn1 - v1
                vb2 = 2 * vn2 - v2
                u, v1, v2 = un, vn1, vn2
            u = u_w + np.clip(u - u_w, -du_max, du_max)
    return u
