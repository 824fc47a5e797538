"""FP64 CPU oracle of the non-rectified variational fisheye stereo method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it.  It is a ctypes wrapper over ``vfs_oracle.c`` (plain C, double
precision) and shares no code with the GPU library.

Every function takes and returns numpy float64 / uint8 arrays in row-major
H x W layout with interleaved vector components (see the C file's header).

What pins each function (each check is against something other than the
oracle itself; the tests named live in ``tests/``):

* ``project`` / ``unproject`` -- round trip pi(pi^-1(x)) = x, equidistant
  closed form theta = r/f, Kannala-Brandt with k = 0 equals equidistant,
  pinhole closed form (test_oracle_geometry).  Unified and enhanced unified
  models: xi = 0 / alpha = 0 equal the pinhole, the enhanced model with
  beta = 1 equals the unified one with xi = alpha / (1 - alpha), the radial
  projection and the closed-form inverse round-trip, agreement with the
  renderer's Newton-inverted camera, angle limits acos(-1/xi) / acos(-xi),
  tangency to the brute-force epipolar curve (test_oracle_unified).
* ``trajectory_field`` -- tangency to the brute-force epipolar curve traced by
  projecting points at 400 depths along back-projected rays; exact (+1, 0)
  for a pinhole with x-translation; radial field for z-translation;
  independence of |t| and of the surface depth; analytic Jacobian direction;
  the epipole flag set is exactly the 2-degree cone around +-t by the
  equidistant closed form, with zero tangents there and unit ones elsewhere
  (test_oracle_geometry).
* ``mask0`` -- the pixels whose normalised radius is at most the radial map
  at half the field of view, by each model's closed form (test_oracle_geometry);
  ``level_mask`` -- nearest-neighbour sampling at 2^l i + 2^(l-1) (same file).
* ``calibration_field`` / ``prerotate`` -- zero field for R = I and equal
  cameras; a scene rendered by a rotated camera and pre-rotated matches the
  unrotated render (test_oracle_geometry).
* ``grad`` / ``div`` -- adjointness <grad u, p> = -<u, div p> on random masks
  (test_oracle_operators).
* ``steps`` -- reciprocal row / column abs-sums of an explicitly assembled
  sparse K (test_oracle_operators).
* ``threshold`` -- dense 1-D argmin of the prox objective (test_oracle_operators).
* ``tensor`` -- eigen-structure {exp(-beta |g|^eta), 1} with eigenvector n,
  identity on constant images (test_oracle_operators).
* ``energy`` -- equals Eq. (10) linearised, written out in the test with
  the sparse gradient of its definition and the tensor entries applied by
  hand, on random masked states with every term non-zero, TGV and TV
  (test_oracle_operators).
* ``pd_iterations`` -- converged iterates satisfy the optimality conditions
  of the linearised energy (subdifferential of Eq. (10), written from the
  energy, not from the iteration); energy decreases over each inner loop
  (test_oracle_solver).
* ``linearise`` -- the warped tangent is unit length and radial away from
  the epipole of a radial field, goes to zero approaching it and is
  Lipschitz across it; on linear images with a constant tangent (where
  every sample is exact) I_u and rho_c equal their closed forms, and both
  are 0 where the data term is off (test_oracle_solver).
* ``rectify_rotations`` / ``rectify`` / ``unrectify`` -- the two virtual
  cameras differ by a pure x-translation for random rigs; rectified renders
  match the renderer's own pinhole renders of the same scene from both
  camera centres, and plausible wrong rotations do not; the round trip
  returns a smooth image; a pinhole camera is its own view
  (test_oracle_rectify).
* ``gradient_magnitude`` -- equals its definition in plain loops; exact
  slope on a linear ramp; invariant under an added constant; transposition
  (test_oracle_rank).
* ``rank_transform`` -- equals its definition written out in plain loops,
  ties included; invariant under strictly increasing intensity maps and
  transposition (test_oracle_rank).
* ``solve`` -- pinhole camera with x-translation equals an independently
  written rectified 1-D TGV-L1 solver; recovered depth of a rendered plane
  and room matches the renderer's ground truth (test_oracle_solver).  With
  the rank data term on the plane: unaffected by a tone-curve change of I1
  that breaks brightness constancy (test_oracle_rank).
* ``clip_accumulate`` -- hand-computed increments above, below, inside and at
  the edge of the 0.2 px clip; with no clip, one warp's w is u times the
  tangent (test_oracle_solver).
* ``triangulate`` -- ground-truth correspondences recover the renderer's
  range; pinhole rectified case gives Z = f b / disparity (test_oracle_geometry).
* ``downsample`` -- a linear ramp returns as the ramp at the coarse pixel
  centres, a +-1 checkerboard vanishes, the total is a quarter of the fine
  one, an odd last row / column is dropped (test_oracle_operators).
* ``upsample`` -- a linear ramp on a full mask returns as twice the ramp at
  the fine pixel centres; down- then up-sampling a fine ramp returns it
  doubled; constants inside a random mask return doubled, values outside it
  never leak, pixels without an in-mask neighbour get 0 (test_oracle_operators).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vfs_oracle.c")
_ABI = os.path.join(_HERE, "vfso.c")      # the library's calls over the oracle (host pointers)
_LIB = os.path.join(_HERE, "liboracle.so")

MODELS = {"pinhole": 0, "equidistant": 1, "kb": 2, "kannala_brandt": 2, "unified": 3, "ucm": 3,
          "eucm": 4, "enhanced_unified": 4}
REGS = {"tgv": 0, "tv": 1}
DATA_TERMS = {"brightness": 0, "rank": 1, "gradient": 2}


class _Camera(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("width", ctypes.c_int), ("height", ctypes.c_int),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("k", ctypes.c_double * 4), ("fov_deg", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("warps", ctypes.c_int), ("iters", ctypes.c_int),
                ("reg", ctypes.c_int), ("lam", ctypes.c_double), ("alpha0", ctypes.c_double),
                ("alpha1", ctypes.c_double), ("beta", ctypes.c_double), ("eta", ctypes.c_double),
                ("du_max", ctypes.c_double), ("theta_gamma", ctypes.c_double), ("data_term", ctypes.c_int)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (C11, strict IEEE double, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                         os.path.getmtime(_ABI)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, _ABI, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_theta_limit.restype = ctypes.c_double
        _lib.or_energy.restype = ctypes.c_double
        _lib.or_threshold.restype = ctypes.c_double
        _lib.or_threshold.argtypes = [ctypes.c_double] * 5
    return _lib


def _cam(c: dict) -> _Camera:
    k = list(c.get("k", (0.0, 0.0, 0.0, 0.0)))
    m = c["model"]
    return _Camera(MODELS[m] if isinstance(m, str) else int(m), int(c["width"]), int(c["height"]),
                   float(c["fx"]), float(c["fy"]), float(c["cx"]), float(c["cy"]),
                   (ctypes.c_double * 4)(*k), float(c["fov_deg"]))


def _par(p: dict) -> _Params:
    reg = p.get("reg", "tgv")
    return _Params(int(p["levels"]), int(p["warps"]), int(p["iters"]),
                   REGS[reg] if isinstance(reg, str) else int(reg), float(p["lambda"]),
                   float(p["alpha0"]), float(p["alpha1"]), float(p["beta"]), float(p["eta"]),
                   float(p["du_max"]), float(p.get("theta_gamma", 0.0)),
                   DATA_TERMS[p.get("data_term", 0)] if isinstance(p.get("data_term", 0), str)
                   else int(p.get("data_term", 0)))


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _R(R):
    return _d(np.asarray(R, dtype=np.float64).reshape(9))


def _t(t):
    return _d(np.asarray(t, dtype=np.float64).reshape(3))


# ---------------------------------------------------------------- cameras

def theta_limit(cam: dict) -> float:
    c = _cam(cam)
    return lib().or_theta_limit(ctypes.byref(c))


def camera_check(cam: dict) -> int:
    c = _cam(cam)
    return lib().or_camera_check(ctypes.byref(c))


def project(cam: dict, X):
    X = _d(np.asarray(X).reshape(-1, 3))
    n = X.shape[0]
    x = np.zeros((n, 2))
    ok = np.zeros(n, np.uint8)
    c = _cam(cam)
    lib().or_project_points(ctypes.byref(c), n, _p(X), _p(x), _p(ok))
    return x, ok.astype(bool)


def unproject(cam: dict, x):
    x = _d(np.asarray(x).reshape(-1, 2))
    n = x.shape[0]
    r = np.zeros((n, 3))
    c = _cam(cam)
    lib().or_unproject_points(ctypes.byref(c), n, _p(x), _p(r))
    return r


# ---------------------------------------------------------------- rig fields

def mask0(cam: dict):
    m = np.zeros((cam["height"], cam["width"]), np.uint8)
    c = _cam(cam)
    lib().or_mask0(ctypes.byref(c), _p(m))
    return m


def level_mask(m0, level: int):
    m0 = _u8(m0)
    H, W = m0.shape
    out = np.zeros((H >> level, W >> level), np.uint8)
    lib().or_level_mask(_p(m0), W, H, level, _p(out))
    return out


def calibration_field(cam0: dict, cam1: dict, R):
    H, W = cam0["height"], cam0["width"]
    cf = np.zeros((H, W, 2))
    valid = np.zeros((H, W), np.uint8)
    c0, c1, Rr = _cam(cam0), _cam(cam1), _R(R)
    lib().or_calibration_field(ctypes.byref(c0), ctypes.byref(c1), _p(Rr), _p(cf), _p(valid))
    return cf, valid


def prerotate(I1, cf):
    I1 = _d(I1)
    cf = _d(cf)
    H, W = I1.shape
    out = np.zeros_like(I1)
    lib().or_prerotate(_p(I1), W, H, _p(cf), _p(out))
    return out


def rectify_rotations(R, t):
    """(Rv0, Rv1, baseline): shared virtual orientation of a rig (see the C file)."""
    R = np.ascontiguousarray(R, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    a, b = np.zeros(9), np.zeros(9)
    base = ctypes.c_double()
    st = lib().or_rectify_rotations(_p(R), _p(t), _p(a), _p(b), ctypes.byref(base))
    if st != 0:
        raise ValueError(f"rectify_rotations: status {st}")
    return a.reshape(3, 3), b.reshape(3, 3), base.value


def rectify(cam: dict, Rv, pinhole: dict, src):
    """(image, valid) of the pinhole view of a camera image."""
    src = _d(src)
    Rv = np.ascontiguousarray(Rv, np.float64)
    out = np.zeros((pinhole["height"], pinhole["width"]))
    valid = np.zeros(out.shape, np.uint8)
    c, pn = _cam(cam), _cam(pinhole)
    lib().or_rectify(ctypes.byref(c), _p(Rv), ctypes.byref(pn), _p(src), _p(out), _p(valid))
    return out, valid


def unrectify(cam: dict, Rv, pinhole: dict, field, field_valid=None):
    """(values, valid) of a pinhole-view field at the camera's pixels."""
    field = _d(field)
    Rv = np.ascontiguousarray(Rv, np.float64)
    out = np.zeros((cam["height"], cam["width"]))
    valid = np.zeros(out.shape, np.uint8)
    fv = None if field_valid is None else _u8(field_valid)
    c, pn = _cam(cam), _cam(pinhole)
    lib().or_unrectify(ctypes.byref(c), _p(Rv), ctypes.byref(pn), _p(field), None if fv is None else _p(fv),
                       _p(out), _p(valid))
    return out, valid


def trajectory_field(cam0: dict, R, t, level: int):
    H, W = cam0["height"] >> level, cam0["width"] >> level
    g = np.zeros((H, W, 2))
    epi = np.zeros((H, W), np.uint8)
    c0, Rr, tt = _cam(cam0), _R(R), _t(t)
    st = lib().or_trajectory_field(ctypes.byref(c0), _p(Rr), _p(tt), level, _p(g), _p(epi))
    if st != 0:
        raise ValueError(f"trajectory field: status {st}")
    return g, epi


def trajectory_at(cam0: dict, R, t, pts):
    """gamma'(x) and the epipole flag at arbitrary level-0 points."""
    pts = _d(np.asarray(pts).reshape(-1, 2))
    n = pts.shape[0]
    g = np.zeros((n, 2))
    epi = np.zeros(n, np.uint8)
    c0, Rr, tt = _cam(cam0), _R(R), _t(t)
    st = lib().or_trajectory_at(ctypes.byref(c0), _p(Rr), _p(tt), n, _p(pts), _p(g), _p(epi))
    if st != 0:
        raise ValueError(f"trajectory: status {st}")
    return g, epi.astype(bool)


def sample_trajectory(gamma, pts):
    gamma = _d(gamma)
    H, W = gamma.shape[:2]
    pts = _d(np.asarray(pts).reshape(-1, 2))
    out = np.zeros_like(pts)
    lib().or_sample_trajectory(_p(gamma), W, H, pts.shape[0], _p(pts), _p(out))
    return out


# ---------------------------------------------------------------- per-level steps

def downsample(J):
    J = _d(J)
    H, W = J.shape
    out = np.zeros((H // 2, W // 2))
    lib().or_downsample(_p(J), W, H, _p(out))
    return out


def tensor(J0, mask, beta: float, eta: float):
    J0, mask = _d(J0), _u8(mask)
    H, W = J0.shape
    T = np.zeros((H, W, 3))
    lib().or_tensor(_p(J0), _p(mask), W, H, ctypes.c_double(beta), ctypes.c_double(eta), _p(T))
    return T


def grad(u, mask):
    u, mask = _d(u), _u8(mask)
    H, W = u.shape
    g = np.zeros((H, W, 2))
    lib().or_grad(_p(u), _p(mask), W, H, _p(g))
    return g


def div(p, mask):
    p, mask = _d(p), _u8(mask)
    H, W = mask.shape
    d = np.zeros((H, W))
    lib().or_div(_p(p), _p(mask), W, H, _p(d))
    return d


def steps(T, mask, alpha0: float, alpha1: float, reg="tgv"):
    T, mask = _d(T), _u8(mask)
    H, W = mask.shape
    sp, tu, tv = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W))
    lib().or_steps(_p(T), _p(mask), W, H, ctypes.c_double(alpha0), ctypes.c_double(alpha1),
                   REGS[reg] if isinstance(reg, str) else int(reg), _p(sp), _p(tu), _p(tv))
    return sp, tu, tv


def rank_transform(I, radius: int = 2):
    """Share of the (2r+1)^2 - 1 neighbours strictly darker than each pixel
    (edge-clamped neighbourhood): the data term's image for data_term
    "rank"."""
    I = _d(I)
    H, W = I.shape
    out = np.zeros((H, W))
    lib().or_rank_transform(_p(I), W, H, int(radius), _p(out))
    return out


def gradient_magnitude(I):
    """sqrt(Ix^2 + Iy^2) with edge-clamped central differences: the data
    term's image for data_term "gradient"."""
    I = _d(I)
    H, W = I.shape
    out = np.zeros((H, W))
    lib().or_gradient_magnitude(_p(I), W, H, _p(out))
    return out


def project_balls(phi, n: int):
    phi = _d(phi).copy()
    lib().or_project_balls(_p(phi), phi.size // n, n)
    return phi


def threshold(uhat, rho_c, Iu, tau, lam: float):
    uhat, rho_c, Iu, tau = (_d(np.broadcast_to(a, np.shape(uhat))) for a in (uhat, rho_c, Iu, tau))
    out = np.zeros_like(uhat)
    lib().or_threshold_many(uhat.size, _p(uhat), _p(rho_c), _p(Iu), _p(tau), ctypes.c_double(lam), _p(out))
    return out


def energy(params: dict, T, mask, Iu, rho, u, v):
    T, mask, Iu, rho, u = _d(T), _u8(mask), _d(Iu), _d(rho), _d(u)
    v = _d(v) if v is not None else None
    H, W = mask.shape
    pp = _par(params)
    return lib().or_energy(W, H, ctypes.byref(pp), _p(T), _p(mask), _p(Iu), _p(rho), _p(u), _p(v))


def pd_iterations(params: dict, T, mask, sig_p, tau_u, tau_v, Iu, rho, u, v, p, q, K: int,
                  ubar=None, vbar=None, trace: bool = False):
    """K iterations of Eq. (11) from the given state; returns the new state
    (u, ubar, v, vbar, p, q) and, with trace=True, the K+1 energies."""
    T, mask = _d(T), _u8(mask)
    H, W = mask.shape
    tgv = params.get("reg", "tgv") in ("tgv", 0)
    u = _d(u).copy()
    ubar = _d(ubar).copy() if ubar is not None else u.copy()
    p = _d(p).copy()
    if tgv:
        v = _d(v).copy()
        vbar = _d(vbar).copy() if vbar is not None else v.copy()
        q = _d(q).copy()
    else:
        v = vbar = q = None
    en = np.zeros(K + 1) if trace else None
    pp = _par(params)
    lib().or_pd_iterations(W, H, ctypes.byref(pp), _p(T), _p(mask), _p(_d(sig_p)), _p(_d(tau_u)),
                           _p(_d(tau_v)), _p(_d(Iu)), _p(_d(rho)), _p(u), _p(ubar), _p(v), _p(vbar),
                           _p(p), _p(q), int(K), _p(en))
    out = dict(u=u, ubar=ubar, v=v, vbar=vbar, p=p, q=q)
    if trace:
        out["energy"] = en
    return out


def linearise(J0, J1, gamma, dvalid, u, w):
    J0, J1, gamma, dvalid, u, w = _d(J0), _d(J1), _d(gamma), _u8(dvalid), _d(u), _d(w)
    H, W = J0.shape
    uw, gw, Iu, rho = np.zeros((H, W)), np.zeros((H, W, 2)), np.zeros((H, W)), np.zeros((H, W))
    lib().or_linearise(W, H, _p(J0), _p(J1), _p(gamma), _p(dvalid), _p(u), _p(w), _p(uw), _p(gw),
                       _p(Iu), _p(rho))
    return uw, gw, Iu, rho


def clip_accumulate(du_max: float, u_w, gamma_w, u, w):
    u_w, gamma_w = _d(u_w), _d(gamma_w)
    u, w = _d(u).copy(), _d(w).copy()
    H, W = u.shape
    lib().or_clip_accumulate(W, H, ctypes.c_double(du_max), _p(u_w), _p(gamma_w), _p(u), _p(w))
    return u, w


def upsample(mask_c, u_c, w_c):
    mask_c, u_c, w_c = _u8(mask_c), _d(u_c), _d(w_c)
    Hc, Wc = mask_c.shape
    Hf, Wf = 2 * Hc, 2 * Wc
    uf, wf = np.zeros((Hf, Wf)), np.zeros((Hf, Wf, 2))
    lib().or_upsample(Wc, Hc, _p(mask_c), _p(u_c), _p(w_c), Wf, Hf, _p(uf), _p(wf))
    return uf, wf


def triangulate(cam0: dict, R, t, w, dvalid):
    H, W = cam0["height"], cam0["width"]
    w, dvalid = _d(w), _u8(dvalid)
    depth, Z, valid = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W), np.uint8)
    c0, Rr, tt = _cam(cam0), _R(R), _t(t)
    lib().or_triangulate(ctypes.byref(c0), _p(Rr), _p(tt), _p(w), _p(dvalid), _p(depth), _p(Z), _p(valid))
    return depth, Z, valid.astype(bool)


def data_valid(cam0: dict, cam1: dict, R, t, level: int):
    """dvalid_l = M_l and D_l and not epi_l (the per-level data-term switch)."""
    m0 = mask0(cam0)
    _, vc = calibration_field(cam0, cam1, R)
    d0 = (m0 & vc).astype(np.uint8)
    _, epi = trajectory_field(cam0, R, t, level)
    ml = level_mask(m0, level)
    dl = level_mask(d0, level)
    return (ml & dl & (1 - epi)).astype(np.uint8)


def solve(cam0: dict, cam1: dict, R, t, params: dict, I0, I1, levels_out: bool = False):
    """Whole method (Algorithm 1 in the pyramid of Sec. IV-B) on one pair."""
    H, W = cam0["height"], cam0["width"]
    I0, I1 = _d(I0), _d(I1)
    u, w = np.zeros((H, W)), np.zeros((H, W, 2))
    depth, Z, valid = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W), np.uint8)
    L = int(params["levels"])
    tot = sum((H >> l) * (W >> l) for l in range(L))
    lu = np.zeros(tot) if levels_out else None
    lw = np.zeros(2 * tot) if levels_out else None
    c0, c1, Rr, tt, pp = _cam(cam0), _cam(cam1), _R(R), _t(t), _par(params)
    st = lib().or_solve(ctypes.byref(c0), ctypes.byref(c1), _p(Rr), _p(tt), ctypes.byref(pp), _p(I0), _p(I1),
                        _p(u), _p(w), _p(depth), _p(Z), _p(valid), _p(lu), _p(lw))
    if st != 0:
        raise ValueError(f"oracle solve: status {st}")
    out = dict(u=u, w=w, depth=depth, Z=Z, valid=valid.astype(bool))
    if levels_out:
        off = 0
        out["levels"] = []
        for l in range(L):
            n = (H >> l) * (W >> l)
            out["levels"].append((lu[off:off + n].reshape(H >> l, W >> l),
                                  lw[2 * off:2 * off + 2 * n].reshape(H >> l, W >> l, 2)))
            off += n
    return out
