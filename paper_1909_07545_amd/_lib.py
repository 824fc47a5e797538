"""ctypes binding of libvfs.so (the C ABI of include/vfs.h)."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvfs.so")

FIELD_TRAJECTORY, FIELD_CALIBRATION, FIELD_FLAGS = 0, 1, 2
F_MASK, F_MX, F_MY, F_DATA, F_EPI = 1, 2, 4, 8, 16
MODELS = {"pinhole": 0, "equidistant": 1, "kb": 2, "kannala_brandt": 2, "unified": 3, "ucm": 3,
          "eucm": 4, "enhanced_unified": 4}
REGS = {"tgv": 0, "tv": 1}
DATA_TERMS = {"brightness": 0, "rank": 1, "gradient": 2}
STATUS = {0: "VFS_OK", -1: "VFS_E_INVALID", -2: "VFS_E_NOMEM", -3: "VFS_E_BUDGET", -4: "VFS_E_MODEL",
          -5: "VFS_E_DEGENERATE", -6: "VFS_E_DEVICE"}


class VfsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("width", ctypes.c_int), ("height", ctypes.c_int),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("k", ctypes.c_double * 4), ("fov_deg", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("warps", ctypes.c_int), ("iters", ctypes.c_int),
                ("reg", ctypes.c_int), ("lam", ctypes.c_double), ("alpha0", ctypes.c_double),
                ("alpha1", ctypes.c_double), ("beta", ctypes.c_double), ("eta", ctypes.c_double),
                ("du_max", ctypes.c_double), ("theta_gamma", ctypes.c_double), ("storage", ctypes.c_int),
                ("pass_iters", ctypes.c_int), ("data_term", ctypes.c_int)]


class Probe(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("warp", ctypes.c_int), ("pair", ctypes.c_int),
                ("pitch", ctypes.c_size_t)] + [(k, ctypes.c_void_p) for k in (
                    "J0", "J1", "u", "w", "v", "p", "q", "tpack", "rho", "gw", "u_pd", "v_pd", "p_pd", "q_pd",
                    "u_next", "w_next")]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("use_graphs", ctypes.c_int)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_longlong), ("peak_active", ctypes.c_longlong),
                ("pool_peak_bytes", ctypes.c_size_t), ("buckets", ctypes.c_int), ("joins", ctypes.c_longlong),
                ("full_ticks", ctypes.c_longlong)]


SERVE_BATCHED, SERVE_PLAIN = 0, 1

_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1909_07545_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.vfs_last_error.restype = ctypes.c_char_p
        L.vfs_rig_create.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp]
        L.vfs_rig_destroy.argtypes = [_vp]
        L.vfs_rig_destroy.restype = None
        L.vfs_rig_field.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp]
        L.vfs_solve_batch.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp]
        L.vfs_solve_batch_noalloc.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp,
                                              _vp, _vp, _vp, _vp]
        L.vfs_solve_probe.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        L.vfs_rig_graphs.argtypes = [_vp, ctypes.c_int]
        L.vfs_solve.argtypes = [_vp, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.vfs_step_tensor.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _vp, _vp, ctypes.c_double,
                                      ctypes.c_double, _vp, _vp]
        L.vfs_step_linearise.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t] + [_vp] * 10 + \
            [ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp]
        L.vfs_step_pd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t] + [_vp] * 11 + \
            [_vp, ctypes.c_int, _vp]
        L.vfs_step_upsample.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _vp, _vp, _vp,
                                        ctypes.c_size_t, _vp, _vp, _vp]
        L.vfs_step_triangulate.argtypes = [_vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        L.vfs_profile_enable.argtypes = [_vp, ctypes.c_int]
        L.vfs_profile_read.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int]
        L.vfs_params_default.argtypes = [_vp]
        L.vfs_step_rank.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        L.vfs_step_gradient.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        L.vfs_rectify_rotations.argtypes = [_vp] * 5
        L.vfs_rectify.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp, _vp]
        L.vfs_unrectify.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp, _vp]
        L.vfs_step_energy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t] + [_vp] * 7 + [_vp]
        L.vfs_step_pd_energy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t] + [_vp] * 11 + \
            [_vp, ctypes.c_int, _vp, _vp]
        L.vfs_diff_stats.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.vfs_server_config_default.argtypes = [_vp]
        L.vfs_server_create.argtypes = [_vp, _vp, _vp]
        L.vfs_server_request_bytes.argtypes = [_vp, _vp, _vp]
        L.vfs_server_submit.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_double, ctypes.c_double, _vp]
        L.vfs_server_poll.argtypes = [_vp, ctypes.c_ulonglong, _vp, _vp]
        L.vfs_server_times.argtypes = [_vp, ctypes.c_ulonglong, _vp, _vp]
        L.vfs_server_wait_all.argtypes = [_vp, ctypes.c_double]
        L.vfs_server_stats.argtypes = [_vp, _vp]
        L.vfs_server_destroy.argtypes = [_vp]
        L.vfs_server_destroy.restype = None
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise VfsError(st, lib().vfs_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _camera(c: dict) -> Camera:
    m = c["model"]
    return Camera(MODELS[m] if isinstance(m, str) else int(m), int(c["width"]), int(c["height"]),
                  float(c["fx"]), float(c["fy"]), float(c["cx"]), float(c["cy"]),
                  (ctypes.c_double * 4)(*[float(x) for x in c.get("k", (0.0,) * 4)]), float(c["fov_deg"]))


def default_params() -> dict:
    p = Params()
    _check(lib().vfs_params_default(ctypes.byref(p)))
    return dict(levels=p.levels, warps=p.warps, iters=p.iters, reg="tgv" if p.reg == 0 else "tv",
                alpha0=p.alpha0, alpha1=p.alpha1, beta=p.beta, eta=p.eta, du_max=p.du_max,
                theta_gamma=p.theta_gamma, storage=p.storage, pass_iters=p.pass_iters,
                data_term={v: k for k, v in DATA_TERMS.items()}[p.data_term], **{"lambda": p.lam})


def _params(d: dict) -> Params:
    reg = d.get("reg", "tgv")
    return Params(int(d["levels"]), int(d["warps"]), int(d["iters"]),
                  REGS[reg] if isinstance(reg, str) else int(reg), float(d["lambda"]), float(d["alpha0"]),
                  float(d["alpha1"]), float(d["beta"]), float(d["eta"]), float(d["du_max"]),
                  float(d.get("theta_gamma", 0.0)), int(d.get("storage", 0)), int(d.get("pass_iters", 0)),
                  DATA_TERMS[dt] if isinstance(dt := d.get("data_term", 0), str) else int(dt))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


_F32, _U8 = (torch.float32,), (torch.uint8,)


def _need(t, shape, dtypes, name, optional=False):
    """t, checked: a contiguous CUDA tensor of one of ``dtypes`` and of this
    shape (None passes when ``optional``).  The C ABI takes bare pointers
    and the sizes given beside them, so these checks are what keeps its
    kernels inside the caller's buffers."""
    if t is None:
        if optional:
            return None
        raise TypeError(f"{name}: a tensor is required")
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise TypeError(f"{name}: expected a contiguous CUDA tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _plane(t, name):
    """(rows, columns) of a 2-D tensor argument that sets the others' sizes."""
    if not (isinstance(t, torch.Tensor) and t.dim() == 2):
        raise ValueError(f"{name}: expected a 2-D tensor")
    return int(t.shape[0]), int(t.shape[1])


def _batch_args(rig, I0s, I1s, betas, etas, out=None):
    """Checks of a batch's images (one I0 and one I1 of the rig's size per
    pair), per-pair tensor parameters and output tensors; returns n."""
    n = len(I0s)
    if len(I1s) != n:
        raise ValueError(f"I1s: {len(I1s)} images for {n} pairs")
    for name, seq in (("betas", betas), ("etas", etas)):
        if seq is not None and len(seq) != n:
            raise ValueError(f"{name}: {len(seq)} values for {n} pairs")
    if out is not None and len(out) != n:
        raise ValueError(f"out: {len(out)} entries for {n} pairs")
    H, W = rig.height, rig.width
    for k in range(n):
        _need(I0s[k], (H, W), _F32, f"I0s[{k}]")
        _need(I1s[k], (H, W), _F32, f"I1s[{k}]")
    if out is not None:
        for k, o in enumerate(out):
            _outputs(o, H, W, f"out[{k}]", required=("u", "w", "depth", "z", "valid"))
    return n


def _outputs(o, H, W, name, required):
    """Output tensors of one pair: u, depth, z (H, W) float32, w (H, W, 2)
    float32, valid (H, W) uint8; the keys not in ``required`` may be absent."""
    shapes = dict(u=((H, W), _F32), w=((H, W, 2), _F32), depth=((H, W), _F32), z=((H, W), _F32),
                  valid=((H, W), _U8))
    for k, (shape, dt) in shapes.items():
        _need(o.get(k), shape, dt, f"{name}['{k}']", optional=k not in required)


class Rig:
    """Trajectory / calibration fields and masks of one calibration (vfs_rig_create)."""

    def __init__(self, cam0: dict, cam1: dict, R, t, levels: int, stream=None):
        self._h = ctypes.c_void_p()
        c0, c1 = _camera(cam0), _camera(cam1)
        Rr = (ctypes.c_double * 9)(*np.asarray(R, np.float64).reshape(9).tolist())
        tt = (ctypes.c_double * 3)(*np.asarray(t, np.float64).reshape(3).tolist())
        _check(lib().vfs_rig_create(ctypes.byref(c0), ctypes.byref(c1), Rr, tt, int(levels), _stream(stream),
                                    ctypes.byref(self._h)))
        self.cam0, self.cam1, self.levels = dict(cam0), dict(cam1), int(levels)
        self.width, self.height = int(cam0["width"]), int(cam0["height"])

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().vfs_rig_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def use_graphs(self, enable: bool = True):
        """Replay captured graphs for this rig's solves (vfs_rig_graphs)."""
        _check(lib().vfs_rig_graphs(self._h, int(bool(enable))))

    def field(self, level: int, which: int, stream=None) -> torch.Tensor:
        H, W = self.height >> level, self.width >> level
        if which == FIELD_FLAGS:
            out = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            pitch = W
        else:
            out = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
            pitch = 8 * W
        _check(lib().vfs_rig_field(self._h, int(level), int(which), _ptr(out), pitch, _stream(stream)))
        return out


def solve_batch(rig: Rig, I0s, I1s, params: dict, betas=None, etas=None, stream=None, out=None):
    """Whole method on a batch of pairs (vfs_solve_batch).  Inputs: lists of
    (H, W) float32 CUDA tensors.  Returns a list of dicts of output tensors
    (u, w, depth, z, valid); ``out`` may pass pre-allocated ones."""
    n = _batch_args(rig, I0s, I1s, betas, etas, out)
    H, W = rig.height, rig.width
    if out is None:
        f32 = dict(dtype=torch.float32, device="cuda")     # whatever torch's default dtype is
        out = [dict(u=torch.empty((H, W), **f32), w=torch.empty((H, W, 2), **f32),
                    depth=torch.empty((H, W), **f32), z=torch.empty((H, W), **f32),
                    valid=torch.empty((H, W), dtype=torch.uint8, device="cuda")) for _ in range(n)]
    arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
    p = _params(params)
    bet = (ctypes.c_double * n)(*betas) if betas is not None else None
    et = (ctypes.c_double * n)(*etas) if etas is not None else None
    _check(lib().vfs_solve_batch(rig.handle, n, arr(I0s), arr(I1s), 4 * W, arr([o["u"] for o in out]),
                                 arr([o["w"] for o in out]), arr([o["depth"] for o in out]),
                                 arr([o["z"] for o in out]), arr([o["valid"] for o in out]), ctypes.byref(p),
                                 bet, et, _stream(stream)))
    return out


_STORAGE_DTYPE = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}


def solve_probe(rig: Rig, I0s, I1s, params: dict, level: int, warp: int, pair: int = 0, betas=None, etas=None,
                stream=None) -> dict:
    """The state of pair ``pair`` of a batched solve at warp ``warp`` of
    level ``level`` (vfs_solve_probe): returns CUDA tensors J0, J1, u, w, v,
    p, q, tpack, rho, gw (after the warp's linearisation), u_pd, v_pd, p_pd,
    q_pd (after its iterations) and u_next, w_next (after its clip); p, q and
    tpack in the storage dtype (float32, float16 or bfloat16)."""
    n = _batch_args(rig, I0s, I1s, betas, etas)
    H, W = rig.height, rig.width
    lv = min(max(int(level), 0), rig.levels - 1)   # plane sizes only: the library checks the level
    Hl, Wl = H >> lv, W >> lv
    sd = _STORAGE_DTYPE[int(params.get("storage", 0))]
    tgv = params.get("reg", "tgv") in ("tgv", 0)
    shapes = dict(J0=(1, torch.float32), J1=(1, torch.float32), u=(1, torch.float32), w=(2, torch.float32),
                  v=(2, torch.float32), p=(2, sd), q=(4, sd), tpack=(4, sd), rho=(1, torch.float32),
                  gw=(2, torch.float32), u_pd=(1, torch.float32), v_pd=(2, torch.float32), p_pd=(2, sd),
                  q_pd=(4, sd), u_next=(1, torch.float32), w_next=(2, torch.float32))
    out = {}
    for k, (c, dt) in shapes.items():
        if not tgv and k in ("v", "q", "v_pd", "q_pd"):
            continue
        out[k] = torch.full((Hl, Wl) if c == 1 else (Hl, Wl, c), float("nan"), dtype=dt, device="cuda")
    pr = Probe(int(level), int(warp), int(pair), Wl, *[out[k].data_ptr() if k in out else None
                                                        for k in shapes])
    arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
    pp = _params(params)
    bet = (ctypes.c_double * n)(*betas) if betas is not None else None
    et = (ctypes.c_double * n)(*etas) if etas is not None else None
    _check(lib().vfs_solve_probe(rig.handle, n, arr(I0s), arr(I1s), 4 * W, ctypes.byref(pp), bet, et,
                                 ctypes.byref(pr), _stream(stream)))
    return out


def solve_batch_noalloc(rig: Rig, I0s, I1s, params: dict, out: list, betas=None, etas=None, stream=None):
    """vfs_solve_batch_noalloc: the batched solve with the library's fixed
    device scratch instead of an allocated workspace.  ``out``: one dict of
    pre-allocated output tensors (u, w, depth, z, valid) per pair."""
    n = _batch_args(rig, I0s, I1s, betas, etas, out)
    W = rig.width
    arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
    p = _params(params)
    bet = (ctypes.c_double * n)(*betas) if betas is not None else None
    et = (ctypes.c_double * n)(*etas) if etas is not None else None
    _check(lib().vfs_solve_batch_noalloc(rig.handle, n, arr(I0s), arr(I1s), 4 * W, arr([o["u"] for o in out]),
                                         arr([o["w"] for o in out]), arr([o["depth"] for o in out]),
                                         arr([o["z"] for o in out]), arr([o["valid"] for o in out]),
                                         ctypes.byref(p), bet, et, _stream(stream)))
    return out


def solve(rig: Rig, I0, I1, params: dict, stream=None):
    return solve_batch(rig, [I0], [I1], params, stream=stream)[0]


def step_tensor(J0, flags, beta: float, eta: float, tpack, stream=None):
    H, W = _plane(J0, "J0")
    _need(J0, (H, W), _F32, "J0")
    _need(flags, (H, W), _U8, "flags")
    _need(tpack, (H, W, 4), _F32, "tpack")
    _check(lib().vfs_step_tensor(W, H, W, _ptr(J0), _ptr(flags), float(beta), float(eta), _ptr(tpack),
                                 _stream(stream)))


def step_linearise(J0, J1, gamma, flags, u, u_w, w, gamma_w, tpack, rho, clip: bool, clip_only: bool,
                   du_max: float, stream=None):
    H, W = _plane(J0, "J0")
    for name, t, c, dt in (("J0", J0, 1, _F32), ("J1", J1, 1, _F32), ("gamma", gamma, 2, _F32),
                           ("flags", flags, 1, _U8), ("u", u, 1, _F32), ("u_w", u_w, 1, _F32), ("w", w, 2, _F32),
                           ("gamma_w", gamma_w, 2, _F32), ("tpack", tpack, 4, _F32), ("rho", rho, 1, _F32)):
        _need(t, (H, W) if c == 1 else (H, W, c), dt, name)
    _check(lib().vfs_step_linearise(W, H, W, _ptr(J0), _ptr(J1), _ptr(gamma), _ptr(flags), _ptr(u), _ptr(u_w),
                                    _ptr(w), _ptr(gamma_w), _ptr(tpack), _ptr(rho), int(clip), int(clip_only),
                                    float(du_max), _stream(stream)))


def step_pd(tpack, rho, flags, u, v, p, q, params: dict, iters: int, stream=None, width=None, height=None):
    """vfs_step_pd on (rows, pitch[, c]) planes; width / height (default: the
    planes' pitch and row count) give the image inside them."""
    rows, pitch = _plane(u, "u")
    W = pitch if width is None else int(width)
    H = rows if height is None else int(height)
    if not (0 < W <= pitch and 0 < H <= rows):
        raise ValueError("step_pd: width / height outside the planes")
    _state_args(tpack, rho, flags, u, v, p, q, rows, pitch, _STORAGE_DTYPE[int(params.get("storage", 0))])
    su, sp = torch.empty_like(u), torch.empty_like(p)
    sv = torch.empty_like(v) if v is not None else None
    sq = torch.empty_like(q) if q is not None else None
    pp = _params(params)
    _check(lib().vfs_step_pd(W, H, pitch, _ptr(tpack), _ptr(rho), _ptr(flags), _ptr(u), _ptr(v), _ptr(p), _ptr(q),
                             _ptr(su), _ptr(sv), _ptr(sp), _ptr(sq), ctypes.byref(pp), int(iters),
                             _stream(stream)))


def _state_args(tpack, rho, flags, u, v, p, q, rows, pitch, sd):
    """The primal-dual state's planes (rows x pitch): u, rho float32, flags
    uint8, v (2) float32, p (2), q (4) and tpack (4) in the storage dtype sd;
    v and q may be None (TV-L1)."""
    _need(tpack, (rows, pitch, 4), (sd,), "tpack")
    _need(rho, (rows, pitch), _F32, "rho")
    _need(flags, (rows, pitch), _U8, "flags")
    _need(u, (rows, pitch), _F32, "u")
    _need(v, (rows, pitch, 2), _F32, "v", optional=True)
    _need(p, (rows, pitch, 2), (sd,), "p")
    _need(q, (rows, pitch, 4), (sd,), "q", optional=True)


def step_rank(I0, I1, R0, R1, stream=None):
    """Rank transforms of two (H, W) planes into R0, R1 (vfs_step_rank)."""
    H, W = _plane(I0, "I0")
    for name, t in (("I0", I0), ("I1", I1), ("R0", R0), ("R1", R1)):
        _need(t, (H, W), _F32, name)
    _check(lib().vfs_step_rank(W, H, W, _ptr(I0), _ptr(I1), _ptr(R0), _ptr(R1), _stream(stream)))


def step_gradient(I0, I1, G0, G1, stream=None):
    """Gradient magnitudes of two (H, W) planes into G0, G1 (vfs_step_gradient)."""
    H, W = _plane(I0, "I0")
    for name, t in (("I0", I0), ("I1", I1), ("G0", G0), ("G1", G1)):
        _need(t, (H, W), _F32, name)
    _check(lib().vfs_step_gradient(W, H, W, _ptr(I0), _ptr(I1), _ptr(G0), _ptr(G1), _stream(stream)))


def step_energy(tpack, rho, flags, u, v, params: dict, stream=None) -> float:
    """Linearised energy of Eq. (10) of the state (u, v) (vfs_step_energy)."""
    H, W = _plane(u, "u")
    _need(tpack, (H, W, 4), _F32, "tpack")
    _need(rho, (H, W), _F32, "rho")
    _need(flags, (H, W), _U8, "flags")
    _need(u, (H, W), _F32, "u")
    _need(v, (H, W, 2), _F32, "v", optional=True)
    e = ctypes.c_double()
    pp = _params(params)
    _check(lib().vfs_step_energy(W, H, W, _ptr(tpack), _ptr(rho), _ptr(flags), _ptr(u), _ptr(v), ctypes.byref(pp),
                                 ctypes.byref(e), _stream(stream)))
    return e.value


def step_pd_energy(tpack, rho, flags, u, v, p, q, params: dict, iters: int, stream=None):
    """vfs_step_pd with the energy of every primal iterate: returns the
    (iters + 1,) energies E(x^0) .. E(x^iters)."""
    H, W = _plane(u, "u")
    _state_args(tpack, rho, flags, u, v, p, q, H, W, torch.float32)
    su, sp = torch.empty_like(u), torch.empty_like(p)
    sv = torch.empty_like(v) if v is not None else None
    sq = torch.empty_like(q) if q is not None else None
    pp = _params(params)
    out = np.zeros(int(iters) + 1, np.float64)
    _check(lib().vfs_step_pd_energy(W, H, W, _ptr(tpack), _ptr(rho), _ptr(flags), _ptr(u), _ptr(v), _ptr(p),
                                    _ptr(q), _ptr(su), _ptr(sv), _ptr(sp), _ptr(sq), ctypes.byref(pp), int(iters),
                                    out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return out


def diff_stats(a, b, flags=None, stream=None):
    """(mean, max, count) of |a - b| over flags bit 0 (all pixels if None)."""
    H, W = _plane(a, "a")
    _need(a, (H, W), _F32, "a")
    _need(b, (H, W), _F32, "b")
    _need(flags, (H, W), _U8, "flags", optional=True)
    mean, mx, cnt = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
    _check(lib().vfs_diff_stats(W, H, W, _ptr(a), _ptr(b), _ptr(flags), ctypes.byref(mean), ctypes.byref(mx),
                                ctypes.byref(cnt), _stream(stream)))
    return mean.value, mx.value, cnt.value


def step_upsample(flags_c, u_c, w_c, u_f, w_f, stream=None):
    """(u, w) of a coarse level (Hc, Wc) to the fine planes (2 Hc, 2 Wc)."""
    Hc, Wc = _plane(u_c, "u_c")
    _need(flags_c, (Hc, Wc), _U8, "flags_c")
    _need(u_c, (Hc, Wc), _F32, "u_c")
    _need(w_c, (Hc, Wc, 2), _F32, "w_c")
    _need(u_f, (2 * Hc, 2 * Wc), _F32, "u_f")
    _need(w_f, (2 * Hc, 2 * Wc, 2), _F32, "w_f")
    _check(lib().vfs_step_upsample(Wc, Hc, Wc, _ptr(flags_c), _ptr(u_c), _ptr(w_c), 2 * Wc, _ptr(u_f), _ptr(w_f),
                                   _stream(stream)))


def step_triangulate(rig: Rig, w, depth, z=None, valid=None, stream=None):
    H, W = rig.height, rig.width
    _need(w, (H, W, 2), _F32, "w")
    _need(depth, (H, W), _F32, "depth")
    _need(z, (H, W), _F32, "z", optional=True)
    _need(valid, (H, W), _U8, "valid", optional=True)
    _check(lib().vfs_step_triangulate(rig.handle, rig.width, _ptr(w), _ptr(depth), _ptr(z), _ptr(valid),
                                      _stream(stream)))


def rectify_rotations(R, t):
    """(Rv0, Rv1, baseline) of the shared virtual orientation of a rig
    (vfs_rectify_rotations; host only)."""
    Rr = (ctypes.c_double * 9)(*np.asarray(R, np.float64).reshape(9).tolist())
    tt = (ctypes.c_double * 3)(*np.asarray(t, np.float64).reshape(3).tolist())
    a, b, base = (ctypes.c_double * 9)(), (ctypes.c_double * 9)(), ctypes.c_double()
    _check(lib().vfs_rectify_rotations(Rr, tt, a, b, ctypes.byref(base)))
    return np.array(a[:]).reshape(3, 3), np.array(b[:]).reshape(3, 3), base.value


def rectify(cam: dict, Rv, pinhole: dict, src, dst, valid=None, stream=None):
    """Virtual pinhole view of a camera image (vfs_rectify): src (H, W) of
    cam, dst / valid (Hp, Wp) of the pinhole view."""
    c, pn = _camera(cam), _camera(pinhole)
    R9 = (ctypes.c_double * 9)(*np.asarray(Rv, np.float64).reshape(9).tolist())
    _check(lib().vfs_rectify(ctypes.byref(c), R9, ctypes.byref(pn), _ptr(src), src.shape[1], _ptr(dst),
                             dst.shape[1], _ptr(valid), _stream(stream)))


def unrectify(cam: dict, Rv, pinhole: dict, field, dst, field_valid=None, valid=None, stream=None):
    """A pinhole-view field sampled at the camera's pixels (vfs_unrectify)."""
    c, pn = _camera(cam), _camera(pinhole)
    R9 = (ctypes.c_double * 9)(*np.asarray(Rv, np.float64).reshape(9).tolist())
    _check(lib().vfs_unrectify(ctypes.byref(c), R9, ctypes.byref(pn), _ptr(field), _ptr(field_valid),
                               field.shape[1], _ptr(dst), dst.shape[1], _ptr(valid), _stream(stream)))


def profile_enable(rig: Rig, on: bool = True):
    _check(lib().vfs_profile_enable(rig.handle, int(on)))


def profile_read(rig: Rig, reset: bool = True):
    """(milliseconds, launches, iterations per launch) of the level-0
    multi-iteration primal-dual launches since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    it = ctypes.c_int()
    _check(lib().vfs_profile_read(rig.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(it), int(reset)))
    return ms.value, n.value, it.value


class Server:
    """Request loop of vfs_server_create: ``mode`` "batched" (continuous
    batching over size buckets, HBM-budget admission, graph replays) or
    "plain" (one request at a time, arrival order, eager launches).  The
    object keeps each request's tensors alive until the request is done."""

    def __init__(self, params: dict, mode: str = "batched", hbm_budget_bytes: int = 1 << 30,
                 max_slots: int = 16, use_graphs: bool = True):
        cfg = ServerConfig()
        _check(lib().vfs_server_config_default(ctypes.byref(cfg)))
        cfg.mode = SERVE_PLAIN if mode == "plain" else SERVE_BATCHED
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.use_graphs = int(bool(use_graphs))
        p = _params(dict(params, levels=params.get("levels", 1)))
        self._h = ctypes.c_void_p()
        _check(lib().vfs_server_create(ctypes.byref(cfg), ctypes.byref(p), ctypes.byref(self._h)))
        self._keep = {}

    def request_bytes(self, rig: Rig) -> int:
        b = ctypes.c_size_t()
        _check(lib().vfs_server_request_bytes(self._h, rig.handle, ctypes.byref(b)))
        return b.value

    def submit(self, rig: Rig, I0, I1, out: dict, beta: float, eta: float) -> int:
        """Queue one pair; ``out`` holds pre-allocated output tensors (keys u,
        w, depth, z, valid; u/w/z/valid may be missing).  Returns the ticket."""
        H, W = rig.height, rig.width
        _need(I0, (H, W), _F32, "I0")
        _need(I1, (H, W), _F32, "I1")
        _outputs(out, H, W, "out", required=("depth",))
        tk = ctypes.c_ulonglong()
        _check(lib().vfs_server_submit(self._h, rig.handle, _ptr(I0), _ptr(I1), 4 * W, _ptr(out.get("u")),
                                       _ptr(out.get("w")), _ptr(out["depth"]), _ptr(out.get("z")),
                                       _ptr(out.get("valid")), float(beta), float(eta), ctypes.byref(tk)))
        self._keep[tk.value] = (rig, I0, I1, out)
        return tk.value

    def poll(self, ticket: int):
        """(done, latency in seconds or None)."""
        done = ctypes.c_int()
        lat = ctypes.c_double()
        _check(lib().vfs_server_poll(self._h, ctypes.c_ulonglong(ticket), ctypes.byref(done), ctypes.byref(lat)))
        if done.value:
            self._keep.pop(ticket, None)
            return True, lat.value
        return False, None

    def times(self, ticket: int):
        """(admission, completion) in seconds after arrival (-1: not yet)."""
        a, d = ctypes.c_double(), ctypes.c_double()
        _check(lib().vfs_server_times(self._h, ctypes.c_ulonglong(ticket), ctypes.byref(a), ctypes.byref(d)))
        return a.value, d.value

    def wait_all(self, timeout_s: float = 600.0):
        _check(lib().vfs_server_wait_all(self._h, float(timeout_s)))
        self._keep.clear()

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib().vfs_server_stats(self._h, ctypes.byref(c)))
        return dict(ticks=c.ticks, peak_active=c.peak_active, pool_peak_bytes=c.pool_peak_bytes,
                    buckets=c.buckets, joins=c.joins, full_ticks=c.full_ticks)

    def close(self):
        if self._h:
            lib().vfs_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
