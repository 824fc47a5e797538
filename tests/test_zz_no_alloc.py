"""The allocation-free batched solve (vfs_solve_batch_noalloc, state in the
library's fixed device scratch) against the allocating one
(vfs_solve_batch): the same kernels on the same inputs, so every output must
be bitwise equal, on two calls in a row, the second with smaller pairs; a
batch beyond the scratch is rejected before any device work."""
import numpy as np
import pytest

from synth import configs, scene

pytestmark = pytest.mark.gpu


def _outs(n, H, W):
    import torch
    return [dict(u=torch.full((H, W), float("nan"), device="cuda"),
                 w=torch.full((H, W, 2), float("nan"), device="cuda"),
                 depth=torch.full((H, W), float("nan"), device="cuda"),
                 z=torch.full((H, W), float("nan"), device="cuda"),
                 valid=torch.full((H, W), 7, dtype=torch.uint8, device="cuda")) for _ in range(n)]


def _pairs(cid, n):
    import torch
    cfg = configs.get(cid)
    rig = scene.make_rig(cfg)
    I0, I1 = scene.render_pair(rig, cfg, 0, with_gt=False)[:2]
    rng = np.random.default_rng(5)
    I0s, I1s = [], []
    for b in range(n):
        # distinct pairs: the rendered pair, then with a seeded offset and noise
        d0 = (0.02 * b + 0.003 * b * rng.standard_normal(I0.shape)).astype(np.float32)
        I0s.append(torch.from_numpy(I0 + d0).cuda())
        I1s.append(torch.from_numpy(I1 + d0).cuda())
    return cfg, rig, I0s, I1s


def test_noalloc_equals_allocating_solve_on_two_calls():
    import torch
    import paper_1909_07545_amd as vfs
    from paper_1909_07545_amd import _lib
    assert torch.cuda.is_available()
    for cid, n, ov in (("c2", 1, {}), ("c1", 2, dict(storage=1))):
        cfg, rig, I0s, I1s = _pairs(cid, n)
        params = configs.solver_params(cfg, **ov)
        R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params["levels"])
        H, W = cfg["height"], cfg["width"]
        na = _lib.solve_batch_noalloc(R, I0s, I1s, params, _outs(n, H, W))
        ref = vfs.solve_batch(R, I0s, I1s, params)
        torch.cuda.synchronize()
        for b in range(n):
            for k in ("u", "w", "depth", "z", "valid"):
                assert torch.equal(na[b][k].nan_to_num(0.0, 1e30), ref[b][k].nan_to_num(0.0, 1e30)), (cid, b, k)
            assert torch.isfinite(na[b]["u"]).all()


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    import torch
    import paper_1909_07545_amd as vfs
    from paper_1909_07545_amd import _lib
    cfg, rig, I0s, I1s = _pairs("c2", 2)
    params = configs.solver_params(cfg)
    R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params["levels"])
    out = _outs(2, cfg["height"], cfg["width"])
    with pytest.raises(vfs.VfsError, match="allocation-free"):
        _lib.solve_batch_noalloc(R, I0s, I1s, params, out)
    torch.cuda.synchronize()
    assert torch.isnan(out[0]["u"]).all()
