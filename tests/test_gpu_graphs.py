"""Graph replay of the direct solves (vfs_rig_graphs): a solve replayed from
the HIP graph captured at the first solve of its launch configuration gives
the eager launches' outputs bit for bit, on every replay (with the library's
and the caller's eager work and synchronisations in between), for new input
and output buffers of the same configuration, and after a configuration
change and back."""
import numpy as np
import pytest

from synth import configs, scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vfs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_07545_amd as v
    return v


def _pairs(cid, n, seed):
    import torch
    cfg = configs.get(cid)
    rig = scene.make_rig(cfg)
    I0, I1 = scene.render_pair(rig, cfg, 0, with_gt=False)[:2]
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        d = (0.01 * b + 0.004 * rng.standard_normal(I0.shape)).astype(np.float32)
        out.append((torch.from_numpy(I0 + d).cuda(), torch.from_numpy(I1 + d).cuda()))
    return cfg, rig, out


def _equal(a, b):
    import torch
    return all(torch.equal(x[k], y[k]) for x, y in zip(a, b) for k in ("u", "w", "depth", "z", "valid"))


@pytest.mark.parametrize("cid,n,ov", [("c1", 2, {}), ("c2", 1, {}), ("r200", 3, dict(reg="tv", storage=1)),
                                      ("c1", 2, dict(storage=2, theta_gamma=0.3))])
def test_graph_replays_equal_eager_launches(vfs, cid, n, ov):
    import torch
    cfg, rig, pairs = _pairs(cid, n, 1)
    params = configs.solver_params(cfg, **ov)
    R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params["levels"])
    I0s = [p[0] for p in pairs]
    I1s = [p[1] for p in pairs]
    R.use_graphs(False)
    eager = vfs.solve_batch(R, I0s, I1s, params)
    torch.cuda.synchronize()
    R.use_graphs(True)
    for rep in range(3):
        got = vfs.solve_batch(R, I0s, I1s, params)       # rep 0 captures, then replays
        torch.cuda.synchronize()
        assert _equal(got, eager), rep
        # eager work of the library and of the caller between replays
        R.use_graphs(False)
        vfs.solve_batch(R, I0s[:1], I1s[:1], dict(params, iters=3))
        R.use_graphs(True)
        (I0s[0] * 2.0).sum().item()
    # new inputs and outputs, same configuration: the same graph, other buffers
    _, _, other = _pairs(cid, n, 2)
    J0s = [p[0] for p in other]
    J1s = [p[1] for p in other]
    got = vfs.solve_batch(R, J0s, J1s, params)
    R.use_graphs(False)
    ref = vfs.solve_batch(R, J0s, J1s, params)
    torch.cuda.synchronize()
    assert _equal(got, ref)
    # another configuration, then back to the first one's graph
    R.use_graphs(True)
    vfs.solve_batch(R, I0s, I1s, dict(params, warps=1))
    again = vfs.solve_batch(R, I0s, I1s, params)
    torch.cuda.synchronize()
    assert _equal(again, eager)
