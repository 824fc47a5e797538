"""The warping-schedule ablation harness (tests/ablation_study.py) on a
reduced grid: one rendered 640x480 Kannala-Brandt room, N = 1, 2, 4 warps
at the 0.2 px clip and N = 2 at a 0.1 px clip.  Checks what the measurement
must show whatever the scene: the evaluated pixels are most of the image
circle's data-term pixels, the outlier shares are percentages ordered
tau>1 >= tau>3 >= tau>5, and the solve time grows with N (each warp adds the
same launches; the paper's Fig. 4 finds it linear)."""
import pytest

pytestmark = pytest.mark.gpu


def test_ablation_harness_on_a_reduced_grid():
    import torch
    import paper_1909_07545_amd as vfs
    from synth import configs
    from tests import ablation_study as ab
    assert torch.cuda.is_available()
    cfg = configs.get("c2")
    R, scenes = ab.prepare(vfs, cfg, 1)
    rows = [ab.run(vfs, cfg, R, scenes, n, 0.2) for n in (1, 2, 4)] + [ab.run(vfs, cfg, R, scenes, 2, 0.1)]
    for r in rows:
        print("ablation", r, flush=True)
        assert 100.0 >= r["tau1_pct"] >= r["tau3_pct"] >= r["tau5_pct"] >= 0.0
        assert r["pixels"] > 0.3 * cfg["width"] * cfg["height"]
    t1, t2, t4 = (r["ms_per_solve"] for r in rows[:3])
    assert t1 < t2 < t4
    # time per added warp roughly constant (within a factor 2)
    assert 0.5 < (t4 - t2) / (2 * (t2 - t1)) < 2.0
