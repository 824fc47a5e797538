"""The solver parameters used everywhere are the ones the paper prints
(golden fixture with its citation)."""
import json
import os

from synth import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def test_paper_parameters():
    g = json.load(open(GOLDEN))
    p = configs.PAPER_PARAMS
    assert p["beta"] == g["beta"] and p["eta"] == g["eta"]
    assert p["alpha0"] == g["alpha0"] and p["alpha1"] == g["alpha1"]
    assert p["du_max"] == g["du_max_px"]
    ex = g["example_800x800"]
    # 800 / 2^(5-1) = 50: the printed pyramid reaches the printed minimum width
    assert 800 / ex["pyramid_scale"] ** (ex["pyramid_levels"] - 1) == ex["min_width"]
