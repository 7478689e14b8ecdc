"""The values the paper prints for its experiments (Sec. V and Table I),
recorded in tests/golden/paper_sec5.json with their citations, against the
constants and configurations the library and the benchmark use."""
import json
import os

import numpy as np
import pytest

from paper_2508_05773_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_sec5.json")


@pytest.fixture(scope="module")
def paper():
    return json.load(open(GOLDEN))


def test_input_bounds_are_the_papers(paper):
    for Ts in (0.04, 0.05, 0.1):
        p = W.make_params(Ts)
        assert [p["j_lo"], p["j_hi"]] == paper["input_bounds"]["j"]
        assert [p["w_lo"], p["w_hi"]] == pytest.approx(paper["input_bounds"]["omega"], abs=1e-7)


def test_paper_configuration(paper):
    prob = W.paper_shape()
    h = paper["horizon"]
    assert prob.S == h["rollouts"] == W.PAPER_ROLLOUTS
    assert prob.T == h["steps"] == W.PAPER_HORIZON_STEPS
    assert prob.T * prob.params["Ts"] == pytest.approx(h["seconds"], rel=1e-6)
    v = paper["vehicle_m"]
    for k in ("l1", "l2", "lh"):
        assert prob.params[k] == pytest.approx(v[k], rel=1e-6)
    # the footprint disc covers the wider body (half the trailer width)
    assert prob.params["r_disc"] == pytest.approx(v["trailer_width"] / 2)
    o = paper["obstacles"]
    assert prob.n_obs == o["count"] == W.PAPER_OBSTACLES
    e = prob.obstacles[:, 5]
    assert np.sum(e == o["parked_vehicle_exponent"]) == o["count"] - 1
    ped = prob.obstacles[e == o["pedestrian_exponent"]]
    assert ped.shape[0] == 1 and np.hypot(ped[0, 6], ped[0, 7]) > 0      # the pedestrian moves


def test_paper_times_used_by_the_benchmark(paper):
    for direction in ("forward", "backward"):
        for method, ms in paper["time_ms"][direction].items():
            assert W.PAPER_TIME_MS[direction][method] == ms
