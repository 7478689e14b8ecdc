"""GPU parity of the multi-disc footprint (Sec. IV-C: the vehicle body covered
by discs of radius r, one barrier row per (disc, obstacle)) against the FP64
oracle, at the stated bars (every sample's cost within relative 1e-4, the new
nominal sequence within 1e-4 of each input's range):

  - tractor discs ahead of (and behind) the rear axle and trailer discs behind
    the hitch, e = 2 and e = 4 obstacles mixed, moving obstacles, up to 32
    obstacle rows (8 obstacles x 4 discs) with the hitch rows;
  - the collision-penalty baseline summing every (disc, obstacle);
  - every launch shape (one, two, four and eight lanes per sample, in-kernel
    and precomputed normals) gives the same bits;
  - the default footprint (the rear axle alone) is eq. (16) as printed: a
    problem that names it explicitly gives the bits of one that does not;
  - more rows than BRMPPI_MAX_OBS, or a body with more than four discs, is
    EINVAL.
"""
import os
import sys

import numpy as np
import pytest

from paper_2508_05773_amd import brmppi as B
from paper_2508_05773_amd import workloads as W

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
J_RTOL = 1e-4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(arena_bytes=2 << 30, n_streams=1, max_controllers=16)
    yield c
    c.close()


def footprint_problem(seed, S, T, n_obs, discs_t, discs_r, e4="odd", flags=0):
    p = W.random_small(seed, S=S, T=T, n_obs=n_obs)
    obs = p.obstacles.copy()
    if e4 == "odd":
        obs[1::2, 5] = 4.0
    elif e4 == "all":
        obs[:, 5] = 4.0
    prm = W.make_params(0.05, disc_tractor=discs_t, disc_trailer=discs_r)
    return p.copy(obstacles=obs, params=prm, flags=flags)


def solve(ctx, prob, controller=0, block=0, variant=0):
    B.brmppi_set_launch(ctx.h, block, variant)
    try:
        ctx.set_path(controller, prob.path, prob.ds)
        log(f"  gpu {prob.name} S={prob.S} T={prob.T} n_obs={prob.n_obs} discs={W.n_discs(prob.params)} "
            f"shape=({block},{variant}) flags={prob.flags}")
        return B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(prob, controller=controller), want_J=True,
                                 allow=(B.OK, B.ENONFINITE))
    finally:
        B.brmppi_set_launch(ctx.h, 0, 0)


def compare(prob, g, o, label):
    J_g, J_o = g["J"].astype(np.float64), o["J"]
    fin = np.isfinite(J_o)
    assert np.array_equal(np.isfinite(J_g), fin), f"{label}: finiteness differs"
    rel = np.abs(J_g[fin] - J_o[fin]) / np.maximum(np.abs(J_o[fin]), 1e-30)
    P = prob.params
    tol = 1e-4 * np.array([P["j_hi"] - P["j_lo"], P["w_hi"] - P["w_lo"], P["nu_bar"]])
    du = np.abs(g["U_new"] - o["U_new"])
    log(f"  {label}: J max rel err {rel.max() if rel.size else 0:.3e}, U max abs err {du.max(axis=0)}")
    assert rel.size == 0 or rel.max() <= J_RTOL, label
    assert np.all(du <= tol), label


CASES = [
    # seed, S, T, n_obs, tractor discs, trailer discs, e4
    (60, 777, 20, 5, (0.0, 2.5), (), "odd"),
    (61, 1500, 25, 4, (-0.8, 1.5, 3.2), (2.0, 7.0), "odd"),
    (62, 1025, 15, 8, (0.0, 3.0), (1.5, 8.0), "all"),
    (63, 640, 12, 3, (), (0.5, 4.0, 9.0), "none"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_footprint_matches_oracle(ctx, case):
    from oracle import oracle as O
    seed, S, T, n_obs, dt, dr, e4 = case
    prob = footprint_problem(seed, S, T, n_obs, dt, dr, e4)
    assert prob.n_obs * W.n_discs(prob.params) <= B.MAX_OBS
    o = O.solve(prob, nthreads=NTHREADS)
    g = solve(ctx, prob)
    compare(prob, g, o, f"footprint seed={seed}")


def test_footprint_penalty_baseline(ctx):
    from oracle import oracle as O
    prob = footprint_problem(64, 900, 18, 6, (0.0, 2.0), (3.0,), "odd",
                             flags=W.FLAG_GUIDANCE_OFF | W.FLAG_COLLISION_PENALTY)
    o = O.solve(prob, nthreads=NTHREADS)
    g = solve(ctx, prob)
    compare(prob, g, o, "footprint penalty")


@pytest.mark.parametrize("block,variant", [(64, 0), (128, 1), (256, 2), (256, 3), (256, 4), (192, 4)])
def test_footprint_launch_shapes_bitwise(ctx, block, variant):
    prob = footprint_problem(65, 1100, 16, 8, (0.0, 1.0, 2.0, 3.5), (), "odd")
    assert prob.n_obs * W.n_discs(prob.params) == 32
    ref = solve(ctx, prob, controller=1, block=64, variant=0)
    got = solve(ctx, prob, controller=1, block=block, variant=variant)
    assert np.array_equal(got["J"], ref["J"])
    assert np.array_equal(got["U_new"], ref["U_new"])


def test_rear_axle_footprint_is_the_default(ctx):
    p = W.random_small(66, S=600, T=10, n_obs=6)
    explicit = p.copy(params=W.make_params(0.05, disc_tractor=(0.0,), disc_trailer=()))
    a, b = solve(ctx, p, controller=2), solve(ctx, explicit, controller=3)
    assert np.array_equal(a["J"], b["J"]) and np.array_equal(a["U_new"], b["U_new"])


def test_footprint_limits(ctx):
    p = footprint_problem(67, 64, 4, 9, (0.0, 2.0), (1.0, 4.0), "none")   # 36 rows
    ctx.set_path(4, p.path, p.ds)
    _, _, rc = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=4), allow=(B.EINVAL,))
    assert rc == B.EINVAL and "BRMPPI_MAX_OBS" in B.last_error()
    prm = B.params_struct(W.make_params(0.05))
    prm.n_disc_tractor = 5
    import ctypes as C
    assert B.lib().brmppi_set_params(ctx.h, 4, C.byref(prm)) == B.EINVAL
    prm.n_disc_tractor, prm.n_disc_trailer = 0, 0
    assert B.lib().brmppi_set_params(ctx.h, 4, C.byref(prm)) == B.EINVAL
