"""GPU parity at full size, against FP64 oracle results stored by
tests/golden/make_oracle_refs.py (the oracle needs minutes of CPU time for these
cases, so its results are computed once, from oracle/ alone):

  - the 65536-sample, 100-step, 32-obstacle update: U_new in full, J_min, Z,
    ESS and 1025 per-sample costs (the unfused reduction at 64 groups);
  - eight requests of the served mix at their full S, T and obstacle counts,
    moving obstacles included, submitted together through the served form;

and the FP32 Box-Muller factors of every one of the 2^23 uniforms against
their FP64 values, which is the measurement behind the normals tolerance.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2508_05773_amd import brmppi as B
from paper_2508_05773_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_oracle_refs as REF  # noqa: E402

J_RTOL = 1e-4


def log(msg):
    print(msg, flush=True)


def u_tol(prob):
    P = prob.params
    return 1e-4 * np.array([P["j_hi"] - P["j_lo"], P["w_hi"] - P["w_lo"], P["nu_bar"]])


@pytest.fixture(scope="module")
def refs():
    d = json.load(open(REF.OUT))
    assert d["oracle_sha"] == REF.oracle_sha(), "stale oracle_large.json: rerun tests/golden/make_oracle_refs.py"
    return d["cases"]


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(arena_bytes=3 << 30, n_streams=3, max_controllers=64)
    yield c
    c.close()


def check_case(name, prob, ref, U, stats, J=None):
    assert ref["fingerprint"] == REF.fingerprint(prob), f"{name}: inputs differ from the stored case"
    du = np.abs(U - np.array(ref["U_new"]))
    tol = u_tol(prob)
    msg = f"  {name}: U max abs err {du.max(axis=0)} vs {tol}"
    if J is not None:
        ids = np.array(ref["J_ids"])
        Jo = np.array(ref["J"])
        fin = np.isfinite(Jo)
        assert np.array_equal(np.isfinite(J[ids]), fin)
        rel = np.abs(J[ids][fin].astype(np.float64) - Jo[fin]) / np.abs(Jo[fin])
        msg += f", J max rel err {rel.max():.3e} over {ids.size} samples"
        assert rel.max() <= J_RTOL, name
    log(msg + f", ess gpu {stats['ess']:.2f} oracle {ref['ess']:.2f}")
    assert np.all(du <= tol), name
    assert stats["J_min"] == pytest.approx(ref["J_min"], rel=J_RTOL)
    # Z and the ESS are sums of exp(-(J - J_min)/lambda): J errors of 1e-4 J
    # move them by about J_max 1e-4 / lambda relative
    assert stats["Z"] == pytest.approx(ref["Z"], rel=1e-2)
    assert stats["ess"] == pytest.approx(ref["ess"], rel=1e-2)


def test_c5_full_matches_oracle(ctx, refs):
    """S = 65536, T = 100, 32 obstacles: the whole update with the default
    launch shape (one lane per sample, normals drawn in the rollout), through
    the unfused reduction (64 groups x 300 rows)"""
    prob = W.config5()
    ctx.set_path(0, prob.path, prob.ds)
    log(f"  gpu solve c5 S={prob.S} T={prob.T} n_obs={prob.n_obs}")
    g = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(prob, controller=0), want_J=True)
    check_case("c5", prob, refs["c5"], g["U_new"], g["stats"], g["J"])


def test_c5_four_lanes_matches_oracle(ctx, refs):
    """the same update with four lanes per sample and the normals drawn ahead
    by the noise kernel (970 MB of them)"""
    prob = W.config5()
    ctx.set_path(1, prob.path, prob.ds)
    B.brmppi_set_launch(ctx.h, 256, 3)
    try:
        log("  gpu solve c5, block 256 variant 3")
        g = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(prob, controller=1), want_J=True)
    finally:
        B.brmppi_set_launch(ctx.h, 0, 0)
    check_case("c5 four lanes", prob, refs["c5"], g["U_new"], g["stats"], g["J"])


def test_served_mix_matches_oracle(ctx, refs):
    """eight requests of the served mix (S up to 32768, T up to 100, up to 32
    obstacles, moving ones among them) submitted together: each result against
    the oracle"""
    ctrl = W.config4_controllers()
    tickets = []
    for k, c in enumerate(REF.SERVED_CONTROLLERS):
        p = ctrl[c]
        ctx.set_path(10 + k, p.path, p.ds)
        log(f"  submit c4[{c}] S={p.S} T={p.T} n_obs={p.n_obs}")
        t, _ = B.brmppi_submit(ctx.h, B.ProblemBuffers(p, controller=10 + k))
        tickets.append(t)
    for k, c in enumerate(REF.SERVED_CONTROLLERS):
        p = ctrl[c]
        u, st, _ = B.brmppi_wait(ctx.h, tickets[k], p.T, timeout_ms=60000)
        check_case(f"c4[{c}]", p, refs[f"c4[{c}]"], u, st)


# The bound the normals test uses (1.5e-6) is composed from the maxima below:
# |d n| <= |d rad| + rad_max |d trig| + ulp(rad_max) / 2, rad_max = sqrt(-2 ln 2^-24) = 5.77
RAD_ERR = 4.9e-7
TRIG_ERR = 1.3e-7


def test_box_muller_every_uniform(ctx):
    """radius sqrt(-2 ln u) and cos / sin(2 pi u) of the kernels for all 2^23
    uniforms u = ((r >> 9) + 1/2) 2^-23, against FP64"""
    k = np.arange(1 << 23, dtype=np.uint64)
    r = (k << np.uint64(9)).astype(np.uint32)
    log("  box-muller over 2^23 uniforms")
    got = B.brmppi_debug_box_muller(ctx.h, r).astype(np.float64)
    u = (k.astype(np.float64) + 0.5) * 2.0 ** -23
    rad = np.sqrt(-2.0 * np.log(u))
    e_rad = np.abs(got[:, 0] - rad).max()
    e_cos = np.abs(got[:, 1] - np.cos(2 * np.pi * u)).max()
    e_sin = np.abs(got[:, 2] - np.sin(2 * np.pi * u)).max()
    log(f"  radius {e_rad:.3e}, cos {e_cos:.3e}, sin {e_sin:.3e}")
    assert e_rad <= RAD_ERR
    assert max(e_cos, e_sin) <= TRIG_ERR
    rad_max = float(rad.max())
    bound = RAD_ERR + rad_max * TRIG_ERR + np.spacing(np.float32(rad_max)) / 2
    from tests.test_gpu_parity import NORMAL_ATOL
    assert bound <= NORMAL_ATOL
