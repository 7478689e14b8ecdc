"""Pins for the hitch-angle stabiliser of Sec. IV-D (eq. (19)).

The oracle solves the 2-variable CBF-QP by enumerating active sets (KKT).  It
is pinned here without its own row algebra: the discrete CBF condition is
evaluated as the central finite difference of the expanded hitch barrier
hhat = h + Ts hdot (the barrier function is pinned in test_oracle_barrier)
along the Euler increment Ts (f_c(x) + g_c u), which is linear in u, and the
optimum is checked against a brute-force grid search of the input box.
"""
import numpy as np
import pytest

from paper_2508_05773_amd import workloads as W
from tests.hitch_qp_cases import binding_state, cbf_terms


def _prm(**kw):
    return W.make_params(0.05, **kw)


def _check_solution(orc, x, uref, prm, tol_fd=1e-6):
    u, st = orc.hitch_qp(x, uref, prm)
    assert st == 0
    assert prm["j_lo"] - 1e-12 <= u[0] <= prm["j_hi"] + 1e-12
    assert prm["w_lo"] - 1e-12 <= u[1] <= prm["w_hi"] + 1e-12
    cons = [cbf_terms(orc, x, prm, s) for s in (1, -1)]
    a = prm["alpha_h"]
    for hh, d0, dj, dw in cons:
        assert d0 + dj * u[0] + dw * u[1] >= -a * hh - tol_fd
    # brute force over the input box: no feasible grid point beats u*
    q = np.array([prm["qh_j"], prm["qh_w"]])
    J, Wg = np.meshgrid(np.linspace(prm["j_lo"], prm["j_hi"], 801), np.linspace(prm["w_lo"], prm["w_hi"], 801))
    ok = np.ones_like(J, dtype=bool)
    for hh, d0, dj, dw in cons:
        ok &= d0 + dj * J + dw * Wg >= -a * hh + 1e-9
    obj = q[0] * (J - uref[0]) ** 2 + q[1] * (Wg - uref[1]) ** 2
    best = obj[ok].min() if ok.any() else np.inf
    ours = q[0] * (u[0] - uref[0]) ** 2 + q[1] * (u[1] - uref[1]) ** 2
    assert ours <= best + 1e-9
    # and the grid comes within its resolution of u*
    if ok.any():
        assert best <= ours + 0.02 * (1 + ours)
    return u, cons


def test_feasible_reference_is_returned(orc):
    prm = _prm()
    x = np.array([0, 0, 0.5, 0.0, 0.2, 0.15, 0.05, 0])
    for uref in ([0.3, -0.1], [-1.5, 0.6], [0.0, 0.0]):
        u, st = orc.hitch_qp(x, uref, prm)
        assert st == 0 and np.array_equal(u, np.array(uref, dtype=np.float64))


def test_reference_outside_box_is_projected(orc):
    """with the hitch rows slack, the weighted projection onto the box is the
    clip of each coordinate"""
    prm = _prm()
    x = np.array([0, 0, 0.5, 0.0, 0.2, 0.15, 0.05, 0])
    u, st = orc.hitch_qp(x, [3.5, -1.4], prm)
    assert st == 0
    assert u == pytest.approx([prm["j_hi"], prm["w_lo"]], abs=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_binding_hitch_rows(orc, seed):
    """the reference violates a hitch row that the box can satisfy: u* moves
    onto the row (equality) and is the optimum of the box-constrained problem"""
    prm = _prm(dtheta_max=0.35)
    x, uref = binding_state(orc, prm, np.random.default_rng(seed))
    u, cons = _check_solution(orc, x, uref, prm)
    a = prm["alpha_h"]
    slack = [d0 + dj * u[0] + dw * u[1] + a * hh for hh, d0, dj, dw in cons]
    assert not np.allclose(u, uref)
    assert min(slack) == pytest.approx(0.0, abs=1e-7)


@pytest.mark.parametrize("seed", range(6))
def test_random_states(orc, seed):
    rng = np.random.default_rng(100 + seed)
    prm = _prm()
    x = np.array([rng.normal(), rng.normal(), rng.uniform(-1.5, 1.5), rng.uniform(-0.5, 0.5),
                  rng.uniform(-1, 1), 0.0, rng.uniform(-0.4, 0.4), 0])
    x[5] = x[4] - rng.uniform(-0.6, 0.6)
    uref = np.array([rng.uniform(-3, 3), rng.uniform(-1.2, 1.2)])
    u, st = orc.hitch_qp(x, uref, prm)
    if st == 0:
        _check_solution(orc, x, uref, prm)


def test_infeasible_returns_clipped_reference(orc):
    """hitch angle far beyond its limit and opening fast: no input in the box
    satisfies the condition; the clipped reference is returned with status 1"""
    prm = _prm(dtheta_max=0.1)
    x = np.array([0, 0, -2.0, -1.0, 0.0, -1.2, 0.4, 0])
    cons = [cbf_terms(orc, x, prm, s) for s in (1, -1)]
    # confirm infeasibility on a grid
    J, Wg = np.meshgrid(np.linspace(prm["j_lo"], prm["j_hi"], 201), np.linspace(prm["w_lo"], prm["w_hi"], 201))
    ok = np.ones_like(J, dtype=bool)
    for hh, d0, dj, dw in cons:
        ok &= d0 + dj * J + dw * Wg >= -prm["alpha_h"] * hh - 1e-9
    assert not ok.any()
    u, st = orc.hitch_qp(x, [3.0, 0.2], prm)
    assert st == 1
    assert u == pytest.approx([prm["j_hi"], 0.2], abs=0)


def test_plant_step_qp(orc):
    """the stabilised plant step applies u* (and the unprojected progress rate)"""
    prm = _prm(dtheta_max=0.35)
    x, uref = binding_state(orc, prm, np.random.default_rng(3))
    U0 = np.array([uref[0], uref[1], 1.3])
    u, st = orc.hitch_qp(x, U0[:2], prm)
    assert st == 0 and not np.allclose(u, U0[:2])
    xn = orc.plant_step_qp(x, U0, prm)
    assert np.array_equal(xn, orc.step(x, np.array([u[0], u[1], U0[2]]), prm))
