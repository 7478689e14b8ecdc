"""Pins for the oracle's barrier rows (eqs. (16)-(18), (9)).

1. The oracle's hhat, its state gradient and its time partial agree with an
   independent sympy derivation from the definitions (symbolic_ref.py).
2. Gradients agree with central finite differences of the oracle's own hhat.
3. hd and hdd are the time derivatives of h along the exact (fine-step RK4)
   flow of the drift, for static and moving obstacles.
4. The rows Lf, g and the h_eps guard match the definitions of eq. (9).
5. Footprint discs (Sec. IV-C): the barrier around a disc centre p + A e1 - B f2
   (tractor discs ahead of the rear axle, trailer discs behind the hitch)
   against the same sympy derivation with the centre substituted, central
   differences and the RK4 flow; the rear-axle disc (0, 0) is eq. (16) as
   printed, bit for bit; rows come disc by disc, obstacles in order, with one
   auxiliary normal each; the collision penalty sums every (disc, obstacle).
"""
import math

import numpy as np
import pytest

from paper_2508_05773_amd import workloads as W
from tests import symbolic_ref as SR


def _rand_state(rng):
    x = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-2, 2), rng.uniform(-1, 1),
                  rng.uniform(-3, 3), 0.0, rng.uniform(-0.5, 0.5), rng.uniform(0, 5)])
    x[5] = x[4] + rng.uniform(-0.6, 0.6)
    return x


def _rand_obs(rng, moving=True, e=2.0):
    return [rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.3, 2.5), rng.uniform(0.3, 2.5),
            rng.uniform(-math.pi, math.pi), e,
            rng.uniform(-1.5, 1.5) if moving else 0.0, rng.uniform(-1.5, 1.5) if moving else 0.0]


@pytest.mark.parametrize("e", [2, 4])
def test_obstacle_barrier_matches_symbolic(orc, e):
    F = SR.obstacle_funcs(exponent=e)
    rng = np.random.default_rng(0 + 10 * e)
    prm = W.make_params(0.05)
    for _ in range(60):
        x, o, tt = _rand_state(rng), _rand_obs(rng, e=float(e)), rng.uniform(0, 3)
        B = orc.obstacle_barrier(x, tt, o, prm)
        args = SR.obstacle_args(x, tt, prm, o)
        for k in ("h", "hd", "hdd", "hhat"):
            assert B[k] == pytest.approx(F[k](*args), rel=1e-11, abs=1e-11), k
        for i in range(8):
            assert B["grad"][i] == pytest.approx(F["grad"][i](*args), rel=1e-10, abs=1e-10), i
        assert B["dt"] == pytest.approx(F["dt"](*args), rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("sign", [1, -1])
def test_hitch_barrier_matches_symbolic(orc, sign):
    F = SR.hitch_funcs(sign)
    rng = np.random.default_rng(1)
    prm = W.make_params(0.1)
    for _ in range(60):
        x = _rand_state(rng)
        B = orc.hitch_barrier(x, sign, prm)
        args = SR.hitch_args(x, prm)
        for k in ("h", "hd", "hhat"):
            assert B[k] == pytest.approx(F[k](*args), rel=1e-12, abs=1e-12), k
        for i in range(8):
            assert B["grad"][i] == pytest.approx(F["grad"][i](*args), rel=1e-11, abs=1e-12), i
        assert B["dt"] == 0.0


@pytest.mark.parametrize("e", [2, 4])
def test_barrier_gradients_finite_difference(orc, e):
    rng = np.random.default_rng(2 + 10 * e)
    prm = W.make_params(0.05)
    eps = 1e-6
    for _ in range(40):
        x, o, tt = _rand_state(rng), _rand_obs(rng, e=float(e)), rng.uniform(0, 3)
        B = orc.obstacle_barrier(x, tt, o, prm)
        for i in range(8):
            xp, xm = x.copy(), x.copy()
            xp[i] += eps
            xm[i] -= eps
            fd = (orc.obstacle_barrier(xp, tt, o, prm)["hhat"] - orc.obstacle_barrier(xm, tt, o, prm)["hhat"]) / (2 * eps)
            assert B["grad"][i] == pytest.approx(fd, rel=1e-6, abs=1e-7), i
        fd = (orc.obstacle_barrier(x, tt + eps, o, prm)["hhat"] - orc.obstacle_barrier(x, tt - eps, o, prm)["hhat"]) / (2 * eps)
        assert B["dt"] == pytest.approx(fd, rel=1e-6, abs=1e-7)
        for sgn in (1, -1):
            H = orc.hitch_barrier(x, sgn, prm)
            for i in range(8):
                xp, xm = x.copy(), x.copy()
                xp[i] += eps
                xm[i] -= eps
                fd = (orc.hitch_barrier(xp, sgn, prm)["hhat"] - orc.hitch_barrier(xm, sgn, prm)["hhat"]) / (2 * eps)
                assert H["grad"][i] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def _rk4_flow(orc, x, prm, dt, n):
    """integrate the drift (inputs zero) with RK4; returns states at k*dt"""
    out = [x.copy()]
    for _ in range(n):
        k1 = orc.drift(x, prm)
        k2 = orc.drift(x + 0.5 * dt * k1, prm)
        k3 = orc.drift(x + 0.5 * dt * k2, prm)
        k4 = orc.drift(x + dt * k3, prm)
        x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        out.append(x.copy())
    return out


@pytest.mark.parametrize("moving,e", [(False, 2), (True, 2), (False, 4), (True, 4)])
def test_barrier_time_derivatives_along_flow(orc, moving, e):
    rng = np.random.default_rng(3 + moving + 10 * e)
    prm = W.make_params(0.05)
    dt = 1e-3
    for _ in range(10):
        x, o, t0 = _rand_state(rng), _rand_obs(rng, moving, e=float(e)), rng.uniform(0, 2)
        fwd = _rk4_flow(orc, x, prm, dt, 2)
        bwd = _rk4_flow(orc, x, prm, -dt, 2)
        hs = {}
        for k, xs in ((1, fwd[1]), (2, fwd[2]), (-1, bwd[1]), (-2, bwd[2]), (0, x)):
            hs[k] = orc.obstacle_barrier(xs, t0 + k * dt, o, prm)["h"]
        hd_fd = (-hs[2] + 8 * hs[1] - 8 * hs[-1] + hs[-2]) / (12 * dt)
        hdd_fd = (-hs[2] + 16 * hs[1] - 30 * hs[0] + 16 * hs[-1] - hs[-2]) / (12 * dt * dt)
        B = orc.obstacle_barrier(x, t0, o, prm)
        assert B["hd"] == pytest.approx(hd_fd, rel=1e-6, abs=1e-7)
        assert B["hdd"] == pytest.approx(hdd_fd, rel=1e-4, abs=1e-5)
        assert B["hhat"] == pytest.approx(B["h"] + prm["Ts"] * B["hd"] + 0.5 * prm["Ts"] ** 2 * B["hdd"], rel=1e-14)
        for sgn in (1, -1):
            hh = {k: orc.hitch_barrier(xs, sgn, prm)["h"] for k, xs in ((1, fwd[1]), (2, fwd[2]), (-1, bwd[1]), (-2, bwd[2]))}
            hd_fd = (-hh[2] + 8 * hh[1] - 8 * hh[-1] + hh[-2]) / (12 * dt)
            assert orc.hitch_barrier(x, sgn, prm)["hd"] == pytest.approx(hd_fd, rel=1e-6, abs=1e-8)


def test_rows_match_definition(orc):
    """Lf = Ts (L hhat), g = Ts (d hhat/da, d hhat/d delta), in the order
    hitch(+), hitch(-), obstacles; hh is hhat guarded by h_eps."""
    Fp, Fm = SR.hitch_funcs(1), SR.hitch_funcs(-1)
    rng = np.random.default_rng(5)
    prob = W.random_small(1, n_obs=4)
    obs = prob.obstacles.copy()
    obs[1::2, 5] = 4.0                        # mix e = 2 and e = 4 rows
    prob = prob.copy(obstacles=obs)
    prm = prob.params
    for _ in range(20):
        x, tt = _rand_state(rng), rng.uniform(0, 2)
        hraw, hh, G, Lf = orc.rows(prob, x, tt)
        assert len(hh) == prob.n_obs + 2
        for o_idx, o in enumerate(prob.obstacles):
            i = 2 + o_idx
            Fo = SR.obstacle_funcs(exponent=int(o[5]))
            args = SR.obstacle_args(x, tt, prm, o)
            assert hraw[i] == pytest.approx(Fo["hhat"](*args), rel=1e-11, abs=1e-12)
            assert Lf[i] == pytest.approx(Fo["Lf"](*args), rel=1e-10, abs=1e-11)
            assert G[i, 0] == pytest.approx(Fo["g0"](*args), rel=1e-10, abs=1e-13)
            assert G[i, 1] == pytest.approx(Fo["g1"](*args), rel=1e-10, abs=1e-13)
        for F, i in ((Fp, 0), (Fm, 1)):
            args = SR.hitch_args(x, prm)
            assert hraw[i] == pytest.approx(F["hhat"](*args), rel=1e-12, abs=1e-13)
            assert Lf[i] == pytest.approx(F["Lf"](*args), rel=1e-11, abs=1e-13)
            assert G[i, 0] == pytest.approx(F["g0"](*args), rel=1e-12, abs=1e-14)
            assert G[i, 1] == pytest.approx(F["g1"](*args), rel=1e-11, abs=1e-14)
        big = np.abs(hraw) >= prm["h_eps"]
        assert np.array_equal(hh[big], hraw[big])
    # hitch-off drops the two hitch rows
    hraw, hh, G, Lf = orc.rows(prob, _rand_state(rng), 0.0, flags=W.FLAG_HITCH_OFF)
    assert len(hh) == prob.n_obs


def test_h_eps_guard(orc):
    """hhat inside (-h_eps, h_eps) is pushed to +-h_eps, zero to +h_eps."""
    prm = W.make_params(0.05)
    prm["kappa"] = 0.0
    # hitch row: hhat = dth_max - (th2 - th1) + Ts*(...) ; at v = a = 0 this is dth_max - (th2-th1)
    x = np.zeros(8)
    prob = W.Problem(S=1, T=1, x0=x.astype(np.float32), u_nom=np.zeros((1, 3), np.float32),
                     obstacles=np.zeros((0, 8), np.float32), path=np.zeros((2, 4), np.float32),
                     ds=0.1, params=prm)
    dmax = prm["dtheta_max"]
    for off, want in ((0.0, prm["h_eps"]), (3e-6, prm["h_eps"]), (-3e-6, -prm["h_eps"]), (0.5, 0.5)):
        xx = x.copy()
        xx[5] = dmax - off        # h(+) = dmax - (th2 - th1) = off
        hraw, hh, _, _ = orc.rows(prob, xx, 0.0)
        assert hraw[0] == pytest.approx(off, abs=1e-15)
        assert hh[0] == pytest.approx(want, rel=1e-12, abs=1e-18)


def _rand_disc(rng, prm):
    """a tractor disc ahead of (or behind) the rear axle, or a trailer disc"""
    if rng.uniform() < 0.5:
        return rng.uniform(-1.0, 4.0), 0.0
    return -prm["lh"], rng.uniform(0.5, 9.0)


@pytest.mark.parametrize("e", [2, 4])
def test_disc_barrier_matches_symbolic(orc, e):
    F = SR.disc_funcs(exponent=e)
    rng = np.random.default_rng(20 + e)
    prm = W.make_params(0.05)
    for _ in range(40):
        x, o, tt = _rand_state(rng), _rand_obs(rng, e=float(e)), rng.uniform(0, 3)
        A, Bd = _rand_disc(rng, prm)
        D = orc.disc_barrier(x, tt, o, A, Bd, prm)
        args = SR.disc_args(x, tt, prm, o, A, Bd)
        for k in ("h", "hd", "hdd", "hhat"):
            assert D[k] == pytest.approx(F[k](*args), rel=1e-10, abs=1e-10), (k, A, Bd)
        for i in range(8):
            assert D["grad"][i] == pytest.approx(F["grad"][i](*args), rel=1e-9, abs=1e-9), (i, A, Bd)
        assert D["dt"] == pytest.approx(F["dt"](*args), rel=1e-9, abs=1e-9)


def test_rear_axle_disc_is_eq16(orc):
    rng = np.random.default_rng(31)
    prm = W.make_params(0.05)
    for e in (2, 4):
        for _ in range(20):
            x, o, tt = _rand_state(rng), _rand_obs(rng, e=float(e)), rng.uniform(0, 3)
            a, b = orc.obstacle_barrier(x, tt, o, prm), orc.disc_barrier(x, tt, o, 0.0, 0.0, prm)
            for k in ("h", "hd", "hdd", "hhat", "dt"):
                assert a[k] == b[k]
            assert np.array_equal(a["grad"], b["grad"])


@pytest.mark.parametrize("e", [2, 4])
def test_disc_gradients_finite_difference_and_flow(orc, e):
    rng = np.random.default_rng(40 + e)
    prm = W.make_params(0.05)
    eps, dt = 1e-6, 1e-3
    for _ in range(20):
        x, o, tt = _rand_state(rng), _rand_obs(rng, e=float(e)), rng.uniform(0, 3)
        A, Bd = _rand_disc(rng, prm)
        D = orc.disc_barrier(x, tt, o, A, Bd, prm)
        for i in range(8):
            xp, xm = x.copy(), x.copy()
            xp[i] += eps
            xm[i] -= eps
            fd = (orc.disc_barrier(xp, tt, o, A, Bd, prm)["hhat"] -
                  orc.disc_barrier(xm, tt, o, A, Bd, prm)["hhat"]) / (2 * eps)
            assert D["grad"][i] == pytest.approx(fd, rel=1e-6, abs=1e-7), i
        fwd = _rk4_flow(orc, x, prm, dt, 2)
        bwd = _rk4_flow(orc, x, prm, -dt, 2)
        hs = {k: orc.disc_barrier(xs, tt + k * dt, o, A, Bd, prm)["h"]
              for k, xs in ((1, fwd[1]), (2, fwd[2]), (-1, bwd[1]), (-2, bwd[2]), (0, x))}
        hd_fd = (-hs[2] + 8 * hs[1] - 8 * hs[-1] + hs[-2]) / (12 * dt)
        hdd_fd = (-hs[2] + 16 * hs[1] - 30 * hs[0] + 16 * hs[-1] - hs[-2]) / (12 * dt * dt)
        assert D["hd"] == pytest.approx(hd_fd, rel=1e-6, abs=1e-7)
        assert D["hdd"] == pytest.approx(hdd_fd, rel=1e-4, abs=1e-5)


def test_disc_rows_order_and_penalty(orc):
    """rows: hitch(+), hitch(-), then every (disc, obstacle), disc by disc;
    Lf and g of each against sympy at that disc; one normal per row; the
    collision penalty sums max(0, -h)^2 over every (disc, obstacle)"""
    F2, F4 = SR.disc_funcs(exponent=2), SR.disc_funcs(exponent=4)
    rng = np.random.default_rng(7)
    prm = W.make_params(0.05, disc_tractor=(0.0, 2.5), disc_trailer=(1.0, 6.0))
    prob = W.random_small(2, n_obs=3)
    obs = prob.obstacles.copy()
    obs[1, 5] = 4.0
    prob = prob.copy(obstacles=obs, params=prm)
    dl = orc.discs(prm)
    assert dl == [(0.0, 0.0), (2.5, 0.0), (-prm["lh"], 1.0), (-prm["lh"], 6.0)]
    op = orc.OracleProblem(prob)
    assert op.n_c == 2 + 4 * 3 and op.n_normals == 5 + 4 * 3
    for _ in range(10):
        x, tt = _rand_state(rng), rng.uniform(0, 2)
        hraw, hh, G, Lf = orc.rows(prob, x, tt)
        assert len(hh) == 14
        for k, (A, Bd) in enumerate(dl):
            for o_idx, o in enumerate(prob.obstacles):
                i = 2 + k * 3 + o_idx
                F = F4 if o[5] == 4.0 else F2
                args = SR.disc_args(x, tt, prm, o, A, Bd)
                assert hraw[i] == pytest.approx(F["hhat"](*args), rel=1e-10, abs=1e-11)
                assert Lf[i] == pytest.approx(F["Lf"](*args), rel=1e-9, abs=1e-10)
                assert G[i, 0] == pytest.approx(F["g0"](*args), rel=1e-9, abs=1e-12)
                assert G[i, 1] == pytest.approx(F["g1"](*args), rel=1e-9, abs=1e-12)
        pen = orc.collision_penalty(x, tt, prob.obstacles, prm)
        want = sum(min(0.0, orc.disc_barrier(x, tt, o, A, Bd, prm)["h"]) ** 2 for A, Bd in dl for o in prob.obstacles)
        assert pen == pytest.approx(prm["w_col"] * want, rel=1e-12, abs=1e-300)
