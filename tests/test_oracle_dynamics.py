"""Pins for the oracle's tractor-trailer kinematics, eq. (6), and the rollout
loop with guidance reduced to the identity (no rows, rho = 0, no noise).

Closed forms (all exact for the explicit Euler recursion):
  straight line (delta = omega = 0, constant jerk):
    a_k = a0 + k Ts j,  v_k = v0 + k Ts a0 + Ts^2 j k(k-1)/2,
    p_k = p0 + e(th)(k Ts v0 + Ts^2 a0 k(k-1)/2 + Ts^3 j k(k-1)(k-2)/6)
  constant curvature (a = j = omega = 0, delta = d0):
    th_k = th0 + k D, D = Ts v0 tan(d0)/l1,
    p_k = p0 + Ts v0 sin(kD/2)/sin(D/2) e(th0 + (k-1) D/2)
  trailer fixed point on that arc: th1 - th2 = atan(B) + asin(C/sqrt(1+B^2)),
    B = (lh/l1) tan d0, C = (l2/l1) tan d0 (both headings then advance by D)
  trailer straightening (delta = 0): tan(phi/2) exp(s/l2) is constant in
    continuous time; Euler converges at first order.
"""
import math

import numpy as np
import pytest

from paper_2508_05773_amd import workloads as W


def _prm(Ts=0.1, **kw):
    return W.make_params(Ts, **kw)


def _iterate(orc, x, U, prm):
    xs = [np.array(x, dtype=np.float64)]
    for u in U:
        xs.append(orc.step(xs[-1], u, prm))
    return np.array(xs)


def test_straight_line_closed_form(orc):
    prm = _prm(0.1)
    Ts = prm["Ts"]
    th = 0.7
    x0 = np.array([1.0, -2.0, 0.5, 0.3, th, th, 0.0, 0.0])
    j = 0.4
    K = 25
    xs = _iterate(orc, x0, [[j, 0.0, 1.0]] * K, prm)
    e = np.array([math.cos(th), math.sin(th)])
    for k in range(K + 1):
        a = x0[3] + k * Ts * j
        v = x0[2] + k * Ts * x0[3] + Ts**2 * j * k * (k - 1) / 2
        s = k * Ts * x0[2] + Ts**2 * x0[3] * k * (k - 1) / 2 + Ts**3 * j * k * (k - 1) * (k - 2) / 6
        assert xs[k, 3] == pytest.approx(a, abs=1e-12)
        assert xs[k, 2] == pytest.approx(v, abs=1e-12)
        assert np.allclose(xs[k, :2], x0[:2] + s * e, atol=1e-12)
        assert xs[k, 4] == pytest.approx(th, abs=1e-14)
        assert xs[k, 5] == pytest.approx(th, abs=1e-14)   # aligned trailer stays aligned
        assert xs[k, 7] == pytest.approx(k * Ts * 1.0, abs=1e-12)


def test_constant_curvature_closed_form(orc):
    prm = _prm(0.05)
    Ts, l1 = prm["Ts"], prm["l1"]
    v0, d0, th0 = 1.3, 0.25, -0.4
    x0 = np.array([3.0, 4.0, v0, 0.0, th0, th0, d0, 0.0])
    K = 200
    xs = _iterate(orc, x0, [[0.0, 0.0, 0.0]] * K, prm)
    D = Ts * v0 * math.tan(d0) / l1
    R = Ts * v0 / (2 * math.sin(D / 2))
    for k in range(K + 1):
        assert xs[k, 4] == pytest.approx(th0 + k * D, abs=1e-11)
        if k == 0:
            continue
        amp = Ts * v0 * math.sin(k * D / 2) / math.sin(D / 2)
        ang = th0 + (k - 1) * D / 2
        assert np.allclose(xs[k, :2], x0[:2] + amp * np.array([math.cos(ang), math.sin(ang)]), atol=1e-10)
    # every point lies on one circle of radius Ts v0 / (2 sin(D/2)) -> l1/tan(d0)
    c = x0[:2] + R * np.array([-math.sin(th0 - D / 2), math.cos(th0 - D / 2)])
    r = np.hypot(xs[:, 0] - c[0], xs[:, 1] - c[1])
    assert np.allclose(r, R, atol=1e-9)
    assert R == pytest.approx(l1 / math.tan(d0), rel=1e-3)


def test_trailer_fixed_point(orc):
    prm = _prm(0.05)
    l1, lh, l2 = prm["l1"], prm["lh"], prm["l2"]
    v0, d0 = -0.8, 0.15          # reversing on an arc
    B = lh / l1 * math.tan(d0)
    Cc = l2 / l1 * math.tan(d0)
    phi = math.atan(B) + math.asin(Cc / math.sqrt(1 + B * B))
    th1 = 0.3
    x0 = np.array([0.0, 0.0, v0, 0.0, th1, th1 - phi, d0, 0.0])
    xs = _iterate(orc, x0, [[0.0, 0.0, 0.0]] * 300, prm)
    assert np.allclose(xs[:, 4] - xs[:, 5], phi, atol=1e-11)
    # a perturbed hitch angle does not stay put
    x1 = x0.copy()
    x1[5] -= 0.05
    ys = _iterate(orc, x1, [[0.0, 0.0, 0.0]] * 50, prm)
    assert abs((ys[-1, 4] - ys[-1, 5]) - (x1[4] - x1[5])) > 1e-3


def test_trailer_straightening_first_order(orc):
    errs = []
    for Ts in (0.02, 0.01, 0.005):
        prm = _prm(Ts)
        l2 = prm["l2"]
        v = 1.0
        phi0 = 0.6
        x0 = np.array([0.0, 0.0, v, 0.0, 0.0, -phi0, 0.0, 0.0])
        Tend = 4.0
        K = int(round(Tend / prm["Ts"]))
        xs = _iterate(orc, x0, [[0.0, 0.0, 0.0]] * K, prm)
        phi = xs[-1, 4] - xs[-1, 5]
        want = 2 * math.atan(math.tan(phi0 / 2) * math.exp(-v * K * prm["Ts"] / l2))
        errs.append(abs(phi - want))
    assert errs[0] < 2e-3
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4


def test_step_is_euler_of_drift(orc):
    rng = np.random.default_rng(3)
    prm = _prm(0.05)
    for _ in range(50):
        x = rng.normal(size=8)
        x[6] = rng.uniform(-0.5, 0.5)
        u = rng.normal(size=3)
        f = orc.drift(x, prm)
        g = np.zeros(8)
        g[3], g[6], g[7] = u
        assert np.allclose(orc.step(x, u, prm), x + prm["Ts"] * (f + g), atol=1e-13)


def test_identity_rollout_follows_nominal(orc):
    """No rows and rho = 0 make the projection the identity (Sec. IV-A); with
    zero noise the applied inputs are the nominal ones and the state follows
    the straight-line closed form."""
    prm = _prm(0.1, rho=0.0, sigma_j=0.0, sigma_w=0.0, sigma_nu=0.0, sigma_a=0.0)
    path, _ = W.path_c1()
    T = 12
    u_nom = np.tile(np.array([0.3, 0.0, 1.0], np.float32), (T, 1))
    x0 = np.array([0, 0, 0.5, 0.1, 0, 0, 0, 0], np.float32)
    p = W.Problem(S=1, T=T, x0=x0, u_nom=u_nom, obstacles=np.zeros((0, 8), np.float32),
                  path=path, ds=0.1, params=prm, flags=W.FLAG_HITCH_OFF)
    J, useq, traj, _ = orc.rollout(p, 0)
    assert np.allclose(useq, u_nom, atol=1e-15)
    Ts = prm["Ts"]
    v0, a0, j = float(x0[2]), float(x0[3]), float(u_nom[0, 0])
    for k in range(T + 1):
        s = k * Ts * v0 + Ts**2 * a0 * k * (k - 1) / 2 + Ts**3 * j * k * (k - 1) * (k - 2) / 6
        assert traj[k, 0] == pytest.approx(s, abs=1e-12)
    assert np.isfinite(J)


@pytest.mark.parametrize("j,w,nu,j_to,w_to", [
    (0.7, -0.4, 1.3, None, None),       # inside the box: applied as given
    (5.0, 0.2, 1.0, "hi", None),        # jerk above its bound
    (-3.5, 0.2, 1.0, "lo", None),       # jerk below its bound
    (1.5, 1.5, 1.0, None, "hi"),        # steer rate above its own bound; jerk 1.5 inside +-2 stays
    (-1.5, -1.2, 1.0, None, "lo"),      # steer rate below its bound
    (0.3, 0.1, 7.5, None, None),        # progress rate far above nu_bar: never clamped
    (0.3, 0.1, -4.0, None, None),       # negative progress rate: never clamped
])
def test_plant_step_clamps_each_input_to_its_own_bounds(orc, j, w, nu, j_to, w_to):
    """The closed-loop plant applies U_new[0] with jerk clamped to [j_lo, j_hi]
    and steer rate to [w_lo, w_hi] (the Sec. V bounds, which differ: +-2 and
    +-0.9), the progress rate as it is, and steps eq. (6).  The inputs enter the
    state only through a_{k+1} = a + Ts j, delta_{k+1} = delta + Ts omega and
    psi_{k+1} = psi + Ts nu (closed forms of the Euler map, checked directly),
    and the whole step equals the Euler step with the clamped input."""
    prm = _prm(0.05)
    ja = {None: j, "hi": prm["j_hi"], "lo": prm["j_lo"]}[j_to]
    wa = {None: w, "hi": prm["w_hi"], "lo": prm["w_lo"]}[w_to]
    x = np.array([3.0, -1.0, -1.2, 0.4, 0.3, 0.1, 0.05, 2.0])
    xn = orc.plant_step(x, [j, w, nu], prm)
    Ts = prm["Ts"]
    assert xn[3] == pytest.approx(x[3] + Ts * ja, rel=0, abs=1e-15)
    assert xn[6] == pytest.approx(x[6] + Ts * wa, rel=0, abs=1e-15)
    assert xn[7] == pytest.approx(x[7] + Ts * nu, rel=0, abs=1e-15)
    assert np.array_equal(xn, orc.step(x, [ja, wa, nu], prm))
