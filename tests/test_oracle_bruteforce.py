"""End-to-end pin of the oracle: S = 4 samples, T = 3 steps, one moving
obstacle (ellipse e = 2 or super-ellipse e = 4) plus the two hitch rows, injected noise in {-1, 0, 1}, recomputed in
50-digit mpmath from the paper's equations:
  rows from the sympy derivation (symbolic_ref.py), eq. (9);
  the projection written literally as eq. (12) with mpmath matrices;
  Euler eq. (6); contouring cost eqs. (13)-(15); weights and eq. (5).
Every intermediate (applied inputs, states, costs, weights, update) must agree
with the FP64 oracle to 1e-12.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_2508_05773_amd import workloads as W
from tests import symbolic_ref as SR

mp.mp.dps = 50


def _wrap(a):
    two_pi = 2 * mp.pi
    return a - two_pi * mp.nint(a / two_pi)


def _ref(path, ds, psi):
    n = len(path)
    f = psi / ds
    i = int(mp.floor(f))
    i = max(0, min(i, n - 2))
    t = f - i
    t = min(max(t, mp.mpf(0)), mp.mpf(1))
    A, B = path[i], path[i + 1]
    return [A[0] + t * (B[0] - A[0]), A[1] + t * (B[1] - A[1]),
            A[2] + t * _wrap(B[2] - A[2]), A[3] + t * _wrap(B[3] - A[3])]


def _track(x, path, ds, P):
    xr, yr, t1, t2 = _ref(path, ds, x[7])
    ex, ey = x[0] - xr, x[1] - yr
    ec = mp.sin(t1) * ex - mp.cos(t1) * ey
    el = -mp.cos(t1) * ex - mp.sin(t1) * ey
    return P["Qc"] * ec**2 + P["Ql"] * el**2 + P["Qth1"] * _wrap(x[4] - t1)**2 + P["Qth2"] * _wrap(x[5] - t2)**2


def _euler(x, u, P):
    Ts = P["Ts"]
    px, py, v, a, t1, t2, dl, psi = x
    return [px + Ts * v * mp.cos(t1), py + Ts * v * mp.sin(t1), v + Ts * a, a + Ts * u[0],
            t1 + Ts * v / P["l1"] * mp.tan(dl),
            t2 + Ts * v / P["l2"] * (mp.sin(t1 - t2) - P["lh"] / P["l1"] * mp.cos(t1 - t2) * mp.tan(dl)),
            dl + Ts * u[1], psi + Ts * u[2]]


def _problem(e=2.0):
    prm = W.make_params(0.1)
    path, _ = W.path_c1()
    path = path[:120]
    x0 = np.array([0.3, 0.1, 1.2, 0.2, 0.05, 0.02, 0.04, 0.3], np.float32)
    obs = np.array([[4.5, 1.6, 0.8, 0.5, 0.3, e, -0.4, 0.2]], np.float32)
    T = 3
    u_nom = np.array([[0.2, 0.05, 1.0], [-0.1, 0.0, 1.2], [0.0, -0.05, 0.8]], np.float32)
    return W.Problem(S=4, T=T, x0=x0, u_nom=u_nom, obstacles=obs, path=path, ds=0.1, params=prm,
                     lam=0.7, seed=9, instance=1, t0=0.25)


@pytest.mark.parametrize("e", [2, 4])
def test_bruteforce_s4_t3(orc, e):
    p = _problem(float(e))
    P = {k: mp.mpf(v) for k, v in p.params.items() if not isinstance(v, list)}
    nc = p.n_obs + 2
    K = 5 + p.n_obs          # normals: 3 inputs, hitch(+), hitch(-), obstacle 0
    rng = np.random.default_rng(11)
    eps = rng.integers(-1, 2, size=(p.S, p.T, K)).astype(np.float64)
    path = [[mp.mpf(float(v)) for v in row] for row in p.path]
    ds = mp.mpf(p.ds)
    Fo = SR.obstacle_funcs("mpmath", exponent=e)
    Fh = {s: SR.hitch_funcs(s, "mpmath") for s in (1, -1)}
    sig = [P["sigma_j"], P["sigma_w"], P["sigma_nu"]]

    Js, U_all, X_all = [], [], []
    for s in range(p.S):
        x = [mp.mpf(float(v)) for v in p.x0]
        alpha = [P["alpha0"]] * nc
        J = mp.mpf(0)
        us, xs = [], [list(x)]
        for tau in range(p.T):
            tt = mp.mpf(p.t0) + tau * P["Ts"]
            e = [mp.mpf(v) for v in eps[s, tau]]
            u = [mp.mpf(float(p.u_nom[tau, k])) + sig[k] * e[k] for k in range(3)]
            at = [P["sigma_a"] * e[3 + i] for i in range(nc)]   # rows: hitch+, hitch-, obstacle
            # rows
            hh, G, Lf = [], [], []
            oargs = list(x) + [tt, P["Ts"], P["l1"], P["lh"], P["l2"], P["r_disc"]] + \
                [mp.mpf(float(v)) for v in (p.obstacles[0, 2], p.obstacles[0, 3], p.obstacles[0, 4],
                                            p.obstacles[0, 0], p.obstacles[0, 1], p.obstacles[0, 6],
                                            p.obstacles[0, 7])]
            hargs = list(x) + [P["Ts"], P["l1"], P["lh"], P["l2"], P["dtheta_max"], P["kappa"]]
            for F, args in ((Fh[1], hargs), (Fh[-1], hargs), (Fo, oargs)):
                hv = F["hhat"](*args)
                assert abs(hv) > 1e-3          # the h_eps guard is not exercised here
                hh.append(hv)
                G.append([F["g0"](*args), F["g1"](*args)])
                Lf.append(F["Lf"](*args))
            # eq. (12), literally
            nz = 2 + nc
            Wd = [P["W_j"], P["W_w"]] + [P["W_a"]] * nc
            lo = [P["j_lo"], P["w_lo"]] + [P["alpha_lo"] - alpha[i] for i in range(nc)]
            hi = [P["j_hi"], P["w_hi"]] + [P["alpha_hi"] - alpha[i] for i in range(nc)]
            zdes = [u[0], u[1]] + at
            Minv = mp.diag([1 / (Wd[k] + P["rho"]) for k in range(nz)])
            pv = mp.matrix([Wd[k] * zdes[k] + P["rho"] / 2 * (hi[k] + lo[k]) for k in range(nz)])
            A = mp.zeros(nc, nz)
            for i in range(nc):
                A[i, 0], A[i, 1], A[i, 2 + i] = G[i][0], G[i][1], hh[i]
            b = mp.matrix([-Lf[i] - alpha[i] * hh[i] for i in range(nc)])
            z = Minv * (pv - A.T * mp.lu_solve(A * Minv * A.T, A * Minv * pv - b))
            ustar = [z[0], z[1], u[2]]
            J += _track(x, path, ds, P) + P["R_j"] * ustar[0]**2 + P["R_w"] * ustar[1]**2 + \
                P["mu"] * (P["nu_bar"] - ustar[2])**2
            us.append(ustar)
            x = _euler(x, ustar, P)
            alpha = [alpha[i] + z[2 + i] for i in range(nc)]
            xs.append(list(x))
        J += _track(x, path, ds, P)
        Js.append(J)
        U_all.append(us)
        X_all.append(xs)

    lam = mp.mpf(p.lam)
    m = min(Js)
    g = [mp.e ** (-(J - m) / lam) for J in Js]
    Z = sum(g)
    wbar = [gi / Z for gi in g]
    U_new = [[sum(wbar[s] * U_all[s][tau][k] for s in range(p.S)) for k in range(3)] for tau in range(p.T)]

    res = orc.solve(p, nthreads=1, eps=eps.reshape(-1), want_useq=True)
    for s in range(p.S):
        assert res["J"][s] == pytest.approx(float(Js[s]), rel=1e-12)
        assert np.allclose(res["useq"][s], np.array(U_all[s], dtype=float), rtol=1e-12, atol=1e-13)
        _, _, traj, _ = orc.rollout(p, s, eps=eps[s].reshape(-1))
        assert np.allclose(traj, np.array(X_all[s], dtype=float), rtol=1e-12, atol=1e-13)
    assert np.allclose(res["wbar"], np.array(wbar, dtype=float), rtol=1e-11, atol=1e-14)
    assert np.allclose(res["U_new"], np.array(U_new, dtype=float), rtol=1e-11, atol=1e-13)
    # the injected noise actually made the samples differ and the rows mattered
    assert float(max(Js) - min(Js)) > 1e-3
    assert not np.allclose(res["useq"][0, :, :2], p.u_nom[:, :2] + eps[0, :, :2] * [p.params["sigma_j"], p.params["sigma_w"]])
