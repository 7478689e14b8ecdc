"""Pins for the oracle's soft-bound projection, eqs. (10)-(12).

z* must be the minimiser of ||z - z_des||_W^2 + rho/2 (||z - lo||^2 + ||hi - z||^2)
subject to A z = b.  Checked by:
  - feasibility A z* = b and stationarity (M z* - p in range(A')),
  - no feasible perturbation (null space of A) lowers the objective,
  - an independent KKT solve (bordered system, numpy),
  - an independent O(nc) elimination of the auxiliary inputs,
  - textbook cases: one row with rho = 0 is the weighted hyperplane projection;
    no rows with rho = 0 and a feasible z_des are the identity; rho -> inf is
    the Euclidean projection of the box midpoint.
"""
import numpy as np
import pytest

from paper_2508_05773_amd import workloads as W


def _instance(rng, nc, prm):
    zdes = rng.normal(size=2 + nc) * np.r_[1.0, 0.3, np.full(nc, 0.2)]
    alpha = rng.uniform(-1, 1, size=nc)
    hh = rng.uniform(0.05, 3.0, size=nc) * rng.choice([-1, 1], size=nc)
    G = rng.normal(size=(nc, 2)) * 0.1
    b = rng.normal(size=nc)
    return zdes, alpha, hh, G, b


def _mats(zdes, alpha, hh, G, prm):
    nc = len(hh)
    Wd = np.r_[prm["W_j"], prm["W_w"], np.full(nc, prm["W_a"])]
    M = Wd + prm["rho"]
    lo = np.r_[prm["j_lo"], prm["w_lo"], prm["alpha_lo"] - alpha]
    hi = np.r_[prm["j_hi"], prm["w_hi"], prm["alpha_hi"] - alpha]
    A = np.zeros((nc, 2 + nc))
    A[:, :2] = G
    A[np.arange(nc), 2 + np.arange(nc)] = hh
    return Wd, M, lo, hi, A


def _objective(z, zdes, Wd, lo, hi, rho):
    return np.sum(Wd * (z - zdes) ** 2) + 0.5 * rho * (np.sum((z - lo) ** 2) + np.sum((hi - z) ** 2))


@pytest.mark.parametrize("nc", [0, 1, 2, 3, 6, 12])
def test_projection_kkt(orc, nc):
    rng = np.random.default_rng(nc)
    prm = W.make_params(0.05)
    for _ in range(20):
        zdes, alpha, hh, G, b = _instance(rng, nc, prm)
        z, rc = orc.project(zdes, alpha, hh, G, b, prm)
        assert rc == 0
        Wd, M, lo, hi, A = _mats(zdes, alpha, hh, G, prm)
        p = Wd * zdes + 0.5 * prm["rho"] * (lo + hi)
        if nc:
            assert np.allclose(A @ z, b, atol=1e-12 * (1 + np.abs(b).max()))
            # stationarity: M z - p = A' mu for some mu
            r = M * z - p
            mu, *_ = np.linalg.lstsq(A.T, r, rcond=None)
            assert np.allclose(A.T @ mu, r, atol=1e-11)
            # feasible perturbations never help
            _, _, Vt = np.linalg.svd(A)
            N = Vt[nc:].T
            f0 = _objective(z, zdes, Wd, lo, hi, prm["rho"])
            for _ in range(20):
                dz = N @ rng.normal(size=N.shape[1]) * 0.1
                assert _objective(z + dz, zdes, Wd, lo, hi, prm["rho"]) >= f0 - 1e-12
            # bordered KKT system: [2M A'; A 0][z; mu] = [2p; b]
            K = np.zeros((2 + 2 * nc, 2 + 2 * nc))
            K[: 2 + nc, : 2 + nc] = 2 * np.diag(M)
            K[: 2 + nc, 2 + nc:] = A.T
            K[2 + nc:, : 2 + nc] = A
            sol = np.linalg.solve(K, np.r_[2 * p, b])
            assert np.allclose(sol[: 2 + nc], z, atol=1e-11)
        else:
            assert np.allclose(z, p / M, atol=1e-15)


@pytest.mark.parametrize("nc", [1, 2, 5, 10, 34])
def test_projection_matches_elimination(orc, nc):
    """Independent O(nc) route: eliminate u^alpha_i = (b_i - g_i u)/hh_i and solve
    the 2x2 normal equations (M_u + sum c_i g_i g_i') u = p_u + sum c_i g_i r_i,
    c_i = M_a/hh_i^2, r_i = b_i - hh_i abar_i, abar = p_a/M_a."""
    rng = np.random.default_rng(100 + nc)
    prm = W.make_params(0.05)
    for _ in range(20):
        zdes, alpha, hh, G, b = _instance(rng, nc, prm)
        z, rc = orc.project(zdes, alpha, hh, G, b, prm)
        Wd, M, lo, hi, A = _mats(zdes, alpha, hh, G, prm)
        p = Wd * zdes + 0.5 * prm["rho"] * (lo + hi)
        Ma = M[2]
        abar = p[2:] / Ma
        c = Ma / hh ** 2
        rr = b - hh * abar
        N = np.diag(M[:2]) + (G.T * c) @ G
        y = p[:2] + G.T @ (c * rr)
        u = np.linalg.solve(N, y)
        aa = (b - G @ u) / hh
        assert np.allclose(z[:2], u, rtol=1e-11, atol=1e-12)
        assert np.allclose(z[2:], aa, rtol=1e-10, atol=1e-11)


def test_one_row_textbook(orc):
    """rho = 0, one row: z* = z_des - W^-1 a'(a z_des - b)/(a W^-1 a')."""
    rng = np.random.default_rng(7)
    prm = W.make_params(0.05, rho=0.0)
    for _ in range(20):
        zdes, alpha, hh, G, b = _instance(rng, 1, prm)
        z, _ = orc.project(zdes, alpha, hh, G, b, prm)
        Wd, M, lo, hi, A = _mats(zdes, alpha, hh, G, prm)
        a = A[0]
        want = zdes - (a / Wd) * (a @ zdes - b[0]) / (a @ (a / Wd))
        assert np.allclose(z, want, rtol=1e-12, atol=1e-13)


def test_identity_cases(orc):
    rng = np.random.default_rng(8)
    prm = W.make_params(0.05, rho=0.0)
    # no rows, rho = 0
    for _ in range(10):
        zdes = rng.normal(size=2)
        z, _ = orc.project(zdes, [], [], np.zeros((0, 2)), [], prm)
        assert np.allclose(z, zdes, rtol=1e-15, atol=0)
    # rho = 0 and z_des already on the constraint
    for nc in (1, 3, 8):
        zdes, alpha, hh, G, _ = _instance(rng, nc, prm)
        b = G @ zdes[:2] + hh * zdes[2:]
        z, _ = orc.project(zdes, alpha, hh, G, b, prm)
        assert np.allclose(z, zdes, rtol=1e-12, atol=1e-12)


def test_rho_large_is_midpoint_projection(orc):
    rng = np.random.default_rng(9)
    prm = W.make_params(0.05, rho=1e9)
    for nc in (1, 3):
        zdes, alpha, hh, G, b = _instance(rng, nc, prm)
        z, _ = orc.project(zdes, alpha, hh, G, b, prm)
        _, _, lo, hi, A = _mats(zdes, alpha, hh, G, prm)
        mid = 0.5 * (lo + hi)
        want = mid - A.T @ np.linalg.solve(A @ A.T, A @ mid - b)
        assert np.allclose(z, want, atol=1e-6)
