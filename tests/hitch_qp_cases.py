"""Hitch-angle stabiliser test cases shared by the oracle pins and the GPU
tests: the discrete CBF condition of the hitch rows by central differences
of the expanded barrier, and states where that condition binds."""
import numpy as np


def cbf_terms(orc, x, prm, sign, eps=1e-6):
    """hhat(x) and the directional derivative of hhat along Ts (f_c + g_c u) as
    d0 + d_j j + d_w w, by central differences (inputs enter as a_dot = j,
    delta_dot = w)"""
    hh = lambda y: orc.hitch_barrier(y, sign, prm)["hhat"]
    Ts = prm["Ts"]
    f = orc.drift(x, prm)
    def dd(direction):
        return (hh(x + eps * Ts * direction) - hh(x - eps * Ts * direction)) / (2 * eps)
    ej = np.zeros(8)
    ej[3] = 1.0
    ew = np.zeros(8)
    ew[6] = 1.0
    return hh(x), dd(f), dd(ej), dd(ew)


def binding_state(orc, prm, rng):
    """a reversing state and reference for which the reference violates one
    hitch row by 30 % of what the input box can change it in one step (the
    input's authority over hhat is O(Ts^2), so the hitch angle is scanned
    toward its limit until that holds)"""
    sgn = rng.choice([-1.0, 1.0])
    v, a, dl = rng.uniform(-1.2, -0.4), rng.uniform(-0.3, 0.3), sgn * rng.uniform(0.05, 0.3)
    uref = np.array([rng.uniform(-1, 1), sgn * rng.uniform(0.3, 0.9)])
    al = prm["alpha_h"]
    J, Wg = np.meshgrid(np.linspace(prm["j_lo"], prm["j_hi"], 41), np.linspace(prm["w_lo"], prm["w_hi"], 41))
    for phi in np.linspace(0.0, 1.2, 2401):
        x = np.array([0, 0, v, a, 0.3, 0.3 - sgn * phi, dl, 0])
        cons = [cbf_terms(orc, x, prm, s) for s in (1, -1)]
        for hh, d0, dj, dw in cons:
            ref = d0 + dj * uref[0] + dw * uref[1] + al * hh
            best = d0 + max(dj * prm["j_lo"], dj * prm["j_hi"]) + max(dw * prm["w_lo"], dw * prm["w_hi"]) + al * hh
            auth = best - ref
            if auth > 0 and ref < -0.3 * auth:
                # both rows together must leave part of the box feasible
                ok = np.ones_like(J, dtype=bool)
                for h2, e0, ej, ew in cons:
                    ok &= e0 + ej * J + ew * Wg + al * h2 >= 0
                if ok.any():
                    return x, uref
    raise AssertionError("no binding state found")
