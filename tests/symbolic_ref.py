"""Independent symbolic derivation (sympy) of the barriers and their Lie
derivatives, used to pin the oracle's hand-written chain rule.

Everything here is derived mechanically from the definitions in the paper:
  - drift f_c and input columns g_c from eq. (6) (continuous time, psi_dot = nu),
  - the super-ellipse barrier eq. (16) (exponent e = 2 or 4) around a
    constant-velocity obstacle, at the rear axle or at a footprint disc centre
    p + A e1 - B f2 (Sec. IV-C),
  - hhat = h + Ts L h + Ts^2/2 L^2 h  (eq. (17)), L the Lie derivative along f_c
    plus the explicit time derivative,
  - the hitch barrier eq. (18) split in two smooth rows, hhat = h + Ts L h,
  - rows Lf = Ts L hhat, g = Ts (d hhat/da, d hhat/d delta) (f = Ts f_c, g = Ts g_c).
sympy differentiates; nothing here is copied from the oracle.
"""
import functools

import sympy as sp

X = sp.symbols("px py v a th1 th2 dl psi", real=True)
px, py, v, a, th1, th2, dl, psi = X
t = sp.Symbol("t", real=True)
Ts, l1, lh, l2, r = sp.symbols("Ts l1 lh l2 r", positive=True)
mx, my, tho, cx, cy, vx, vy = sp.symbols("mx my tho cx cy vx vy", real=True)
dthmax, kappa = sp.symbols("dthmax kappa", real=True)

FC = [v * sp.cos(th1), v * sp.sin(th1), a, 0, v / l1 * sp.tan(dl),
      v / l2 * (sp.sin(th1 - th2) - lh / l1 * sp.cos(th1 - th2) * sp.tan(dl)), 0, 0]


def lie(F):
    return sum(sp.diff(F, X[i]) * FC[i] for i in range(8)) + sp.diff(F, t)


DA, DB = sp.symbols("DA DB", real=True)


@functools.lru_cache(maxsize=None)
def obstacle_exprs(e=2, disc=False):
    # disc: the barrier around a footprint disc centre p + DA e1 - DB f2
    # (e1, f2 the tractor and trailer heading vectors); otherwise the rear axle
    cpx = px + DA * sp.cos(th1) - DB * sp.cos(th2) if disc else px
    cpy = py + DA * sp.sin(th1) - DB * sp.sin(th2) if disc else py
    dx = cpx - (cx + vx * t)
    dy = cpy - (cy + vy * t)
    xp = sp.cos(tho) * dx + sp.sin(tho) * dy
    yp = -sp.sin(tho) * dx + sp.cos(tho) * dy
    h = (xp / (mx + r)) ** e + (yp / (my + r)) ** e - 1
    hd = lie(h)
    hdd = lie(hd)
    hhat = h + Ts * hd + Ts ** 2 / 2 * hdd
    Lf = Ts * lie(hhat)
    g = [Ts * sp.diff(hhat, a), Ts * sp.diff(hhat, dl)]
    grad = [sp.diff(hhat, xi) for xi in X]
    dt = sp.diff(hhat, t)
    return dict(h=h, hd=hd, hdd=hdd, hhat=hhat, Lf=Lf, g0=g[0], g1=g[1], grad=grad, dt=dt)


@functools.lru_cache(maxsize=None)
def hitch_exprs(sign):
    h = dthmax - kappa * v - sign * (th2 - th1)
    hd = lie(h)
    hhat = h + Ts * hd
    Lf = Ts * lie(hhat)
    g = [Ts * sp.diff(hhat, a), Ts * sp.diff(hhat, dl)]
    grad = [sp.diff(hhat, xi) for xi in X]
    return dict(h=h, hd=hd, hhat=hhat, Lf=Lf, g0=g[0], g1=g[1], grad=grad)


OBS_ARGS = list(X) + [t, Ts, l1, lh, l2, r, mx, my, tho, cx, cy, vx, vy]
DISC_ARGS = OBS_ARGS + [DA, DB]
HITCH_ARGS = list(X) + [Ts, l1, lh, l2, dthmax, kappa]


@functools.lru_cache(maxsize=None)
def obstacle_funcs(module="numpy", exponent=2):
    e = obstacle_exprs(exponent)
    out = {}
    for k in ("h", "hd", "hdd", "hhat", "Lf", "g0", "g1", "dt"):
        out[k] = sp.lambdify(OBS_ARGS, e[k], module)
    out["grad"] = [sp.lambdify(OBS_ARGS, gi, module) for gi in e["grad"]]
    return out


@functools.lru_cache(maxsize=None)
def disc_funcs(module="numpy", exponent=2):
    e = obstacle_exprs(exponent, disc=True)
    out = {}
    for k in ("h", "hd", "hdd", "hhat", "Lf", "g0", "g1", "dt"):
        out[k] = sp.lambdify(DISC_ARGS, e[k], module)
    out["grad"] = [sp.lambdify(DISC_ARGS, gi, module) for gi in e["grad"]]
    return out


@functools.lru_cache(maxsize=None)
def hitch_funcs(sign, module="numpy"):
    e = hitch_exprs(sign)
    out = {}
    for k in ("h", "hd", "hhat", "Lf", "g0", "g1"):
        out[k] = sp.lambdify(HITCH_ARGS, e[k], module)
    out["grad"] = [sp.lambdify(HITCH_ARGS, gi, module) for gi in e["grad"]]
    return out


def obstacle_args(x, tt, prm, obs):
    cx_, cy_, mx_, my_, th_, _e, vx_, vy_ = [float(q) for q in obs]
    return list(x) + [tt, prm["Ts"], prm["l1"], prm["lh"], prm["l2"], prm["r_disc"],
                      mx_, my_, th_, cx_, cy_, vx_, vy_]


def disc_args(x, tt, prm, obs, A, B):
    return obstacle_args(x, tt, prm, obs) + [A, B]


def hitch_args(x, prm):
    return list(x) + [prm["Ts"], prm["l1"], prm["lh"], prm["l2"], prm["dtheta_max"], prm["kappa"]]
