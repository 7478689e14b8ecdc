"""ctypes wrapper of the FP64 C oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this module.  The HIP product path never imports it.  See brmppi_oracle.c for
the method and the paper passages each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PARAM_FIELDS = (
    "Ts", "l1", "lh", "l2", "dtheta_max", "kappa", "r_disc",
    "Qc", "Ql", "Qth1", "Qth2", "R_j", "R_w", "mu", "nu_bar",
    "W_j", "W_w", "W_a", "rho", "j_lo", "j_hi", "w_lo", "w_hi",
    "alpha0", "alpha_lo", "alpha_hi", "sigma_j", "sigma_w", "sigma_nu", "sigma_a",
    "h_eps", "w_col", "qh_j", "qh_w", "alpha_h",
)

GUIDANCE_OFF = 1
HITCH_OFF = 2
COLLISION_PENALTY = 16
HITCH_QP = 32


class Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in PARAM_FIELDS] + [
        ("disc_tractor", C.c_double * 4), ("disc_trailer", C.c_double * 4),
        ("n_disc_tractor", C.c_int), ("n_disc_trailer", C.c_int)]


class Obstacle(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("cx", "cy", "mx", "my", "heading", "e", "vx", "vy")]


class ProblemC(C.Structure):
    _fields_ = [
        ("S", C.c_int), ("T", C.c_int), ("x0", C.c_double * 8),
        ("u_nom", C.POINTER(C.c_double)), ("obs", C.POINTER(Obstacle)), ("n_obs", C.c_int),
        ("path", C.POINTER(C.c_double)), ("n_path", C.c_int),
        ("ds", C.c_double), ("t0", C.c_double), ("lam", C.c_double),
        ("seed", C.c_uint64), ("instance", C.c_uint32), ("flags", C.c_int),
    ]


class Barrier(C.Structure):
    _fields_ = [("h", C.c_double), ("hd", C.c_double), ("hdd", C.c_double), ("hhat", C.c_double),
                ("grad", C.c_double * 8), ("dt", C.c_double)]


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "brmppi_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        D, P, U32, U64, I = C.c_double, C.POINTER(C.c_double), C.c_uint32, C.c_uint64, C.c_int
        L.orc_philox4x32_10.argtypes = [C.POINTER(U32), C.POINTER(U32), C.POINTER(U32)]
        L.orc_uniform23.argtypes = [U32]
        L.orc_uniform23.restype = D
        L.orc_normals.argtypes = [U64, U32, U32, U32, I, P]
        L.orc_drift.argtypes = [P, C.POINTER(Params), P]
        L.orc_step.argtypes = [P, P, C.POINTER(Params), P]
        L.orc_obstacle_barrier.argtypes = [P, D, C.POINTER(Obstacle), C.POINTER(Params), C.POINTER(Barrier)]
        L.orc_hitch_barrier.argtypes = [P, I, C.POINTER(Params), C.POINTER(Barrier)]
        L.orc_num_rows.argtypes = [C.POINTER(ProblemC), C.POINTER(Params)]
        L.orc_num_rows.restype = I
        L.orc_num_normals.argtypes = [C.POINTER(ProblemC), C.POINTER(Params)]
        L.orc_num_normals.restype = I
        L.orc_disc_barrier.argtypes = [P, D, C.POINTER(Obstacle), D, D, C.POINTER(Params), C.POINTER(Barrier)]
        L.orc_num_discs.argtypes = [C.POINTER(Params)]
        L.orc_num_discs.restype = I
        L.orc_disc.argtypes = [C.POINTER(Params), I, P, P]
        L.orc_rows.argtypes = [C.POINTER(ProblemC), C.POINTER(Params), P, D, P, P, P, P]
        L.orc_project.argtypes = [I, P, P, P, P, P, C.POINTER(Params), P]
        L.orc_project.restype = I
        L.orc_reference.argtypes = [P, I, D, D, P]
        L.orc_wrap.argtypes = [D]
        L.orc_wrap.restype = D
        L.orc_stage_cost.argtypes = [P, P, P, I, D, C.POINTER(Params)]
        L.orc_stage_cost.restype = D
        L.orc_terminal_cost.argtypes = [P, P, I, D, C.POINTER(Params)]
        L.orc_terminal_cost.restype = D
        L.orc_collision_penalty.argtypes = [P, D, C.POINTER(Obstacle), I, C.POINTER(Params)]
        L.orc_hitch_qp.argtypes = [P, P, C.POINTER(Params), P]
        L.orc_hitch_qp.restype = I
        L.orc_plant_step_qp.argtypes = [P, P, C.POINTER(Params), P]
        L.orc_collision_penalty.restype = D
        L.orc_rollout.argtypes = [C.POINTER(ProblemC), C.POINTER(Params), U32, P, P, P, P]
        L.orc_rollout.restype = D
        L.orc_rollout_samples.argtypes = [C.POINTER(ProblemC), C.POINTER(Params), C.POINTER(U32), I, I, P, P]
        L.orc_weights.argtypes = [P, I, D, P, P, P]
        L.orc_weights.restype = I
        L.orc_solve.argtypes = [C.POINTER(ProblemC), C.POINTER(Params), I, P, P, P, P, P, P]
        L.orc_solve.restype = I
        L.orc_plant_step.argtypes = [P, P, C.POINTER(Params), P]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def params_struct(p: dict) -> Params:
    P = Params(**{k: float(p[k]) for k in PARAM_FIELDS})
    dt, dr = list(p.get("disc_tractor", [0.0])), list(p.get("disc_trailer", []))
    assert len(dt) <= 4 and len(dr) <= 4
    for i, v in enumerate(dt):
        P.disc_tractor[i] = float(v)
    for i, v in enumerate(dr):
        P.disc_trailer[i] = float(v)
    P.n_disc_tractor, P.n_disc_trailer = len(dt), len(dr)
    return P


def obstacle_struct(o) -> Obstacle:
    return Obstacle(*[float(v) for v in o])


class OracleProblem:
    """Holds the C problem struct and keeps its arrays alive."""

    def __init__(self, prob, S=None, T=None, u_nom=None, x0=None, flags=None):
        self.T = int(T if T is not None else prob.T)
        self.S = int(S if S is not None else prob.S)
        u = prob.u_nom if u_nom is None else u_nom
        self.u_nom = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1)[: 3 * self.T])
        self.path = np.ascontiguousarray(np.asarray(prob.path, dtype=np.float64).reshape(-1))
        obs = np.asarray(prob.obstacles, dtype=np.float64).reshape(-1, 8)
        if obs.shape[0] and np.any((obs[:, 5] != 2.0) & (obs[:, 5] != 4.0)):
            raise ValueError("the oracle implements the e = 2 and e = 4 barriers only")
        self.obs = (Obstacle * max(1, obs.shape[0]))(*[obstacle_struct(o) for o in obs])
        self.params = params_struct(prob.params)
        xx = prob.x0 if x0 is None else x0
        self.c = ProblemC()
        self.c.S, self.c.T = self.S, self.T
        for i in range(8):
            self.c.x0[i] = float(xx[i])
        self.c.u_nom = _dp(self.u_nom)
        self.c.obs = self.obs
        self.c.n_obs = int(obs.shape[0])
        self.c.path = _dp(self.path)
        self.c.n_path = int(np.asarray(prob.path).shape[0])
        self.c.ds, self.c.t0, self.c.lam = float(prob.ds), float(prob.t0), float(prob.lam)
        self.c.seed, self.c.instance = int(prob.seed) & (2**64 - 1), int(prob.instance) & 0xFFFFFFFF
        self.c.flags = int(prob.flags if flags is None else flags)

    @property
    def n_c(self):
        return lib().orc_num_rows(C.byref(self.c), C.byref(self.params))

    @property
    def n_normals(self):
        return lib().orc_num_normals(C.byref(self.c), C.byref(self.params))


def solve(prob, nthreads=None, eps=None, want_useq=False, **kw):
    """Full update.  Returns dict(U_new (T,3), J (S,), wbar (S,), rc, stats, useq)."""
    op = OracleProblem(prob, **kw)
    S, T = op.S, op.T
    nthreads = nthreads or os.cpu_count() or 1
    U = np.zeros(3 * T)
    J = np.zeros(S)
    w = np.zeros(S)
    st = np.zeros(3)
    useq = np.zeros(S * T * 3) if want_useq else None
    ep = None
    if eps is not None:
        eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
        assert eps.size == S * T * op.n_normals
        ep = _dp(eps)
    rc = lib().orc_solve(C.byref(op.c), C.byref(op.params), int(nthreads), ep, _dp(U), _dp(J), _dp(w),
                         _dp(useq) if useq is not None else None, _dp(st))
    out = dict(U_new=U.reshape(T, 3), J=J, wbar=w, rc=rc,
               stats=dict(J_min=st[0], Z=st[1], ess=st[2]))
    if useq is not None:
        out["useq"] = useq.reshape(S, T, 3)
    return out


def rollout(prob, s, eps=None, **kw):
    """One sample: returns (J, useq (T,3), traj (T+1,8), alphas (T,nc))."""
    op = OracleProblem(prob, **kw)
    T, nc = op.T, op.n_c
    useq = np.zeros(3 * T)
    traj = np.zeros(8 * (T + 1))
    al = np.zeros(max(1, nc * T))
    ep = None
    if eps is not None:
        eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
        assert eps.size == T * op.n_normals
        ep = _dp(eps)
    J = lib().orc_rollout(C.byref(op.c), C.byref(op.params), int(s), ep, _dp(useq), _dp(traj), _dp(al))
    return J, useq.reshape(T, 3), traj.reshape(T + 1, 8), al[: nc * T].reshape(T, nc)


def rollout_samples(prob, ids, nthreads=None, want_useq=False, **kw):
    op = OracleProblem(prob, **kw)
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
    J = np.zeros(ids.size)
    useq = np.zeros(ids.size * op.T * 3) if want_useq else None
    lib().orc_rollout_samples(C.byref(op.c), C.byref(op.params),
                              ids.ctypes.data_as(C.POINTER(C.c_uint32)), int(ids.size),
                              int(nthreads or os.cpu_count() or 1), _dp(J),
                              _dp(useq) if useq is not None else None)
    if useq is not None:
        return J, useq.reshape(ids.size, op.T, 3)
    return J


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normals(seed, instance, s, tau, K):
    e = np.zeros(K)
    lib().orc_normals(int(seed) & (2**64 - 1), int(instance) & 0xFFFFFFFF, int(s), int(tau), int(K), _dp(e))
    return e


def uniform23(r):
    return lib().orc_uniform23(int(r) & 0xFFFFFFFF)


def step(x, u, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    xn = np.zeros(8)
    P = params_struct(params)
    lib().orc_step(_dp(x), _dp(u), C.byref(P), _dp(xn))
    return xn


def plant_step(x, U0, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    u = np.ascontiguousarray(np.asarray(U0, dtype=np.float64))
    xn = np.zeros(8)
    P = params_struct(params)
    lib().orc_plant_step(_dp(x), _dp(u), C.byref(P), _dp(xn))
    return xn


def drift(x, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    f = np.zeros(8)
    P = params_struct(params)
    lib().orc_drift(_dp(x), C.byref(P), _dp(f))
    return f


def obstacle_barrier(x, t, obs, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    B = Barrier()
    P = params_struct(params)
    O = obstacle_struct(obs)
    lib().orc_obstacle_barrier(_dp(x), float(t), C.byref(O), C.byref(P), C.byref(B))
    return dict(h=B.h, hd=B.hd, hdd=B.hdd, hhat=B.hhat, grad=np.array(B.grad[:]), dt=B.dt)


def disc_barrier(x, t, obs, A, B, params):
    """the obstacle barrier around the footprint disc centre p + A e1 - B f2"""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    Bo = Barrier()
    P = params_struct(params)
    O = obstacle_struct(obs)
    lib().orc_disc_barrier(_dp(x), float(t), C.byref(O), float(A), float(B), C.byref(P), C.byref(Bo))
    return dict(h=Bo.h, hd=Bo.hd, hdd=Bo.hdd, hhat=Bo.hhat, grad=np.array(Bo.grad[:]), dt=Bo.dt)


def discs(params):
    """(A, B) of every footprint disc in row order"""
    P = params_struct(params)
    out = []
    for k in range(lib().orc_num_discs(C.byref(P))):
        A, B = C.c_double(), C.c_double()
        lib().orc_disc(C.byref(P), k, C.byref(A), C.byref(B))
        out.append((A.value, B.value))
    return out


def hitch_barrier(x, sign, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    B = Barrier()
    P = params_struct(params)
    lib().orc_hitch_barrier(_dp(x), int(sign), C.byref(P), C.byref(B))
    return dict(h=B.h, hd=B.hd, hdd=B.hdd, hhat=B.hhat, grad=np.array(B.grad[:]), dt=B.dt)


def rows(prob, x, t, **kw):
    op = OracleProblem(prob, **kw)
    nc = op.n_c
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    hraw, hh, Lf = np.zeros(max(nc, 1)), np.zeros(max(nc, 1)), np.zeros(max(nc, 1))
    G = np.zeros(max(2 * nc, 1))
    lib().orc_rows(C.byref(op.c), C.byref(op.params), _dp(x), float(t), _dp(hraw), _dp(hh), _dp(G), _dp(Lf))
    return hraw[:nc], hh[:nc], G[: 2 * nc].reshape(nc, 2), Lf[:nc]


def project(zdes, alpha, hh, G, b, params):
    nc = len(hh)
    zdes = np.ascontiguousarray(np.asarray(zdes, dtype=np.float64))
    alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64).reshape(-1))
    hh = np.ascontiguousarray(np.asarray(hh, dtype=np.float64).reshape(-1))
    G = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(-1))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    z = np.zeros(2 + nc)
    P = params_struct(params)
    pad = lambda a: a if a.size else np.zeros(1)
    alpha, hh, G, b = pad(alpha), pad(hh), pad(G), pad(b)
    rc = lib().orc_project(nc, _dp(zdes), _dp(alpha), _dp(hh), _dp(G), _dp(b), C.byref(P), _dp(z))
    return z, rc


def reference(path, ds, psi):
    path = np.ascontiguousarray(np.asarray(path, dtype=np.float64).reshape(-1))
    ref = np.zeros(4)
    lib().orc_reference(_dp(path), path.size // 4, float(ds), float(psi), _dp(ref))
    return ref


def wrap(a):
    return lib().orc_wrap(float(a))


def stage_cost(x, u, path, ds, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    path = np.ascontiguousarray(np.asarray(path, dtype=np.float64).reshape(-1))
    P = params_struct(params)
    return lib().orc_stage_cost(_dp(x), _dp(u), _dp(path), path.size // 4, float(ds), C.byref(P))


def terminal_cost(x, path, ds, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    path = np.ascontiguousarray(np.asarray(path, dtype=np.float64).reshape(-1))
    P = params_struct(params)
    return lib().orc_terminal_cost(_dp(x), _dp(path), path.size // 4, float(ds), C.byref(P))


def collision_penalty(x, t, obstacles, params):
    """w_col * sum_o max(0, -h_o(x, t))^2 (the collision-penalty baseline)"""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    obs = np.ascontiguousarray(np.asarray(obstacles, dtype=np.float64).reshape(-1, 8))
    arr = (Obstacle * max(len(obs), 1))(*[obstacle_struct(o) for o in obs])
    P = params_struct(params)
    return lib().orc_collision_penalty(_dp(x), float(t), arr, len(obs), C.byref(P))


def hitch_qp(x, uref, params):
    """hitch-angle stabiliser (eq. (19)) at state x for the reference (j, omega):
    returns (u*, status) with status 1 when the constraints are infeasible"""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    ur = np.ascontiguousarray(np.asarray(uref, dtype=np.float64)[:2])
    out = np.zeros(2)
    P = params_struct(params)
    st = lib().orc_hitch_qp(_dp(x), _dp(ur), C.byref(P), _dp(out))
    return out, st


def plant_step_qp(x, U0, params):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    u = np.ascontiguousarray(np.asarray(U0, dtype=np.float64))
    xn = np.zeros(8)
    P = params_struct(params)
    lib().orc_plant_step_qp(_dp(x), _dp(u), C.byref(P), _dp(xn))
    return xn


def weights(J, lam):
    J = np.ascontiguousarray(np.asarray(J, dtype=np.float64))
    w = np.zeros(J.size)
    m, Z = C.c_double(), C.c_double()
    rc = lib().orc_weights(_dp(J), J.size, float(lam), _dp(w), C.byref(m), C.byref(Z))
    return w, m.value, Z.value, rc
