"""Thin ctypes binding of libbrmppi.so (include/brmppi.h).

The functions keep the C names and only marshal arguments; every step of the
control update runs in the library's HIP kernels.  PyTorch provides the device
arena and the HIP streams.  Importing this module does not need a GPU; opening
a context does, and fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbrmppi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "brmppi.h")

# return codes / flags (include/brmppi.h)
OK, PENDING = 0, 1
EINVAL, ENOMEM, EAGAIN, ENONFINITE, ENOTICKET, EDEVICE, ETIMEDOUT, ESTATE, ECANCELED = (
    -1, -2, -3, -4, -5, -6, -7, -8, -9)
GUIDANCE_OFF, HITCH_OFF, X0_RESIDENT, ADVANCE_PLANT, COLLISION_PENALTY, HITCH_QP = 1, 2, 4, 8, 16, 32
CTX_PROFILE, CTX_PROFILE_ROLLOUT = 1, 2
MAX_OBS, MAX_T = 32, 512

PARAM_FIELDS = (
    "Ts", "l1", "lh", "l2", "dtheta_max", "kappa", "r_disc",
    "Qc", "Ql", "Qth1", "Qth2", "R_j", "R_w", "mu", "nu_bar",
    "W_j", "W_w", "W_a", "rho", "j_lo", "j_hi", "w_lo", "w_hi",
    "alpha0", "alpha_lo", "alpha_hi", "sigma_j", "sigma_w", "sigma_nu", "sigma_a",
    "h_eps", "w_col", "qh_j", "qh_w", "alpha_h",
)


class BrmppiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"brmppi error {code}: {msg}")
        self.code = code


class brmppi_config(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("streams", C.c_void_p * 4),
                ("n_streams", C.c_uint32), ("max_controllers", C.c_uint32), ("max_inflight", C.c_uint32),
                ("autotune_cache", C.c_char_p), ("flags", C.c_uint32), ("device", C.c_int32)]


MAX_DISCS = 4


class brmppi_params(C.Structure):
    _fields_ = [(k, C.c_float) for k in PARAM_FIELDS] + [
        ("disc_tractor", C.c_float * MAX_DISCS), ("disc_trailer", C.c_float * MAX_DISCS),
        ("n_disc_tractor", C.c_uint32), ("n_disc_trailer", C.c_uint32)]


class brmppi_obstacle(C.Structure):
    _fields_ = [(k, C.c_float) for k in ("cx", "cy", "mx", "my", "heading", "e", "vx", "vy")]


class brmppi_problem(C.Structure):
    _fields_ = [("controller", C.c_uint32), ("S", C.c_uint32), ("T", C.c_uint32), ("x0", C.c_float * 8),
                ("u_nom", C.POINTER(C.c_float)), ("obs", C.POINTER(brmppi_obstacle)), ("n_obs", C.c_uint32),
                ("t0", C.c_float), ("lambda_", C.c_float), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("flags", C.c_uint32), ("params", C.POINTER(brmppi_params))]


class brmppi_stats(C.Structure):
    _fields_ = [("J_min", C.c_float), ("Z", C.c_float), ("ess", C.c_float), ("status", C.c_int32),
                ("latency_us", C.c_double)]


class brmppi_info(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("scratch_grows", "pinned_grows", "arena_bytes", "arena_used",
                                          "served_done", "served_failed")]


class brmppi_outputs(C.Structure):
    _fields_ = [("u_out", C.POINTER(C.c_float)), ("J_out", C.POINTER(C.c_float)),
                ("useq_out", C.POINTER(C.c_float))]


_lib = None


def declared_symbols() -> list:
    """Every function the header declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(brmppi_[a-z_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_05773_amd.build` "
                           "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    P, U32, U64, I, F, D, VP = C.POINTER, C.c_uint32, C.c_uint64, C.c_int, C.c_float, C.c_double, C.c_void_p
    ctx = VP
    sig = {
        "brmppi_create": (I, [P(brmppi_config), P(VP)]),
        "brmppi_destroy": (I, [ctx]),
        "brmppi_last_error": (C.c_char_p, []),
        "brmppi_set_path": (I, [ctx, U32, P(F), U32, F]),
        "brmppi_get_nominal": (I, [ctx, U32, P(F), U32]),
        "brmppi_set_nominal": (I, [ctx, U32, P(F), U32]),
        "brmppi_set_state": (I, [ctx, U32, P(D)]),
        "brmppi_get_state": (I, [ctx, U32, P(D)]),
        "brmppi_solve": (I, [ctx, P(brmppi_problem), P(F), P(brmppi_stats)]),
        "brmppi_solve_ex": (I, [ctx, P(brmppi_problem), P(brmppi_outputs), P(brmppi_stats)]),
        "brmppi_solve_noalloc": (I, [ctx, P(brmppi_problem), P(F), P(brmppi_stats)]),
        "brmppi_solve_batch": (I, [ctx, P(brmppi_problem), U32, P(P(F)), P(brmppi_stats)]),
        "brmppi_submit": (I, [ctx, P(brmppi_problem), P(U64)]),
        "brmppi_poll": (I, [ctx, U64, P(F), P(brmppi_stats)]),
        "brmppi_wait": (I, [ctx, U64, P(F), P(brmppi_stats), U32]),
        "brmppi_closed_loop": (I, [ctx, P(brmppi_problem), U32, P(D), P(F)]),
        "brmppi_autotune": (I, [ctx]),
        "brmppi_set_launch": (I, [ctx, U32, U32]),
        "brmppi_profile_read": (I, [ctx, P(D)]),
        "brmppi_profile_reset": (I, [ctx]),
        "brmppi_debug_philox": (I, [ctx, P(U32), P(U32), U32, P(U32)]),
        "brmppi_debug_normals": (I, [ctx, U64, U32, P(U32), U32, U32, P(F)]),
        "brmppi_debug_box_muller": (I, [ctx, P(U32), U32, P(F)]),
        "brmppi_get_info": (I, [ctx, P(brmppi_info)]),
        "brmppi_default_params": (I, [P(brmppi_params)]),
        "brmppi_set_params": (I, [ctx, U32, P(brmppi_params)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().brmppi_last_error().decode(errors="replace")


def check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise BrmppiError(rc, last_error())
    return rc


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def params_struct(p: dict) -> brmppi_params:
    P = brmppi_params(**{k: float(p[k]) for k in PARAM_FIELDS})
    dt, dr = list(p.get("disc_tractor", [0.0])), list(p.get("disc_trailer", []))
    if len(dt) > MAX_DISCS or len(dr) > MAX_DISCS:
        raise ValueError("at most 4 footprint discs per body")
    for i, v in enumerate(dt):
        P.disc_tractor[i] = float(v)
    for i, v in enumerate(dr):
        P.disc_trailer[i] = float(v)
    P.n_disc_tractor, P.n_disc_trailer = len(dt), len(dr)
    return P


class ProblemBuffers:
    """A brmppi_problem plus the host arrays it points to."""

    def __init__(self, prob, controller=None, with_nominal=True, flags=None, seed=None, x0=None,
                 with_params=True):
        self.params = params_struct(prob.params)
        obs = np.ascontiguousarray(np.asarray(prob.obstacles, dtype=np.float32).reshape(-1, 8))
        self.obs = (brmppi_obstacle * max(1, obs.shape[0]))(*[brmppi_obstacle(*map(float, o)) for o in obs])
        self.u_nom = np.ascontiguousarray(np.asarray(prob.u_nom, dtype=np.float32).reshape(-1))
        c = brmppi_problem()
        c.controller = int(prob.controller if controller is None else controller)
        c.S, c.T = int(prob.S), int(prob.T)
        xx = prob.x0 if x0 is None else x0
        for i in range(8):
            c.x0[i] = float(xx[i])
        if with_nominal and self.u_nom.size < 3 * c.T:
            raise ValueError(f"nominal sequence holds {self.u_nom.size} floats, the horizon needs {3 * c.T}")
        c.u_nom = _fp(self.u_nom) if with_nominal else None
        c.obs = self.obs
        c.n_obs = int(obs.shape[0])
        c.t0 = float(prob.t0)
        c.lambda_ = float(prob.lam)
        c.seed = int(prob.seed if seed is None else seed) & (2**64 - 1)
        c.instance = int(prob.instance) & 0xFFFFFFFF
        c.flags = int(prob.flags if flags is None else flags)
        c.params = C.pointer(self.params) if with_params else None
        self.c = c


# ---------------------------------------------------------------------------
# C-named wrappers (argument marshalling only)
# ---------------------------------------------------------------------------

def brmppi_create(cfg: brmppi_config):
    h = C.c_void_p()
    check(lib().brmppi_create(C.byref(cfg), C.byref(h)))
    return h


def brmppi_destroy(ctx):
    return check(lib().brmppi_destroy(ctx))


def brmppi_set_path(ctx, controller, path, ds):
    path = np.ascontiguousarray(np.asarray(path, dtype=np.float32).reshape(-1, 4))
    return check(lib().brmppi_set_path(ctx, int(controller), _fp(path), path.shape[0], float(ds)))


def brmppi_get_nominal(ctx, controller, T):
    u = np.zeros(3 * T, np.float32)
    check(lib().brmppi_get_nominal(ctx, int(controller), _fp(u), int(T)))
    return u.reshape(T, 3)


def brmppi_set_nominal(ctx, controller, u):
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float32).reshape(-1))
    return check(lib().brmppi_set_nominal(ctx, int(controller), _fp(u), u.size // 3))


def brmppi_set_state(ctx, controller, x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return check(lib().brmppi_set_state(ctx, int(controller), _dp(x)))


def brmppi_get_state(ctx, controller):
    x = np.zeros(8)
    check(lib().brmppi_get_state(ctx, int(controller), _dp(x)))
    return x


def _stats_dict(st: brmppi_stats) -> dict:
    return dict(J_min=st.J_min, Z=st.Z, ess=st.ess, status=st.status, latency_us=st.latency_us)


def brmppi_solve(ctx, pb: ProblemBuffers, allow=(OK,)):
    T = pb.c.T
    u = np.zeros(3 * T, np.float32)
    st = brmppi_stats()
    rc = check(lib().brmppi_solve(ctx, C.byref(pb.c), _fp(u), C.byref(st)), allow)
    return u.reshape(T, 3), _stats_dict(st), rc


def brmppi_solve_noalloc(ctx, pb: ProblemBuffers, allow=(OK,)):
    T = pb.c.T
    u = np.zeros(3 * T, np.float32)
    st = brmppi_stats()
    rc = check(lib().brmppi_solve_noalloc(ctx, C.byref(pb.c), _fp(u), C.byref(st)), allow)
    return u.reshape(T, 3), _stats_dict(st), rc


def brmppi_solve_ex(ctx, pb: ProblemBuffers, want_J=True, want_useq=False, allow=(OK,)):
    T, S = pb.c.T, pb.c.S
    u = np.zeros(3 * T, np.float32)
    J = np.zeros(S, np.float32) if want_J else None
    us = np.zeros(3 * T * S, np.float32) if want_useq else None
    out = brmppi_outputs(_fp(u), _fp(J) if J is not None else None, _fp(us) if us is not None else None)
    st = brmppi_stats()
    rc = check(lib().brmppi_solve_ex(ctx, C.byref(pb.c), C.byref(out), C.byref(st)), allow)
    res = dict(U_new=u.reshape(T, 3), stats=_stats_dict(st), rc=rc)
    if J is not None:
        res["J"] = J
    if us is not None:
        res["useq"] = us.reshape(T, 3, S)
    return res


class BatchBuffers:
    """The marshalled arguments of brmppi_solve_batch over a fixed list of
    problems, reusable across calls: the problem array (a copy of each
    ProblemBuffers' struct as it is now), one output buffer with a pointer per
    instance, and the stats array.  The results a call returns are views of
    the output buffer, which the next call with the same object overwrites."""

    def __init__(self, pbs: list):
        n = len(pbs)
        self.pbs = list(pbs)          # keeps the problems' host arrays alive
        self.n = n
        self.arr = (brmppi_problem * n)(*[pb.c for pb in pbs])
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum([3 * pb.c.T for pb in pbs])
        self.out = np.zeros(int(off[-1]), np.float32)
        base = self.out.ctypes.data
        self.ptrs = (C.POINTER(C.c_float) * n)(*[C.cast(base + 4 * int(o), C.POINTER(C.c_float)) for o in off[:-1]])
        self.st = (brmppi_stats * n)()
        self.views = [self.out[off[i]:off[i + 1]].reshape(-1, 3) for i in range(n)]


def brmppi_solve_batch(ctx, pbs, allow=(OK,)):
    """pbs: a list of ProblemBuffers (marshalled for this call) or a
    BatchBuffers (marshalled once, reused)."""
    bb = pbs if isinstance(pbs, BatchBuffers) else BatchBuffers(pbs)
    rc = check(lib().brmppi_solve_batch(ctx, bb.arr, bb.n, bb.ptrs, bb.st), allow)
    return bb.views, [_stats_dict(s) for s in bb.st], rc


def brmppi_submit(ctx, pb: ProblemBuffers, allow=(OK,)):
    t = C.c_uint64()
    rc = check(lib().brmppi_submit(ctx, C.byref(pb.c), C.byref(t)), allow)
    return t.value, rc


def brmppi_poll(ctx, ticket, T, allow=(OK, PENDING)):
    u = np.zeros(3 * T, np.float32)
    st = brmppi_stats()
    rc = check(lib().brmppi_poll(ctx, int(ticket), _fp(u), C.byref(st)), allow)
    return u.reshape(T, 3), _stats_dict(st), rc


def brmppi_wait(ctx, ticket, T, timeout_ms=60000, allow=(OK,)):
    u = np.zeros(3 * T, np.float32)
    st = brmppi_stats()
    rc = check(lib().brmppi_wait(ctx, int(ticket), _fp(u), C.byref(st), int(timeout_ms)), allow)
    return u.reshape(T, 3), _stats_dict(st), rc


def brmppi_closed_loop(ctx, pb: ProblemBuffers, n_updates, want_x=True, want_u=True):
    x = np.zeros(8 * (n_updates + 1)) if want_x else None
    u = np.zeros(3 * n_updates, np.float32) if want_u else None
    check(lib().brmppi_closed_loop(ctx, C.byref(pb.c), int(n_updates), _dp(x) if x is not None else None,
                                   _fp(u) if u is not None else None))
    return (x.reshape(-1, 8) if x is not None else None), (u.reshape(-1, 3) if u is not None else None)


def brmppi_autotune(ctx):
    return check(lib().brmppi_autotune(ctx))


def brmppi_set_launch(ctx, block, variant=0):
    """variant: 0 one lane per sample (in-kernel noise), 1 one lane (noise kernel),
    2 / 3 / 4 two / four / eight lanes per sample (noise kernel); block 0 = tuned default"""
    return check(lib().brmppi_set_launch(ctx, int(block), int(variant)))


def brmppi_profile_read(ctx):
    out = np.zeros(6)
    check(lib().brmppi_profile_read(ctx, _dp(out)))
    names = ("rollout", "reduce", "noise")
    return {n: dict(ms=out[2 * i], count=out[2 * i + 1]) for i, n in enumerate(names)}


def brmppi_profile_reset(ctx):
    return check(lib().brmppi_profile_reset(ctx))


def brmppi_debug_philox(ctx, ctr, key):
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    k = (C.c_uint32 * 2)(int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF)
    out = np.zeros_like(ctr)
    check(lib().brmppi_debug_philox(ctx, ctr.ctypes.data_as(C.POINTER(C.c_uint32)), k, ctr.shape[0],
                                    out.ctypes.data_as(C.POINTER(C.c_uint32))))
    return out


def brmppi_debug_normals(ctx, seed, instance, s_tau, K):
    s_tau = np.ascontiguousarray(np.asarray(s_tau, dtype=np.uint32).reshape(-1, 2))
    out = np.zeros((s_tau.shape[0], K), np.float32)
    check(lib().brmppi_debug_normals(ctx, int(seed) & (2**64 - 1), int(instance) & 0xFFFFFFFF,
                                     s_tau.ctypes.data_as(C.POINTER(C.c_uint32)), s_tau.shape[0], int(K),
                                     _fp(out)))
    return out


def brmppi_debug_box_muller(ctx, r):
    r = np.ascontiguousarray(np.asarray(r, dtype=np.uint32).reshape(-1))
    out = np.zeros((r.size, 3), np.float32)
    check(lib().brmppi_debug_box_muller(ctx, r.ctypes.data_as(C.POINTER(C.c_uint32)), r.size, _fp(out)))
    return out


def brmppi_get_info(ctx) -> dict:
    info = brmppi_info()
    check(lib().brmppi_get_info(ctx, C.byref(info)))
    return {k: int(getattr(info, k)) for k, _ in brmppi_info._fields_}


def brmppi_default_params() -> dict:
    p = brmppi_params()
    check(lib().brmppi_default_params(C.byref(p)))
    out = {k: float(getattr(p, k)) for k in PARAM_FIELDS}
    out["disc_tractor"] = [float(p.disc_tractor[i]) for i in range(p.n_disc_tractor)]
    out["disc_trailer"] = [float(p.disc_trailer[i]) for i in range(p.n_disc_trailer)]
    return out


def brmppi_set_params(ctx, controller, params):
    ps = params_struct(params) if params is not None else None
    return check(lib().brmppi_set_params(ctx, int(controller), C.byref(ps) if ps is not None else None))


# ---------------------------------------------------------------------------
# context over a torch-allocated arena and torch streams
# ---------------------------------------------------------------------------

class Context:
    """Owns a torch device arena and streams and the library context over them."""

    def __init__(self, arena_bytes=1 << 30, n_streams=2, max_controllers=512, profile=False,
                 autotune_cache=None, max_inflight=0, device=0, flags_extra=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
        lib()
        torch.cuda.set_device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        cfg = brmppi_config()
        cfg.arena = self.arena.data_ptr()
        cfg.arena_bytes = int(arena_bytes)
        for i, s in enumerate(self.streams):
            cfg.streams[i] = s.cuda_stream
        cfg.n_streams = n_streams
        cfg.max_controllers = max_controllers
        cfg.max_inflight = max_inflight
        self._tc = autotune_cache.encode() if autotune_cache else None
        cfg.autotune_cache = self._tc
        cfg.flags = (CTX_PROFILE if profile else 0) | int(flags_extra)
        cfg.device = device
        torch.cuda.synchronize()
        self.h = brmppi_create(cfg)
        self.paths = {}

    def set_path(self, controller, path, ds):
        brmppi_set_path(self.h, controller, path, ds)
        self.paths[controller] = (np.asarray(path, np.float32), float(ds))

    def close(self):
        if self.h is not None:
            brmppi_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
