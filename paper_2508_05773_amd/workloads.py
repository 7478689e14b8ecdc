"""Seeded synthetic inputs for one BR-MPPI control update.

This module produces *inputs only* (reference paths, obstacles, initial states,
parameter sets, arrival processes).  It holds none of the method's arithmetic:
no dynamics, no barrier, no projection, no cost, no weights.  Both the HIP path
and the FP64 oracle consume what it returns.

The paper evaluates on a CarMaker parking lot with Hybrid A* reference paths and
hyper-parameters tuned by falsification (Sec. V); none of those are available, so
the workloads below stand in for them.  Paths are sampled every ``ds`` metres with
columns (x, y, theta1_ref, theta2_ref); on reverse segments the tractor heading
reference is the path tangent plus pi and the trailer reference equals the
tractor reference.

Obstacle record (8 float32): cx, cy, mx, my, heading, e, vx, vy  (Sec. IV-C,
super-ellipse centre, semi-axes, orientation, exponent; velocity for the
constant-velocity prediction of Assumption 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Parameter vector layout shared by the C-ABI struct (float32 fields, this order).
PARAM_FIELDS = (
    "Ts", "l1", "lh", "l2", "dtheta_max", "kappa", "r_disc",
    "Qc", "Ql", "Qth1", "Qth2", "R_j", "R_w", "mu", "nu_bar",
    "W_j", "W_w", "W_a", "rho", "j_lo", "j_hi", "w_lo", "w_hi",
    "alpha0", "alpha_lo", "alpha_hi", "sigma_j", "sigma_w", "sigma_nu", "sigma_a",
    "h_eps", "w_col", "qh_j", "qh_w", "alpha_h",
)

# flags (same bit values as the C-ABI header)
FLAG_GUIDANCE_OFF = 1   # plain MPPI: sampled inputs are applied unprojected
FLAG_HITCH_OFF = 2      # no hitch-angle rows
FLAG_COLLISION_PENALTY = 16  # baseline: w_col * sum_o max(0, -h_o)^2 added to the cost
FLAG_HITCH_QP = 32      # closed loop: hitch-angle stabiliser QP on the applied input


MAX_DISCS = 4   # footprint discs per body (tractor, trailer)


def make_params(Ts, sigma=(1.0, 0.3, 0.5), l1=4.0, lh=0.5, l2=10.0,
                dtheta_max=0.7, kappa=0.05, **over) -> dict:
    """Full explicit parameter set (float32-representable values).

    Values the paper fixes: input bounds j in [-2, 2] m/s^3 and omega in
    [-0.9, 0.9] rad/s (Sec. V).  Everything else was tuned by the authors and is
    unpublished; the stand-ins are: disc radius 1 m (half the 2 m tractor
    width), alpha0 = 0.5 with soft bounds [-1, 1], aux-input noise 0.2, the
    projection weight W equal to the inverse sampling covariance, rho = 0.1,
    contouring weights Qc = Ql = 2, heading weights 1, effort 0.05, progress
    weight 0.5 toward a maximum progress rate of 2 m/s.  The collision-penalty
    baseline (a flag) weighs max(0, -h_o)^2 by w_col = 1000, so that a sample
    reaching an obstacle's centre (h = -1) costs far more than any tracking
    error of the horizon.  The hitch-angle stabiliser QP weighs the deviation
    from the averaged input by the inverse sampling covariance (as W does) and
    uses the class-K rate alpha_h = 0.5.
    """
    sj, sw, sn = (float(s) for s in sigma)
    sa = 0.2
    p = dict(
        Ts=Ts, l1=l1, lh=lh, l2=l2, dtheta_max=dtheta_max, kappa=kappa, r_disc=1.0,
        Qc=2.0, Ql=2.0, Qth1=1.0, Qth2=1.0, R_j=0.05, R_w=0.05, mu=0.5, nu_bar=2.0,
        W_j=1.0 / sj ** 2, W_w=1.0 / sw ** 2, W_a=1.0 / sa ** 2, rho=0.1,
        j_lo=-2.0, j_hi=2.0, w_lo=-0.9, w_hi=0.9,
        alpha0=0.5, alpha_lo=-1.0, alpha_hi=1.0,
        sigma_j=sj, sigma_w=sw, sigma_nu=sn, sigma_a=sa, h_eps=1e-5, w_col=1000.0,
        qh_j=1.0 / sj ** 2, qh_w=1.0 / sw ** 2, alpha_h=0.5,
    )
    discs_t = over.pop("disc_tractor", (0.0,))
    discs_r = over.pop("disc_trailer", ())
    if not 1 <= len(discs_t) + len(discs_r) or len(discs_t) > MAX_DISCS or len(discs_r) > MAX_DISCS:
        raise ValueError("footprint: 1..8 discs, at most 4 on each body")
    p.update(over)
    # round every value to float32 so both sides see identical numbers
    out = {k: float(np.float32(p[k])) for k in PARAM_FIELDS}
    # footprint discs (Sec. IV-C): offsets ahead of the tractor's rear axle and
    # behind the hitch along the trailer; the default is the rear axle alone
    out["disc_tractor"] = [float(np.float32(v)) for v in discs_t]
    out["disc_trailer"] = [float(np.float32(v)) for v in discs_r]
    return out


def n_discs(params: dict) -> int:
    return len(params.get("disc_tractor", (0.0,))) + len(params.get("disc_trailer", ()))


def params_array(p: dict) -> np.ndarray:
    return np.array([p[k] for k in PARAM_FIELDS], dtype=np.float32)


# --------------------------------------------------------------------------
# reference paths
# --------------------------------------------------------------------------

def _segments_path(x0, y0, h0, segments, ds, reverse):
    """Sample a G1 path made of straights and circular arcs every ``ds`` metres.

    segments: list of ("line", length) or ("arc", radius, sweep_rad) in travel
    order, starting at (x0, y0) with travel tangent h0.
    """
    # closed-form position along each piece
    pieces = []
    x, y, h = x0, y0, h0
    for seg in segments:
        if seg[0] == "line":
            L = float(seg[1])
            pieces.append(("line", x, y, h, L))
            x, y = x + L * math.cos(h), y + L * math.sin(h)
        else:
            R, sweep = float(seg[1]), float(seg[2])
            L = abs(R * sweep)
            pieces.append(("arc", x, y, h, L, R, math.copysign(1.0, sweep)))
            k = math.copysign(1.0, sweep) / R
            h1 = h + k * L
            x, y = x + (math.sin(h1) - math.sin(h)) / k, y - (math.cos(h1) - math.cos(h)) / k
            h = h1
    total = sum(p[4] for p in pieces)
    n = int(math.floor(total / ds + 1e-9)) + 1
    out = np.zeros((n, 4), dtype=np.float64)
    starts = np.cumsum([0.0] + [p[4] for p in pieces])
    for i in range(n):
        s = i * ds
        j = min(int(np.searchsorted(starts, s, side="right")) - 1, len(pieces) - 1)
        pc = pieces[j]
        u = s - starts[j]
        if pc[0] == "line":
            _, px, py, ph, _ = pc
            out[i, 0], out[i, 1], th = px + u * math.cos(ph), py + u * math.sin(ph), ph
        else:
            _, px, py, ph, _, R, sg = pc
            k = sg / R
            th = ph + k * u
            out[i, 0] = px + (math.sin(th) - math.sin(ph)) / k
            out[i, 1] = py - (math.cos(th) - math.cos(ph)) / k
        out[i, 2] = th + (math.pi if reverse else 0.0)
    out[:, 3] = out[:, 2]
    return out.astype(np.float32), total


def path_c1(ds=0.1):
    """30 m straight along +x from the origin, then a left 90-degree arc, R = 15 m."""
    return _segments_path(0.0, 0.0, 0.0, [("line", 30.0), ("arc", 15.0, math.pi / 2)], ds, False)


def path_c2(ds=0.1):
    """Reverse S-curve into a 4 m bay: +45 deg arc (R 12), -45 deg arc (R 12), 20 m straight.

    Traversed in reverse (tractor heading reference = travel tangent + pi).  The
    bay is the final straight; its axis is the travel direction of that straight.
    """
    segs = [("arc", 12.0, math.pi / 4), ("arc", 12.0, -math.pi / 4), ("line", 20.0)]
    return _segments_path(0.0, 0.0, 0.0, segs, ds, True)


def random_segment_path(rng, ds=0.1):
    """2-4 pieces, each a straight U(5, 20) m or an arc with radius U(8, 25) m and
    sweep +-U(20, 90) degrees; forward or reverse with probability 1/2."""
    nseg = int(rng.integers(2, 5))
    segs = []
    for _ in range(nseg):
        if rng.random() < 0.5:
            segs.append(("line", float(rng.uniform(5.0, 20.0))))
        else:
            sweep = math.radians(float(rng.uniform(20.0, 90.0))) * (1 if rng.random() < 0.5 else -1)
            segs.append(("arc", float(rng.uniform(8.0, 25.0)), sweep))
    reverse = bool(rng.random() < 0.5)
    h0 = float(rng.uniform(-math.pi, math.pi))
    return _segments_path(0.0, 0.0, h0, segs, ds, reverse)


def path_c5(ds=0.1, n_points=2000):
    """Cubic-spline parking-lot route with two cusps (forward -> reverse -> forward).

    Three scipy CubicSpline pieces through hand-placed knots (12 knots in total),
    joined at the cusps so that the vehicle heading reference is continuous; the
    concatenation is resampled by arc length every ``ds`` and cut to n_points.
    """
    from scipy.interpolate import CubicSpline

    def spline_piece(knots, d0, d1, reverse):
        # d0, d1: unit travel directions at the ends (clamped boundary)
        k = np.asarray(knots, dtype=np.float64)
        t = np.concatenate([[0.0], np.cumsum(np.hypot(*np.diff(k, axis=0).T))])
        bx = ((1, d0[0]), (1, d1[0]))
        by = ((1, d0[1]), (1, d1[1]))
        cx, cy = CubicSpline(t, k[:, 0], bc_type=bx), CubicSpline(t, k[:, 1], bc_type=by)
        tt = np.linspace(0.0, t[-1], 20001)
        xs, ys = cx(tt), cy(tt)
        seg = np.hypot(np.diff(xs), np.diff(ys))
        arc = np.concatenate([[0.0], np.cumsum(seg)])
        return tt, arc, cx, cy, reverse

    def unit(x, y):
        n = math.hypot(x, y)
        return (x / n, y / n)

    a = unit(0.45, 0.9)    # travel direction entering the first cusp
    b = unit(-1.0, 0.0)    # travel direction entering the second cusp
    pieces = [
        spline_piece([(0, 0), (20, 1), (40, 6), (60, 16), (72, 30)], (1.0, 0.0), a, False),
        spline_piece([(72, 30), (66, 20), (56, 14), (44, 14)], (-a[0], -a[1]), b, True),
        spline_piece([(44, 14), (64, 12), (84, 6), (104, 0), (124, -2)], (-b[0], -b[1]),
                     unit(1.0, -0.1), False),
    ]
    total = sum(p[1][-1] for p in pieces)
    scale = (n_points * ds) / total * 1.001
    out = np.zeros((n_points, 4), dtype=np.float64)
    starts = np.concatenate([[0.0], np.cumsum([p[1][-1] * scale for p in pieces])])
    for i in range(n_points):
        s = i * ds
        j = min(int(np.searchsorted(starts, s, side="right")) - 1, len(pieces) - 1)
        tt, arc, cx, cy, rev = pieces[j]
        a = (s - starts[j]) / scale
        tp = float(np.interp(a, arc, tt))
        out[i, 0], out[i, 1] = scale * cx(tp), scale * cy(tp)
        dx, dy = cx(tp, 1), cy(tp, 1)
        th = math.atan2(dy, dx) + (math.pi if rev else 0.0)
        out[i, 2] = th
    # keep headings continuous (no 2*pi jumps) for readability of the table
    out[:, 2] = np.unwrap(out[:, 2])
    out[:, 3] = out[:, 2]
    return out.astype(np.float32), n_points * ds


# --------------------------------------------------------------------------
# obstacles
# --------------------------------------------------------------------------

def place_obstacles(rng, path, n, axes=(0.3, 1.0), offset=3.0, x0=None, r_disc=1.0,
                    moving_frac=0.0, speed=1.5):
    """Ellipses (e = 2) centred at a random path point plus a normal offset
    U(-offset, offset); semi-axes U(axes); heading U(-pi, pi).  A candidate whose
    centre is closer to the start position than its largest inflated semi-axis
    plus 0.5 m is redrawn (keeps the start outside every inflated obstacle)."""
    obs = np.zeros((n, 8), dtype=np.float32)
    npts = path.shape[0]
    for i in range(n):
        while True:
            k = int(rng.integers(0, npts))
            px, py, th = float(path[k, 0]), float(path[k, 1]), float(path[k, 2])
            off = float(rng.uniform(-offset, offset))
            cx, cy = px - off * math.sin(th), py + off * math.cos(th)
            mx, my = float(rng.uniform(*axes)), float(rng.uniform(*axes))
            hd = float(rng.uniform(-math.pi, math.pi))
            if x0 is not None:
                if math.hypot(cx - x0[0], cy - x0[1]) < max(mx, my) + r_disc + 0.5:
                    continue
            break
        vx = vy = 0.0
        if moving_frac > 0 and rng.random() < moving_frac:
            mh = float(rng.uniform(-math.pi, math.pi))
            vx, vy = speed * math.cos(mh), speed * math.sin(mh)
        obs[i] = (cx, cy, mx, my, hd, 2.0, vx, vy)
    return obs


def bay_obstacles(rng, path, bay_len=20.0, ds=0.1, jitter=0.5, jitter_h=0.2):
    """Eight parked-vehicle ellipses (2.5 x 1.0 m), four per bay edge at lateral
    +-3 m and 5 m spacing along the bay (the last ``bay_len`` metres of the path),
    with U(+-jitter) m position and U(+-jitter_h) rad heading jitter."""
    n = path.shape[0]
    k0 = n - 1 - int(round(bay_len / ds))
    bx, by = float(path[k0, 0]), float(path[k0, 1])
    ex, ey = float(path[-1, 0]), float(path[-1, 1])
    ax = math.atan2(ey - by, ex - bx)
    obs = []
    for side in (-1.0, 1.0):
        for j in range(4):
            along = 2.5 + 5.0 * j
            cx = bx + along * math.cos(ax) - side * 3.0 * math.sin(ax)
            cy = by + along * math.sin(ax) + side * 3.0 * math.cos(ax)
            cx += float(rng.uniform(-jitter, jitter))
            cy += float(rng.uniform(-jitter, jitter))
            hd = ax + float(rng.uniform(-jitter_h, jitter_h))
            obs.append((cx, cy, 2.5, 1.0, hd, 2.0, 0.0, 0.0))
    return np.asarray(obs, dtype=np.float32)


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------

@dataclass
class Problem:
    S: int
    T: int
    x0: np.ndarray            # (8,) float32: px, py, v, a, theta1, theta2, delta, psi
    u_nom: np.ndarray         # (T, 3) float32: jerk, steer rate, progress rate
    obstacles: np.ndarray     # (n_obs, 8) float32
    path: np.ndarray          # (n, 4) float32
    ds: float
    params: dict
    lam: float = 1.0
    seed: int = 0
    instance: int = 0
    t0: float = 0.0
    flags: int = 0
    controller: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_obs(self) -> int:
        return int(self.obstacles.shape[0])

    @property
    def n_c(self) -> int:
        hitch = 0 if (self.flags & FLAG_HITCH_OFF) else 2
        return self.n_obs + hitch

    def copy(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        for k in ("x0", "u_nom", "obstacles", "path"):
            d[k] = np.array(d[k], dtype=np.float32, copy=True)
        d["params"] = dict(d["params"])
        d["meta"] = dict(d["meta"])
        return Problem(**d)


def _start_state(path):
    x0 = np.zeros(8, dtype=np.float32)
    x0[0], x0[1] = path[0, 0], path[0, 1]
    x0[4], x0[5] = path[0, 2], path[0, 3]
    return x0


def config1() -> Problem:
    """Plain solve, S = 1024, T = 30, Ts = 0.1, two ellipses, at rest at the path start."""
    rng = np.random.default_rng(0)
    path, L = path_c1()
    x0 = _start_state(path)
    obs = place_obstacles(rng, path, 2, axes=(0.3, 1.0), x0=x0)
    T = 30
    return Problem(S=1024, T=T, x0=x0, u_nom=np.zeros((T, 3), np.float32), obstacles=obs,
                   path=path, ds=0.1, params=make_params(0.1), lam=1.0, seed=0, instance=0,
                   name="c1", meta={"L": L})


def config2(update: int = 0) -> Problem:
    """Reverse parking, S = 8192, T = 50, Ts = 0.05, eight parked-vehicle ellipses.

    ``update`` selects the seed of one closed-loop update (2000 + update); the
    closed loop itself (state and warm start) is driven by the caller.
    """
    rng = np.random.default_rng(2)
    path, L = path_c2()
    x0 = _start_state(path)
    obs = bay_obstacles(rng, path)
    T = 50
    return Problem(S=8192, T=T, x0=x0, u_nom=np.zeros((T, 3), np.float32), obstacles=obs,
                   path=path, ds=0.1, params=make_params(0.05), lam=1.0, seed=2000 + update,
                   instance=0, name="c2", meta={"L": L})


# Values the paper prints for its experiments (Sec. V and its table of parking
# results).  tests/test_paper_constants.py checks them against the cited
# fixture tests/golden/paper_sec5.json.
PAPER_VEHICLE = dict(l1=3.23, l2=2.9, lh=1.15)     # tractor wheelbase, trailer length, hitch length [m]
PAPER_HORIZON_STEPS = 120                          # H
PAPER_HORIZON_S = 4.8                              # H Ts [s]
PAPER_ROLLOUTS = 5000
PAPER_OBSTACLES = 8
PAPER_TIME_MS = {"forward": {"mppi": 3.20, "mppi_col": 13.00, "br_mppi": 9.92},
                 "backward": {"mppi": 3.00, "mppi_col": 14.00, "br_mppi": 9.75}}


def paper_shape(flags: int = 0) -> Problem:
    """The configuration of the paper's timing comparison (Sec. V): 5000
    rollouts over H = 120 steps of 0.04 s with the Sec. V vehicle and eight
    obstacles on the reverse-parking scene: seven parked vehicles as e = 4
    super-ellipses along the bay and a pedestrian (e = 2, a disc of 0.5 m)
    crossing the bay entrance at 1.2 m/s.  The footprint disc radius is half the
    2.5 m trailer width."""
    rng = np.random.default_rng(6)
    path, L = path_c2()
    x0 = _start_state(path)
    parked = bay_obstacles(rng, path)[:7].copy()
    parked[:, 5] = 4.0
    # the pedestrian starts 4 m to the side of the bay entrance and walks across it
    n = path.shape[0]
    k0 = n - 1 - int(round(20.0 / 0.1))
    tx, ty = float(path[k0 + 1, 0] - path[k0, 0]), float(path[k0 + 1, 1] - path[k0, 1])
    tn = math.hypot(tx, ty)
    nx, ny = -ty / tn, tx / tn
    ped = np.array([[path[k0, 0] - 4.0 * nx, path[k0, 1] - 4.0 * ny, 0.5, 0.5, 0.0, 2.0, 1.2 * nx, 1.2 * ny]],
                   dtype=np.float32)
    obs = np.vstack([parked, ped]).astype(np.float32)
    T = PAPER_HORIZON_STEPS
    params = make_params(PAPER_HORIZON_S / PAPER_HORIZON_STEPS, r_disc=1.25, **PAPER_VEHICLE)
    return Problem(S=PAPER_ROLLOUTS, T=T, x0=x0, u_nom=np.zeros((T, 3), np.float32), obstacles=obs,
                   path=path, ds=0.1, params=params, lam=1.0, seed=6, instance=0, flags=flags,
                   name="paper", meta={"L": L})


def config3(n_instances: int = 64, seed: int = 3) -> list:
    """64 uneven instances: S in {1024..16384}, T in [20, 80], 0-16 obstacles."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_instances):
        path, L = random_segment_path(rng)
        x0 = _start_state(path)
        S = int(rng.choice([1024, 2048, 4096, 8192, 16384]))
        T = int(rng.integers(20, 81))
        n_o = int(rng.integers(0, 17))
        obs = place_obstacles(rng, path, n_o, x0=x0)
        out.append(Problem(S=S, T=T, x0=x0, u_nom=np.zeros((T, 3), np.float32), obstacles=obs,
                           path=path, ds=0.1, params=make_params(0.05), lam=1.0,
                           seed=3000 + i, instance=i, controller=i, name=f"c3[{i}]",
                           meta={"L": L}))
    return out


def config4_controllers(n_ctrl: int = 256, seed: int = 4) -> list:
    """256 controllers: c3-style paths, S in {2048, 8192, 32768}, T in {30, 50, 100},
    0-32 obstacles of which 10 % move at 1.5 m/s."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_ctrl):
        path, L = random_segment_path(rng)
        x0 = _start_state(path)
        S = int(rng.choice([2048, 8192, 32768]))
        T = int(rng.choice([30, 50, 100]))
        n_o = int(rng.integers(0, 33))
        obs = place_obstacles(rng, path, n_o, x0=x0, moving_frac=0.1, speed=1.5)
        out.append(Problem(S=S, T=T, x0=x0, u_nom=np.zeros((T, 3), np.float32), obstacles=obs,
                           path=path, ds=0.1, params=make_params(0.05), lam=1.0,
                           seed=4000 + c, instance=c, controller=c, name=f"c4[{c}]",
                           meta={"L": L}))
    return out


def config4_arrivals(n_ctrl: int, duration_s: float, tick_s: float = 0.01,
                     jitter_mean_s: float = 0.001, seed: int = 44):
    """Arrival times: controller c submits at phase_c + k*tick + Exp(jitter_mean)."""
    rng = np.random.default_rng(seed)
    phase = rng.uniform(0.0, tick_s, size=n_ctrl)
    events = []
    k = 0
    while True:
        base = k * tick_s
        if base >= duration_s:
            break
        jit = rng.exponential(jitter_mean_s, size=n_ctrl)
        for c in range(n_ctrl):
            t = base + phase[c] + jit[c]
            if t < duration_s:
                events.append((t, c, k))
        k += 1
    events.sort()
    return events


def config5() -> Problem:
    """Large solve: S = 65536, T = 100, 32 ellipses with semi-axes U(0.3, 2.5)."""
    rng = np.random.default_rng(5)
    path, L = path_c5()
    x0 = _start_state(path)
    obs = place_obstacles(rng, path, 32, axes=(0.3, 2.5), x0=x0)
    T = 100
    return Problem(S=65536, T=T, x0=x0, u_nom=np.zeros((T, 3), np.float32), obstacles=obs,
                   path=path, ds=0.1, params=make_params(0.05), lam=1.0, seed=5, instance=0,
                   name="c5", meta={"L": L})


def random_small(seed: int, S=None, T=None, n_obs=None, moving=True) -> Problem:
    """Small random problem for parity sweeps (ragged S, odd T, mixed obstacles)."""
    rng = np.random.default_rng(10_000 + seed)
    path, L = random_segment_path(rng)
    x0 = _start_state(path)
    x0[2] = np.float32(rng.uniform(-1.0, 1.5))          # nonzero speed
    x0[3] = np.float32(rng.uniform(-0.5, 0.5))
    x0[6] = np.float32(rng.uniform(-0.2, 0.2))
    x0[5] = np.float32(x0[4] + rng.uniform(-0.2, 0.2))
    x0[7] = np.float32(rng.uniform(0.0, 2.0))
    S = int(S if S is not None else rng.integers(1, 3000))
    T = int(T if T is not None else rng.integers(1, 40))
    n_o = int(n_obs if n_obs is not None else rng.integers(0, 12))
    obs = place_obstacles(rng, path, n_o, x0=x0, moving_frac=0.3 if moving else 0.0)
    u_nom = (rng.standard_normal((T, 3)) * np.array([0.5, 0.1, 0.5]) + np.array([0, 0, 1.0])).astype(np.float32)
    return Problem(S=S, T=T, x0=x0, u_nom=u_nom, obstacles=obs, path=path, ds=0.1,
                   params=make_params(0.05), lam=float(np.float32(rng.uniform(0.3, 3.0))),
                   seed=int(rng.integers(0, 2**63)), instance=int(rng.integers(0, 2**31)),
                   t0=float(np.float32(rng.uniform(0, 2))), name=f"rand{seed}", meta={"L": L})
