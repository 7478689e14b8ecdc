"""GPU tests of the batched, served and closed-loop forms.

- batched (persistent kernels in a HIP graph) == plain per-instance solves,
  bitwise, on uneven instances; every graph replay == the eager launch;
- served: a request's result is bitwise the same alone and inside a mix of
  concurrent requests; per-controller ordering and warm starts hold;
- closed loop on the device: the first update equals a plain solve, and K
  updates match an oracle closed loop run from the same start;
- launch shapes, the parameter defaults, buffer reuse and the served form's
  admission errors.
"""
import sys
import time

import numpy as np
import pytest

from paper_2508_05773_amd import brmppi as B
from paper_2508_05773_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(arena_bytes=3 << 30, n_streams=3, max_controllers=700)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c3_small():
    insts = W.config3(n_instances=24, seed=33)
    # keep the test quick: cap the sample counts
    return [p.copy(S=min(p.S, 4096)) for p in insts]


def test_batched_equals_plain(ctx, c3_small):
    log(f"  batched vs plain on {len(c3_small)} instances")
    plain = []
    for i, p in enumerate(c3_small):
        ctx.set_path(100 + i, p.path, p.ds)
        u, st, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=100 + i))
        plain.append(u)
    pbs = [B.ProblemBuffers(p, controller=100 + i) for i, p in enumerate(c3_small)]
    for rep in range(3):          # first call captures the graph, the rest replay it
        outs, stats, _ = B.brmppi_solve_batch(ctx.h, pbs)
        for i in range(len(c3_small)):
            assert np.array_equal(outs[i], plain[i]), (rep, i)
        # eager work between replays
        B.brmppi_solve(ctx.h, B.ProblemBuffers(c3_small[0], controller=100))


def test_batch_buffers_reuse(ctx, c3_small):
    # arguments marshalled once (BatchBuffers) give the same results as a
    # list marshalled per call; each call refreshes the returned views
    log(f"  batch buffers reused over {len(c3_small)} instances")
    pbs = []
    for i, p in enumerate(c3_small):
        ctx.set_path(100 + i, p.path, p.ds)
        pbs.append(B.ProblemBuffers(p, controller=100 + i))
    ref, ref_st, _ = B.brmppi_solve_batch(ctx.h, pbs)
    ref = [r.copy() for r in ref]
    bb = B.BatchBuffers(pbs)
    for rep in range(3):
        bb.out[:] = np.nan
        outs, st, _ = B.brmppi_solve_batch(ctx.h, bb)
        for i in range(len(c3_small)):
            assert np.array_equal(outs[i], ref[i]), (rep, i)
            assert np.shares_memory(outs[i], bb.out), i
            assert st[i]["Z"] == ref_st[i]["Z"], (rep, i)


def test_batch_plan_reuse(ctx, c3_small):
    # a batch with the previous one's composition reuses its plan (layout,
    # tiles, reduce items) and refills only the descriptors: new seeds and
    # states must give the plain solves' results; a changed composition
    # plans afresh
    log(f"  batch plan reuse over {len(c3_small)} instances")
    for i, p in enumerate(c3_small):
        ctx.set_path(100 + i, p.path, p.ds)

    def check(probs, tag):
        pbs = [B.ProblemBuffers(p, controller=100 + i) for i, p in enumerate(probs)]
        outs, _, _ = B.brmppi_solve_batch(ctx.h, pbs)
        for i, pb in enumerate(pbs):
            u, _, _ = B.brmppi_solve(ctx.h, pb)
            assert np.array_equal(outs[i], u), (tag, i)

    base = list(c3_small)
    check(base, "first")
    # same composition, other contents: seeds and start states
    moved = [p.copy(seed=p.seed + 17, x0=p.x0 + np.float32(0.05)) for p in base]
    check(moved, "same composition")
    # another composition (one horizon changed), then the first again
    other = list(base)
    other[3] = other[3].copy(T=other[3].T + 4, u_nom=np.zeros((other[3].T + 4, 3), np.float32))
    check(other, "changed composition")
    check(base, "first again")


def test_batched_matches_oracle(ctx, c3_small):
    from oracle import oracle as O
    pbs = [B.ProblemBuffers(p, controller=100 + i) for i, p in enumerate(c3_small)]
    for i, p in enumerate(c3_small):
        ctx.set_path(100 + i, p.path, p.ds)
    outs, stats, _ = B.brmppi_solve_batch(ctx.h, pbs)
    for i in (0, 5, 11, 23):
        p = c3_small[i]
        o = O.solve(p, nthreads=16)
        tol = 1e-4 * np.array([4.0, 1.8, p.params["nu_bar"]])
        du = np.abs(outs[i] - o["U_new"]).max(axis=0)
        log(f"  batched inst {i}: S={p.S} T={p.T} n_obs={p.n_obs} U err {du}")
        assert np.all(du <= tol)
        assert stats[i]["J_min"] == pytest.approx(o["stats"]["J_min"], rel=1e-4)


def test_batched_mixed_guidance_and_hitch(ctx):
    """one launch holding guided, unguided and hitch-off instances"""
    probs = [W.random_small(60 + k, S=500 + 37 * k, T=9 + k, n_obs=k % 5) for k in range(6)]
    probs[1] = probs[1].copy(flags=W.FLAG_GUIDANCE_OFF)
    probs[4] = probs[4].copy(flags=W.FLAG_HITCH_OFF)
    for k, p in enumerate(probs):
        ctx.set_path(200 + k, p.path, p.ds)
    plain = [B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=200 + k))[0] for k, p in enumerate(probs)]
    outs, _, _ = B.brmppi_solve_batch(ctx.h, [B.ProblemBuffers(p, controller=200 + k) for k, p in enumerate(probs)])
    for k in range(len(probs)):
        assert np.array_equal(outs[k], plain[k]), k


def test_batched_split_by_bucket(ctx):
    """enough 2-obstacle samples for a launch of their own beside 32-obstacle
    and unguided instances (several rollout launches in one batch), and a thin
    bucket that joins a heavier one: every instance equals its plain solve"""
    probs = []
    for k in range(12):     # 12 x 32768 samples with 2 obstacles: a launch of their own
        probs.append(W.random_small(90 + k, S=32768, T=4, n_obs=2))
    for k in range(3):      # a few 32-obstacle instances
        probs.append(W.random_small(110 + k, S=3000 + 500 * k, T=5, n_obs=32))
    probs.append(W.random_small(120, S=2500, T=6, n_obs=12))                         # thin 16-slot bucket
    probs.append(W.random_small(121, S=1800, T=5, n_obs=3).copy(flags=W.FLAG_GUIDANCE_OFF))  # thin unguided
    for k, p in enumerate(probs):
        ctx.set_path(400 + k, p.path, p.ds)
    log(f"  split batch: {len(probs)} instances, {sum(p.S for p in probs)} samples")
    plain = [B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=400 + k))[0] for k, p in enumerate(probs)]
    pbs = [B.ProblemBuffers(p, controller=400 + k) for k, p in enumerate(probs)]
    for rep in range(2):
        outs, _, _ = B.brmppi_solve_batch(ctx.h, pbs)
        for k in range(len(probs)):
            assert np.array_equal(outs[k], plain[k]), (rep, k)


def test_served_alone_vs_mix(ctx):
    probs = W.config4_controllers(n_ctrl=40, seed=44)
    probs = [p.copy(S=min(p.S, 8192), T=min(p.T, 50)) for p in probs]
    for k, p in enumerate(probs):
        ctx.set_path(300 + k, p.path, p.ds)
    # alone: one request at a time
    alone = []
    for k, p in enumerate(probs[:8]):
        t, _ = B.brmppi_submit(ctx.h, B.ProblemBuffers(p, controller=300 + k))
        u, st, rc = B.brmppi_wait(ctx.h, t, p.T)
        alone.append(u)
    # in the mix: all 40 submitted at once (the first 8 again, same inputs)
    tickets = []
    for k, p in enumerate(probs):
        t, _ = B.brmppi_submit(ctx.h, B.ProblemBuffers(p, controller=300 + k))
        tickets.append(t)
    mixed = [B.brmppi_wait(ctx.h, t, p.T)[0] for t, p in zip(tickets, probs)]
    for k in range(8):
        assert np.array_equal(alone[k], mixed[k]), k
    # and the served result equals the plain solve
    for k in (0, 3, 17, 39):
        u, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(probs[k], controller=300 + k))
        assert np.array_equal(u, mixed[k]), k


def test_served_order_and_warm_start(ctx):
    """two requests of one controller: the second (u_nom = NULL) starts from the
    first one's shifted result"""
    p = W.random_small(70, S=2000, T=20, n_obs=3)
    ctx.set_path(400, p.path, p.ds)
    t1, _ = B.brmppi_submit(ctx.h, B.ProblemBuffers(p, controller=400))
    p2 = p.copy(seed=p.seed + 1)
    t2, _ = B.brmppi_submit(ctx.h, B.ProblemBuffers(p2, controller=400, with_nominal=False))
    u1, _, _ = B.brmppi_wait(ctx.h, t1, p.T)
    u2, _, _ = B.brmppi_wait(ctx.h, t2, p.T)
    # replay with the plain path
    ctx.set_path(401, p.path, p.ds)
    v1, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=401))
    v2, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(p2, controller=401, with_nominal=False))
    assert np.array_equal(u1, v1) and np.array_equal(u2, v2)
    # consumed / unknown tickets
    with pytest.raises(B.BrmppiError) as e:
        B.brmppi_poll(ctx.h, t1, p.T)
    assert e.value.code == B.ENOTICKET


def test_served_closed_loop_on_device(ctx):
    """X0_RESIDENT | ADVANCE_PLANT requests == brmppi_closed_loop, bitwise"""
    p = W.random_small(71, S=1500, T=15, n_obs=4)
    ctx.set_path(402, p.path, p.ds)
    ctx.set_path(403, p.path, p.ds)
    K = 5
    x_cl, u_cl = B.brmppi_closed_loop(ctx.h, B.ProblemBuffers(p, controller=402), K)
    B.brmppi_set_state(ctx.h, 403, p.x0.astype(np.float64))
    flags = p.flags | B.X0_RESIDENT | B.ADVANCE_PLANT
    outs = []
    for k in range(K):
        pb = B.ProblemBuffers(p, controller=403, with_nominal=(k == 0), flags=flags, seed=p.seed + k)
        t, _ = B.brmppi_submit(ctx.h, pb)
        outs.append(B.brmppi_wait(ctx.h, t, p.T)[0])
    assert np.array_equal(np.array([o[0] for o in outs]), u_cl)
    assert np.array_equal(B.brmppi_get_state(ctx.h, 403), x_cl[-1])


def test_closed_loop_matches_plain(ctx):
    """the first update of the device closed loop equals a plain solve"""
    p = W.config2().copy(S=2048, T=30)
    ctx.set_path(404, p.path, p.ds)
    ctx.set_path(405, p.path, p.ds)
    x_cl, u_cl = B.brmppi_closed_loop(ctx.h, B.ProblemBuffers(p, controller=404), 3)
    assert np.all(np.isfinite(x_cl))
    u0, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=405))
    assert np.array_equal(u0[0], u_cl[0])


@pytest.mark.parametrize("K,chunk_crossing", [(6, False), (35, True)])
def test_closed_loop_matches_oracle_loop(ctx, K, chunk_crossing):
    """K device-resident receding-horizon updates against an oracle closed loop
    run from the same start: oracle update k solves from the oracle's own plant
    state and warm start with seed + k, then the oracle plant steps by its first
    input (clamped to the input bounds) and the warm start shifts.  Every applied
    input is compared (1e-4 of each input's range), the plant states within the
    drift those input errors allow (K Ts 1e-4 range on a and delta, and their
    effect on the rest), and the final warm start in full.  K = 35 crosses
    several staging chunks of the loop."""
    from oracle import oracle as O
    p = W.config2().copy(S=2048, T=30) if not chunk_crossing else W.config2().copy(S=1024, T=20)
    cid = 416 if not chunk_crossing else 417
    ctx.set_path(cid, p.path, p.ds)
    x_cl, u_cl = B.brmppi_closed_loop(ctx.h, B.ProblemBuffers(p, controller=cid), K)
    U_warm = B.brmppi_get_nominal(ctx.h, cid, p.T)
    x = p.x0.astype(np.float64)
    U = p.u_nom.astype(np.float64)
    tol = 1e-4 * np.array([4.0, 1.8, p.params["nu_bar"]])
    worst_u, worst_x = 0.0, 0.0
    for k in range(K):
        o = O.solve(p.copy(seed=p.seed + k), nthreads=16, x0=x, u_nom=U)
        du = np.abs(u_cl[k] - o["U_new"][0])
        worst_u = max(worst_u, float((du / tol).max()))
        assert np.all(du <= tol), (k, du)
        x = O.plant_step(x, o["U_new"][0], p.params)
        U = np.concatenate([o["U_new"][1:], o["U_new"][-1:]])
        dx = np.abs(x_cl[k + 1] - x)
        worst_x = max(worst_x, float(dx.max()))
        assert dx.max() <= (k + 1) * p.params["Ts"] * tol.max() * 10.0, (k, dx)
    log(f"  closed loop K={K}: worst applied-input error {worst_u:.3e} of the tolerance, worst state error {worst_x:.3e}")
    assert np.all(np.abs(U_warm - U) <= tol)


@pytest.mark.parametrize("n_obs,flags,e4", [(7, 0, False), (2, 0, False), (13, W.FLAG_HITCH_OFF, False),
                                            (29, 0, False), (5, W.FLAG_GUIDANCE_OFF, False),
                                            (7, W.FLAG_COLLISION_PENALTY, False),
                                            (4, W.FLAG_GUIDANCE_OFF | W.FLAG_COLLISION_PENALTY, False),
                                            (9, 0, True), (6, W.FLAG_COLLISION_PENALTY, True)])
def test_launch_shapes_bitwise_identical(ctx, n_obs, flags, e4):
    """every (block size, lanes per sample, noise source) gives the same bits:
    costs, applied sequences and the update (e4: every other obstacle a
    super-ellipse, so lanes of a group take different row code)"""
    p = W.random_small(80 + n_obs, S=2999, T=12, n_obs=n_obs).copy(flags=flags)
    if e4:
        obs = p.obstacles.copy()
        obs[1::2, 5] = 4.0
        p = p.copy(obstacles=obs)
    ctx.set_path(406, p.path, p.ds)
    B.brmppi_set_launch(ctx.h, 64, 0)
    ref = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(p, controller=406), want_J=True, want_useq=True)
    for variant in (0, 1, 2, 3, 4):
        if flags & W.FLAG_GUIDANCE_OFF and variant > 1:
            continue
        for block in (64, 128, 192, 256):
            log(f"  shape block={block} variant={variant} n_obs={n_obs}")
            B.brmppi_set_launch(ctx.h, block, variant)
            g = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(p, controller=406), want_J=True, want_useq=True)
            assert np.array_equal(g["J"], ref["J"]), (block, variant)
            assert np.array_equal(g["useq"], ref["useq"]), (block, variant)
            assert np.array_equal(g["U_new"], ref["U_new"]), (block, variant)
    B.brmppi_set_launch(ctx.h, 0, 0)


@pytest.mark.parametrize("T", [1, 2, 3, 7, 300])
def test_horizons_odd_short_and_long_bitwise(ctx, T):
    """the precomputed-normals forms step in pairs, the fewer-lane ones with an
    odd last step peeled and the nominal inputs staged in LDS (3T floats, more
    than two per thread at T = 300): every horizon gives the bits of the
    one-lane in-kernel-noise form, which steps one at a time"""
    p = W.random_small(91, S=1000, T=T, n_obs=9)
    obs = p.obstacles.copy()
    obs[1::3, 5] = 4.0
    p = p.copy(obstacles=obs)
    ctx.set_path(407, p.path, p.ds)
    B.brmppi_set_launch(ctx.h, 64, 0)
    ref = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(p, controller=407), want_J=True, want_useq=True)
    for variant in (1, 2, 3, 4):
        for block in (64, 256):
            log(f"  horizon T={T} block={block} variant={variant}")
            B.brmppi_set_launch(ctx.h, block, variant)
            g = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(p, controller=407), want_J=True, want_useq=True)
            assert np.array_equal(g["J"], ref["J"]), (T, block, variant)
            assert np.array_equal(g["useq"], ref["useq"]), (T, block, variant)
            assert np.array_equal(g["U_new"], ref["U_new"]), (T, block, variant)
    B.brmppi_set_launch(ctx.h, 0, 0)


@pytest.mark.parametrize("block,variant", [(192, 0), (192, 2), (192, 3), (96 * 2, 4)])
def test_block_192_many_groups(ctx, block, variant):
    """tiles of 192 samples (or 96, 48, 24 with lanes per sample) straddle the
    groups of 1024 samples: the rollout must leave the reduction to k_reduce,
    and the update equals the one of block 256, bitwise, over eight groups"""
    p = W.random_small(85, S=8192, T=10, n_obs=6)
    ctx.set_path(418, p.path, p.ds)
    B.brmppi_set_launch(ctx.h, 256, variant)
    ref = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(p, controller=418), want_J=True)
    B.brmppi_set_launch(ctx.h, block, variant)
    try:
        g = B.brmppi_solve_ex(ctx.h, B.ProblemBuffers(p, controller=418), want_J=True)
    finally:
        B.brmppi_set_launch(ctx.h, 0, 0)
    assert np.array_equal(g["J"], ref["J"])
    assert np.array_equal(g["U_new"], ref["U_new"])
    assert g["stats"]["ess"] == ref["stats"]["ess"]


def test_params_null_uses_controller_params(ctx):
    """a problem without a params pointer runs with its controller's parameters
    (the library defaults until brmppi_set_params), bitwise as if passed"""
    p = W.random_small(86, S=1500, T=12, n_obs=4)
    p = p.copy(params=W.make_params(0.05, dtheta_max=0.5, kappa=0.03, l2=8.0))
    ctx.set_path(419, p.path, p.ds)
    want, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=419))
    B.brmppi_set_params(ctx.h, 419, p.params)
    got, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=419, with_params=False))
    assert np.array_equal(got, want)
    # defaults: Ts = 0.05 parameter set of the workloads
    B.brmppi_set_params(ctx.h, 419, None)
    q = p.copy(params=W.make_params(0.05))
    want2, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(q, controller=419))
    got2, _, _ = B.brmppi_solve(ctx.h, B.ProblemBuffers(q, controller=419, with_params=False))
    assert np.array_equal(got2, want2)
    bad = dict(p.params, Ts=-1.0)
    with pytest.raises(B.BrmppiError) as e:
        B.brmppi_set_params(ctx.h, 419, bad)
    assert e.value.code == B.EINVAL


def test_closed_loop_reuses_its_buffers(ctx):
    """a longer closed loop after a shorter one of the same problem allocates
    nothing: no scratch or pinned staging is re-allocated"""
    p = W.config2().copy(S=4096, T=40)
    ctx.set_path(420, p.path, p.ds)
    B.brmppi_closed_loop(ctx.h, B.ProblemBuffers(p, controller=420), 5, want_x=False, want_u=False)
    before = B.brmppi_get_info(ctx.h)
    B.brmppi_closed_loop(ctx.h, B.ProblemBuffers(p, controller=420), 60, want_x=True, want_u=True)
    after = B.brmppi_get_info(ctx.h)
    assert after["scratch_grows"] == before["scratch_grows"]
    assert after["pinned_grows"] == before["pinned_grows"]


def test_served_admission_errors():
    """EAGAIN once max_inflight requests are queued or unpolled; ETIMEDOUT from
    a deadline that passes while a request runs, after which the result is
    still delivered; ENOMEM for a request larger than the arena at submit, and
    at admission for one that fits the arena's size but can never fit its free
    space (the context's scratch holds the rest)"""
    c = B.Context(arena_bytes=96 << 20, n_streams=2, max_controllers=8, max_inflight=2)
    try:
        small = W.random_small(87, S=300, T=6, n_obs=2)
        for k in range(4):
            c.set_path(k, small.path, small.ds)
        t1, _ = B.brmppi_submit(c.h, B.ProblemBuffers(small, controller=0))
        t2, _ = B.brmppi_submit(c.h, B.ProblemBuffers(small, controller=1))
        _, rc = B.brmppi_submit(c.h, B.ProblemBuffers(small, controller=2), allow=(B.EAGAIN,))
        assert rc == B.EAGAIN
        B.brmppi_wait(c.h, t1, small.T)
        t3, _ = B.brmppi_submit(c.h, B.ProblemBuffers(small, controller=2))   # a slot is free again
        B.brmppi_wait(c.h, t2, small.T)
        B.brmppi_wait(c.h, t3, small.T)
        # ETIMEDOUT: a zero deadline on a request that takes milliseconds
        big = W.random_small(88, S=32768, T=80, n_obs=20)
        c.set_path(4, big.path, big.ds)
        tb, _ = B.brmppi_submit(c.h, B.ProblemBuffers(big, controller=4))
        _, _, rc = B.brmppi_wait(c.h, tb, big.T, timeout_ms=0, allow=(B.ETIMEDOUT,))
        assert rc == B.ETIMEDOUT
        u, st, rc = B.brmppi_wait(c.h, tb, big.T, timeout_ms=60000)
        assert rc == B.OK and np.all(np.isfinite(u))
        # ENOMEM at submit: more than the whole arena
        huge = big.copy(S=1 << 21, T=100, u_nom=np.zeros((100, 3), np.float32))
        c.set_path(5, huge.path, huge.ds)
        _, rc = B.brmppi_submit(c.h, B.ProblemBuffers(huge, controller=5), allow=(B.ENOMEM,))
        assert rc == B.ENOMEM
        # ENOMEM at admission: a blocking solve leaves a scratch of about half
        # the arena behind; a request that needs about 60 % of it then never fits
        mid = big.copy(S=45056, T=100, u_nom=np.zeros((100, 3), np.float32),
                       obstacles=np.zeros((0, 8), np.float32))
        c.set_path(6, mid.path, mid.ds)
        B.brmppi_set_launch(c.h, 128, 0)
        B.brmppi_solve(c.h, B.ProblemBuffers(mid, controller=6))
        B.brmppi_set_launch(c.h, 0, 0)
        info = B.brmppi_get_info(c.h)
        need = mid.copy(S=60000)
        c.set_path(7, need.path, need.ds)
        log(f"  arena used {info['arena_used'] >> 20} MiB of {info['arena_bytes'] >> 20} MiB")
        tn, rc = B.brmppi_submit(c.h, B.ProblemBuffers(need, controller=7), allow=(B.OK, B.ENOMEM))
        if rc == B.OK:
            _, _, rc = B.brmppi_wait(c.h, tn, need.T, timeout_ms=10000, allow=(B.ENOMEM,))
        assert rc == B.ENOMEM
        assert B.brmppi_get_info(c.h)["served_failed"] >= 1
    finally:
        c.close()


def test_default_launch_table_in_effect():
    """a fresh context uses its launch table (no shape forced): a guided solve
    with S <= 8192 runs four lanes per sample with the separate noise kernel,
    an unguided one a single lane"""
    c = B.Context(arena_bytes=1 << 30, n_streams=1, max_controllers=4, flags_extra=B.CTX_PROFILE_ROLLOUT)
    try:
        p = W.random_small(91, S=3000, T=12, n_obs=7)
        c.set_path(0, p.path, p.ds)
        B.brmppi_solve(c.h, B.ProblemBuffers(p, controller=0))
        prof = B.brmppi_profile_read(c.h)
        assert prof["rollout"]["count"] == 1 and prof["noise"]["count"] == 1
        B.brmppi_profile_reset(c.h)
        B.brmppi_set_launch(c.h, 128, 0)
        B.brmppi_solve(c.h, B.ProblemBuffers(p, controller=0))
        prof = B.brmppi_profile_read(c.h)
        assert prof["rollout"]["count"] == 1 and prof["noise"]["count"] == 0
    finally:
        c.close()


def test_large_noise_buffer():
    """S = 65536, T = 100, 32 obstacles: 970 MB of precomputed normals.  With a
    3 GiB arena the four-lane form draws them in the noise kernel; with a 1 GiB
    arena (half of it is the limit) the same request falls back to in-kernel
    normals.  Both give the bits of the one-lane in-kernel solve."""
    p = W.config5()
    runs = {}
    for arena, shape in ((3 << 30, (256, 3)), (3 << 30, (128, 0)), (1 << 30, (256, 3))):
        c = B.Context(arena_bytes=arena, n_streams=1, max_controllers=4, flags_extra=B.CTX_PROFILE_ROLLOUT)
        try:
            log(f"  c5 arena={arena >> 30} GiB shape={shape}")
            c.set_path(0, p.path, p.ds)
            B.brmppi_set_launch(c.h, *shape)
            g = B.brmppi_solve_ex(c.h, B.ProblemBuffers(p, controller=0), want_J=True)
            prof = B.brmppi_profile_read(c.h)
            runs[(arena, shape)] = (g, prof["noise"]["count"])
        finally:
            c.close()
    ref, n_ref = runs[(3 << 30, (128, 0))]
    assert n_ref == 0
    assert runs[(3 << 30, (256, 3))][1] == 1
    assert runs[(1 << 30, (256, 3))][1] == 0
    for key, (g, _) in runs.items():
        assert np.array_equal(g["J"], ref["J"]), key
        assert np.array_equal(g["U_new"], ref["U_new"]), key


def test_autotune(ctx, tmp_path):
    p = W.random_small(90, S=3000, T=12, n_obs=7)
    ctx.set_path(406, p.path, p.ds)
    before = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=406))[0]
    B.brmppi_autotune(ctx.h)
    after = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=406))[0]
    assert np.array_equal(before, after)


def test_invalid_arguments_leave_state(ctx):
    p = W.random_small(81, S=100, T=5, n_obs=1)
    ctx.set_path(407, p.path, p.ds)
    good = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=407))[0]
    bad = p.copy(lam=-1.0)
    with pytest.raises(B.BrmppiError) as e:
        B.brmppi_solve(ctx.h, B.ProblemBuffers(bad, controller=407))
    assert e.value.code == B.EINVAL
    obs = p.obstacles.copy()
    obs[0, 5] = 3.0                          # only e = 2 and e = 4 are implemented
    with pytest.raises(B.BrmppiError) as e:
        B.brmppi_solve(ctx.h, B.ProblemBuffers(p.copy(obstacles=obs), controller=407))
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BrmppiError) as e:      # no warm start of that length
        B.brmppi_solve(ctx.h, B.ProblemBuffers(p.copy(T=7, u_nom=np.zeros((7, 3), np.float32)), controller=408,
                                               with_nominal=False))
    assert e.value.code in (B.ESTATE,)
    # the warm start of 407 is unchanged by the failed calls
    assert np.array_equal(B.brmppi_get_nominal(ctx.h, 407, p.T), np.concatenate([good[1:], good[-1:]]))


@pytest.mark.parametrize("seed", [0, 1, 2, 4])
def test_hitch_stabiliser_plant_step(ctx, seed):
    """The device hitch-angle QP (eq. (19)) against the oracle's, at plant
    states where the hitch row binds.  With zero sampling noise and guidance
    off every sample applies the nominal sequence, so U_new[0] is exactly the
    chosen reference; the stabilised plant step must match the oracle's (FP64,
    different exact methods: candidate enumeration vs active-set KKT)."""
    from oracle import oracle as O
    from tests.hitch_qp_cases import binding_state
    base = W.random_small(95, S=64, T=4, n_obs=2)
    prm = W.make_params(0.05, dtheta_max=0.35)
    prm.update(sigma_j=0.0, sigma_w=0.0, sigma_nu=0.0, sigma_a=0.0)
    x, uref = binding_state(O, prm, np.random.default_rng(seed))
    # few significant bits: the weighted average of identical sequences is then exact
    uref = np.round(uref * 1024.0) / 1024.0
    uq, st = O.hitch_qp(x, uref, prm)
    assert st == 0 and not np.allclose(uq, uref)
    u_nom = np.zeros((base.T, 3), np.float32)
    u_nom[:, 0], u_nom[:, 1], u_nom[:, 2] = uref[0], uref[1], 0.5
    uref32 = u_nom[0].astype(np.float64)
    p = base.copy(params=prm, u_nom=u_nom, flags=W.FLAG_GUIDANCE_OFF)
    cid = 410 + seed
    ctx.set_path(cid, p.path, p.ds)
    for flags, plant in ((B.HITCH_QP, O.plant_step_qp), (0, O.plant_step)):
        B.brmppi_set_state(ctx.h, cid, x)
        pb = B.ProblemBuffers(p, controller=cid, flags=p.flags | B.X0_RESIDENT | B.ADVANCE_PLANT | flags)
        u, _, _ = B.brmppi_solve(ctx.h, pb)
        assert np.array_equal(u[0], u_nom[0])                 # U_new[0] is the reference
        xn = B.brmppi_get_state(ctx.h, cid)
        want = plant(x, uref32, prm)
        log(f"  hitch QP seed {seed} flags {flags}: max |dx| {np.abs(xn - want).max():.2e}")
        assert np.allclose(xn, want, rtol=1e-12, atol=1e-13), (flags, xn, want)
    # the stabiliser changed the applied input
    assert not np.allclose(O.plant_step_qp(x, uref32, prm), O.plant_step(x, uref32, prm))


def test_hitch_stabiliser_needs_plant_step(ctx):
    p = W.random_small(96, S=64, T=4, n_obs=1)
    ctx.set_path(415, p.path, p.ds)
    with pytest.raises(B.BrmppiError) as e:
        B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=415, flags=B.HITCH_QP))
    assert e.value.code == B.EINVAL
