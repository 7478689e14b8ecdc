"""GPU test of brmppi_solve_noalloc, the plain update whose scratch is the
device's static array instead of a block of the arena.

Two calls in a row, the second with a smaller input (the 8192-sample, 50-step,
8-obstacle update, then the 1024-sample, 30-step, 2-obstacle one), each equal
brmppi_solve's result and stats bitwise; the smaller one also matches the FP64
oracle at the parity tolerances (per-sample costs are not returned by this entry
point, so U_new is compared).  An update larger than the array is refused with
ENOMEM, and the context's arena is not touched by any of these calls.
"""
import os
import sys

import numpy as np
import pytest

from paper_2508_05773_amd import brmppi as B
from paper_2508_05773_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def u_tol(prob):
    P = prob.params
    return 1e-4 * np.array([P["j_hi"] - P["j_lo"], P["w_hi"] - P["w_lo"], P["nu_bar"]])


def test_noalloc_equals_solve_twice():
    big = W.config2()
    small = W.config1()
    assert (big.S, big.T, big.n_obs) == (8192, 50, 8) and (small.S, small.T, small.n_obs) == (1024, 30, 2)
    with B.Context(arena_bytes=512 << 20, n_streams=1, max_controllers=4) as ctx:
        ctx.set_path(0, big.path, big.ds)
        ctx.set_path(1, small.path, small.ds)
        ref = {}
        for k, p in ((0, big), (1, small)):
            log(f"  brmppi_solve S={p.S} T={p.T} n_obs={p.n_obs}")
            ref[k] = B.brmppi_solve(ctx.h, B.ProblemBuffers(p, controller=k))
        info0 = B.brmppi_get_info(ctx.h)
        for rep in range(2):
            for k, p in ((0, big), (1, small)):
                log(f"  brmppi_solve_noalloc S={p.S} T={p.T} n_obs={p.n_obs} (pass {rep})")
                u, st, rc = B.brmppi_solve_noalloc(ctx.h, B.ProblemBuffers(p, controller=k))
                assert rc == B.OK
                assert np.array_equal(u, ref[k][0]), (rep, k, np.abs(u - ref[k][0]).max())
                for f in ("J_min", "Z", "ess", "status"):
                    assert st[f] == ref[k][1][f], (rep, k, f, st[f], ref[k][1][f])
        info1 = B.brmppi_get_info(ctx.h)
        assert info1["arena_used"] == info0["arena_used"]
        assert info1["scratch_grows"] == info0["scratch_grows"]
        assert info1["pinned_grows"] == info0["pinned_grows"]
        # larger than the static array: refused before any device work
        huge = big.copy(S=1 << 20, T=100, u_nom=np.zeros((100, 3), np.float32))
        _, _, rc = B.brmppi_solve_noalloc(ctx.h, B.ProblemBuffers(huge, controller=0), allow=(B.ENOMEM,))
        assert rc == B.ENOMEM
        assert "static scratch" in B.last_error()
        # the refusal left the controller as it was: the next call still matches
        u, _, _ = B.brmppi_solve_noalloc(ctx.h, B.ProblemBuffers(small, controller=1))
        assert np.array_equal(u, ref[1][0])

    from oracle import oracle as O
    o = O.solve(small, nthreads=min(16, os.cpu_count() or 1))
    du = np.abs(ref[1][0] - o["U_new"]).max(axis=0)
    log(f"  S={small.S} U max abs err vs oracle {du}")
    assert np.all(du <= u_tol(small)), du
