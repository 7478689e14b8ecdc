"""GPU tests of the hand-off of partial results between blocks.

The fused epilogue (tile -> group -> instance) and the reduce kernel (item ->
instance) pass partials between blocks that may run on different XCDs.  The
partials are written and read as device-scope relaxed atomics and a publisher
drains its stores before its counter increment.  A stale read in the merging
block would change U_new, so repeated solves of the same inputs must agree
bit for bit, on every merge path:

- the fused epilogue at the c2 size (256 tiles, 8 groups), in plain solves and
  in the closed loop's first update;
- the reduce kernel behind batched solves (one round of items, and several
  rounds when its grid is smaller than the item count) and behind a plain
  solve whose tiles do not divide a group.
"""
import sys

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
    c = B.Context(arena_bytes=4 << 30, n_streams=2, max_controllers=640)
    yield c
    c.close()


def test_fused_epilogue_repeats_bitwise(ctx):
    p = W.config2()
    log(f"  fused epilogue: S={p.S} T={p.T}, block 256 eight lanes, 200 repeats")
    B.brmppi_set_launch(ctx.h, 256, 4)
    try:
        ctx.set_path(0, p.path, p.ds)
        pb = B.ProblemBuffers(p, controller=0)
        u0, st0, _ = B.brmppi_solve(ctx.h, pb)
        for k in range(200):
            u, st, _ = B.brmppi_solve(ctx.h, pb)
            assert np.array_equal(u, u0), k
            assert st["Z"] == st0["Z"] and st["ess"] == st0["ess"], k
    finally:
        B.brmppi_set_launch(ctx.h, 0, 0)


@pytest.mark.parametrize("block,variant", [(256, 0), (128, 1)])
def test_reduce_kernel_repeats_bitwise(ctx, block, variant):
    # one lane per sample: 64- or 128-sample tiles reduce through k_reduce
    p = W.config2().copy(S=20000)
    log(f"  reduce kernel (plain): S={p.S} block {block} variant {variant}, 60 repeats")
    B.brmppi_set_launch(ctx.h, block, variant)
    try:
        ctx.set_path(1, p.path, p.ds)
        pb = B.ProblemBuffers(p, controller=1)
        u0, _, _ = B.brmppi_solve(ctx.h, pb)
        for k in range(60):
            u, _, _ = B.brmppi_solve(ctx.h, pb)
            assert np.array_equal(u, u0), k
    finally:
        B.brmppi_set_launch(ctx.h, 0, 0)


def test_batched_reduce_repeats_bitwise(ctx):
    insts = W.config3()     # 64 uneven instances: reduce items of up to 136 rows
    log(f"  batched: {len(insts)} uneven instances, 40 repeats (graph replays)")
    pbs = []
    for i, p in enumerate(insts):
        ctx.set_path(20 + i, p.path, p.ds)
        pbs.append(B.ProblemBuffers(p, controller=20 + i))
    outs0, st0, _ = B.brmppi_solve_batch(ctx.h, pbs)
    for k in range(40):
        outs, st, _ = B.brmppi_solve_batch(ctx.h, pbs)
        for i in range(len(insts)):
            assert np.array_equal(outs[i], outs0[i]), (k, i)
            assert st[i]["Z"] == st0[i]["Z"], (k, i)
    # the batch's long reduce items give the bits of plain solves
    for i in range(0, len(insts), 5):
        u, _, _ = B.brmppi_solve(ctx.h, pbs[i])
        assert np.array_equal(u, outs0[i]), i


def test_batched_reduce_several_rounds(ctx):
    # more reduce items than the kernel's grid (8 blocks per CU): the later
    # items come from the work queue
    base = W.config3(n_instances=600, seed=9)
    insts = [p.copy(S=4096, T=20) for p in base]
    log(f"  batched, reduce items past the grid: {len(insts)} x S=4096 T=20, 6 repeats")
    pbs = []
    for i, p in enumerate(insts):
        ctx.set_path(i, p.path, p.ds)
        pbs.append(B.ProblemBuffers(p, controller=i))
    outs0, _, _ = B.brmppi_solve_batch(ctx.h, pbs)
    check = (0, 299, 599)
    plain = [B.brmppi_solve(ctx.h, pbs[i])[0] for i in check]
    for k in range(6):
        outs, _, _ = B.brmppi_solve_batch(ctx.h, pbs)
        for i in range(len(insts)):
            assert np.array_equal(outs[i], outs0[i]), (k, i)
    for j, i in enumerate(check):
        assert np.array_equal(outs0[i], plain[j]), i
