"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every function include/brmppi.h declares, the ctypes structs match the C
layout, and argument validation fails before touching a device."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2508_05773_amd import brmppi as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    syms = B.declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    # and the exports are real functions of this library
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    for s in syms:
        assert f" T {s}" in out, s


LAYOUT_SRC = r"""
#include <stdio.h>
#include <stddef.h>
#include "brmppi.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("brmppi_config %zu\n", sizeof(brmppi_config));
  F(brmppi_config, arena) F(brmppi_config, arena_bytes) F(brmppi_config, streams) F(brmppi_config, n_streams)
  F(brmppi_config, max_controllers) F(brmppi_config, max_inflight) F(brmppi_config, autotune_cache)
  F(brmppi_config, flags) F(brmppi_config, device)
  printf("brmppi_params %zu\n", sizeof(brmppi_params));
  F(brmppi_params, Ts) F(brmppi_params, Qc) F(brmppi_params, W_j) F(brmppi_params, alpha0) F(brmppi_params, h_eps)
  printf("brmppi_obstacle %zu\n", sizeof(brmppi_obstacle));
  printf("brmppi_problem %zu\n", sizeof(brmppi_problem));
  F(brmppi_problem, controller) F(brmppi_problem, S) F(brmppi_problem, T) F(brmppi_problem, x0)
  F(brmppi_problem, u_nom) F(brmppi_problem, obs) F(brmppi_problem, n_obs) F(brmppi_problem, t0)
  F(brmppi_problem, lambda) F(brmppi_problem, seed) F(brmppi_problem, instance) F(brmppi_problem, flags)
  F(brmppi_problem, params)
  printf("brmppi_stats %zu\n", sizeof(brmppi_stats));
  F(brmppi_stats, J_min) F(brmppi_stats, status) F(brmppi_stats, latency_us)
  printf("brmppi_outputs %zu\n", sizeof(brmppi_outputs));
  F(brmppi_outputs, u_out) F(brmppi_outputs, J_out) F(brmppi_outputs, useq_out)
  printf("brmppi_info %zu\n", sizeof(brmppi_info));
  F(brmppi_info, scratch_grows) F(brmppi_info, pinned_grows) F(brmppi_info, arena_used)
  F(brmppi_info, served_failed)
  return 0;
}
"""


def test_struct_layouts_match_header():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "layout.c")
    exe = os.path.join(d, "layout")
    open(src, "w").write(LAYOUT_SRC)
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
    got = {}
    for line in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.splitlines():
        k, v = line.split()
        got[k] = int(v)
    cls = {"brmppi_config": B.brmppi_config, "brmppi_params": B.brmppi_params,
           "brmppi_obstacle": B.brmppi_obstacle, "brmppi_problem": B.brmppi_problem,
           "brmppi_stats": B.brmppi_stats, "brmppi_outputs": B.brmppi_outputs, "brmppi_info": B.brmppi_info}
    for k, v in got.items():
        if "." in k:
            t, f = k.split(".")
            f = "lambda_" if f == "lambda" else f
            assert getattr(cls[t], f).offset == v, k
        else:
            assert C.sizeof(cls[k]) == v, k


def test_create_rejects_bad_config_without_a_device():
    L = B.lib()
    h = C.c_void_p()
    cfg = B.brmppi_config()
    assert L.brmppi_create(None, C.byref(h)) == B.EINVAL
    assert L.brmppi_create(C.byref(cfg), C.byref(h)) == B.EINVAL        # NULL arena
    assert "arena" in B.last_error()
    cfg.arena = 0x1001                                                   # misaligned
    cfg.arena_bytes = 1 << 30
    assert L.brmppi_create(C.byref(cfg), C.byref(h)) == B.EINVAL
    cfg.arena = 0x100000
    cfg.n_streams = 0
    assert L.brmppi_create(C.byref(cfg), C.byref(h)) == B.EINVAL
    assert "n_streams" in B.last_error()
    assert L.brmppi_destroy(None) == B.EINVAL
    assert L.brmppi_solve(None, None, None, None) == B.EINVAL
    assert L.brmppi_poll(None, 1, None, None) == B.EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        B.lib()


def test_default_params_without_a_device():
    """brmppi_default_params needs no context: the library's defaults equal the
    workloads' parameter set at Ts = 0.05 s (the values used by every
    benchmark configuration but c1)"""
    from paper_2508_05773_amd import workloads as W
    got = B.brmppi_default_params()
    want = W.make_params(0.05)
    for k in B.PARAM_FIELDS:
        assert np.float32(got[k]) == np.float32(want[k]), k
    assert got["disc_tractor"] == want["disc_tractor"] == [0.0] and got["disc_trailer"] == want["disc_trailer"] == []
    assert B.lib().brmppi_default_params(None) == B.EINVAL
    assert B.lib().brmppi_set_params(None, 0, None) == B.EINVAL
    assert B.lib().brmppi_get_info(None, None) == B.EINVAL


def test_batch_buffers_layout():
    # BatchBuffers: one output buffer, a pointer per instance at its offset,
    # views of 3T floats each, and the problem array copied from the structs
    from paper_2508_05773_amd import workloads as W

    insts = W.config3(n_instances=5, seed=1)
    pbs = [B.ProblemBuffers(p, controller=i) for i, p in enumerate(insts)]
    bb = B.BatchBuffers(pbs)
    assert bb.n == 5 and bb.out.size == sum(3 * p.T for p in insts)
    base = bb.out.ctypes.data
    off = 0
    for i, p in enumerate(insts):
        assert C.cast(bb.ptrs[i], C.c_void_p).value == base + 4 * off, i
        assert bb.views[i].shape == (p.T, 3)
        assert np.shares_memory(bb.views[i], bb.out)
        bb.views[i][:] = i
        off += 3 * p.T
        assert bb.arr[i].S == p.S and bb.arr[i].T == p.T and bb.arr[i].controller == i
    assert np.array_equal(np.unique(bb.out), np.arange(5, dtype=np.float32))
