"""Pins for the oracle's noise: Philox4x32-10 and Box-Muller.

Philox is pinned by *running* an independent implementation, rocRAND's
PHILOX4_32_10 device/host API (compiled here for the host from the installed
headers), whose rocrand_init(seed, subsequence, offset) places the 64-bit seed
in the key and (offset/4, subsequence) in the counter words (0,1) and (2,3).
The normals are pinned by the distribution (Kolmogorov-Smirnov, moments,
independence across inputs and steps) and by the exact uniform mapping.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

RR_SRC = r"""
#include <cstdio>
#include <rocrand/rocrand_kernel.h>
int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_bin():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp(prefix="rr_")
    src = os.path.join(d, "rr.cpp")
    with open(src, "w") as f:
        f.write(RR_SRC)
    exe = os.path.join(d, "rr")
    subprocess.check_call([hipcc, "-O1", "--cuda-host-only", src, "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_bin):
    rng = np.random.default_rng(1)
    cases = []
    for _ in range(400):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        c = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        c[1] &= 0x3FFFFFFF    # rocrand takes the counter as offset*4 in 64 bits
        cases.append((seed, c))
    # edge counters and keys
    cases += [(0, [0, 0, 0, 0]), (2**64 - 1, [2**32 - 1] * 4), (1, [1, 0, 0, 0]),
              (2**32, [0, 2**32 - 1, 0, 1])]
    lines = []
    for seed, c in cases:
        sub = c[2] | (c[3] << 32)
        off = 4 * (c[0] | (c[1] << 32))
        off &= 2**64 - 1
        lines.append(f"{seed} {sub} {off}")
    out = subprocess.run([rocrand_bin], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    n_checked = 0
    for (seed, c), line in zip(cases, out):
        off = 4 * (c[0] | (c[1] << 32))
        if off >= 2**64:      # offset would overflow rocrand's 64-bit argument
            continue
        want = [int(v) for v in line.split()]
        got = orc.philox(c, [seed & 0xFFFFFFFF, seed >> 32])
        assert got == want, (seed, c)
        n_checked += 1
    assert n_checked > 300


def test_uniform23_exact(orc):
    assert orc.uniform23(0) == 2.0 ** -24
    assert orc.uniform23(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.uniform23(0x80000000) == 0.5 + 2.0 ** -24
    # the low 9 bits are discarded, and every value is a float32
    assert orc.uniform23(0x12345600) == orc.uniform23(0x123457FF)
    rng = np.random.default_rng(0)
    for r in rng.integers(0, 2**32, size=1000, dtype=np.uint64):
        u = orc.uniform23(int(r))
        assert float(np.float32(u)) == u and 0.0 < u < 1.0


def test_normal_block_layout(orc):
    """normal k of (s, tau) comes from block k//4 with counter (s, tau, k//4, inst)."""
    seed, inst = 0x0123456789ABCDEF, 77
    e = orc.normals(seed, inst, 5, 9, 11)
    for b in range(3):
        r = orc.philox([5, 9, b, inst], [seed & 0xFFFFFFFF, seed >> 32])
        u = [orc.uniform23(v) for v in r]
        rad0 = math.sqrt(-2 * math.log(u[0]))
        rad1 = math.sqrt(-2 * math.log(u[2]))
        blk = [rad0 * math.cos(2 * math.pi * u[1]), rad0 * math.sin(2 * math.pi * u[1]),
               rad1 * math.cos(2 * math.pi * u[3]), rad1 * math.sin(2 * math.pi * u[3])]
        for j in range(4):
            k = 4 * b + j
            if k < 11:
                assert e[k] == pytest.approx(blk[j], rel=1e-15, abs=1e-15)
    # a prefix request gives the same leading normals
    assert np.array_equal(orc.normals(seed, inst, 5, 9, 3), e[:3])


def test_normals_distribution(orc):
    xs = []
    for s in range(2000):
        for tau in range(5):
            xs.append(orc.normals(42, 3, s, tau, 10))
    X = np.array(xs)                       # (10000, 10)
    flat = X.reshape(-1)
    ks = stats.kstest(flat, "norm")
    assert ks.pvalue > 1e-3, ks
    assert abs(flat.mean()) < 0.01
    assert abs(flat.var() - 1.0) < 0.02
    # inputs of one step are uncorrelated, and so are consecutive steps
    C = np.corrcoef(X.T)
    off = C[~np.eye(10, dtype=bool)]
    assert np.abs(off).max() < 0.05
    a = np.array([orc.normals(42, 3, s, 0, 3) for s in range(3000)])
    b = np.array([orc.normals(42, 3, s, 1, 3) for s in range(3000)])
    assert abs(np.corrcoef(a[:, 0], b[:, 0])[0, 1]) < 0.06
    # a different instance gives a different stream
    assert not np.array_equal(orc.normals(42, 3, 0, 0, 4), orc.normals(42, 4, 0, 0, 4))
