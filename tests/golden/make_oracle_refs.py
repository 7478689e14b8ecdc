"""Expected values of the full-size GPU parity cases, written by the FP64 oracle.

    python tests/golden/make_oracle_refs.py        (about two minutes on 8 cores)

The large cases (the 65536-sample, 100-step, 32-obstacle update and eight
requests of the served mix at their full sizes) take the oracle minutes of
CPU time, so their results are computed once here and stored in
oracle_large.json.  Every value comes from oracle/ alone, on inputs from the
seeded generators of paper_2508_05773_amd/workloads.py.  Each case records a
fingerprint of its inputs and the file records a hash of the oracle's source,
so that a test reading a stale file fails instead of comparing against it.
"""
from __future__ import annotations

import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O                       # noqa: E402
from paper_2508_05773_amd import workloads as W      # noqa: E402

OUT = os.path.join(HERE, "oracle_large.json")
ORACLE_SRC = os.path.join(ROOT, "oracle", "brmppi_oracle.c")

# requests of the served mix (controllers of the 256-controller workload),
# chosen to cover S in {2048, 8192, 32768}, T in {30, 50, 100}, 0 to 32
# obstacles and moving obstacles
SERVED_CONTROLLERS = (0, 1, 2, 4, 5, 7, 17, 33)
N_J_SAMPLES = 1024        # per-sample costs stored for the large update (plus the argmin)


def oracle_sha() -> str:
    """hash of the oracle's code (comments and blank lines do not count)"""
    src = open(ORACLE_SRC, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [ln.split("//", 1)[0].rstrip() for ln in src.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()[:16]


def fingerprint(p) -> str:
    h = hashlib.sha256()
    for a in (p.x0, p.u_nom, p.obstacles, p.path):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    for k in sorted(p.params):
        h.update(np.asarray(p.params[k], np.float64).reshape(-1).tobytes())
    h.update(repr((p.S, p.T, p.ds, p.lam, p.seed, p.instance, p.t0, p.flags)).encode())
    return h.hexdigest()[:16]


def cases():
    out = {"c5": W.config5()}
    ctrl = W.config4_controllers()
    for c in SERVED_CONTROLLERS:
        out[f"c4[{c}]"] = ctrl[c]
    return out


def sample_ids(S: int, J: np.ndarray) -> np.ndarray:
    rng = np.random.default_rng(S)
    ids = np.concatenate([np.arange(min(S, 64)), np.arange(max(0, S - 64), S),
                          rng.integers(0, S, N_J_SAMPLES - 128), [int(np.argmin(J))]])
    return np.unique(ids)


def main():
    nthreads = os.cpu_count() or 1
    res = {"oracle_sha": oracle_sha(), "cases": {}}
    for name, p in cases().items():
        t0 = time.time()
        o = O.solve(p, nthreads=nthreads)
        case = {
            "fingerprint": fingerprint(p), "S": p.S, "T": p.T, "n_obs": p.n_obs,
            "U_new": o["U_new"].tolist(), "J_min": o["stats"]["J_min"], "Z": o["stats"]["Z"],
            "ess": o["stats"]["ess"], "rc": int(o["rc"]),
        }
        if name == "c5":       # the served form returns no per-sample costs
            ids = sample_ids(p.S, o["J"])
            case["J_ids"] = ids.tolist()
            case["J"] = o["J"][ids].tolist()
        res["cases"][name] = case
        print(f"{name}: S={p.S} T={p.T} n_obs={p.n_obs} in {time.time() - t0:.1f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
