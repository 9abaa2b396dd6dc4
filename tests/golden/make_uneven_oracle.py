"""Writes uneven_oracle.json: the CPU oracle's scores of 256 sampled candidates
of the uneven-rank workload (10,000-bus / 15,500-branch grid, 65,536 candidates
of rank 1..8, one perturbed injection each, every branch monitored, 2,000
contingencies).  Each sampled candidate's grid is rebuilt and factorised by
dense LU (oracle.dcflow_oracle.score_candidate), about a minute of one core per
candidate, so the values are stored instead of recomputed in the GPU test.

It calls only the oracle and the seeded input generator; the file holds a
fingerprint of the inputs so that a test can tell when the generator changed.

    python tests/golden/make_uneven_oracle.py [--procs 8]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gridgen as G  # noqa: E402
from oracle import dcflow_oracle as O  # noqa: E402

N_CAND = 65536
N_SAMPLE = 256
SAMPLE_SEED = 2025
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uneven_oracle.json")
_W = None


def sample_indices():
    rng = np.random.default_rng(SAMPLE_SEED)
    return sorted(int(i) for i in rng.choice(N_CAND, size=N_SAMPLE, replace=False))


def fingerprint(w, idx):
    """SHA-256 over the grid, the monitored and contingency sets, and the sampled
    candidates' elements and injections."""
    g = w.grid
    h = hashlib.sha256()
    for a in (g.f, g.t, g.b, g.p, w.mon, w.out):
        h.update(np.ascontiguousarray(a).tobytes())
    for i in idx:
        h.update(json.dumps(w.cands.elements(i)).encode())
        h.update(np.ascontiguousarray(w.inj[i]).tobytes())
    return h.hexdigest()


def _one(i):
    from threadpoolctl import threadpool_limits
    w = _W
    g = w.grid
    r = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, w.rating_scale, w.rating_offset)
    with threadpool_limits(limits=1):
        sc = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, w.cands.elements(i), w.inj[i],
                               w.mon, w.out, r)
    worst = O.worst_cases(sc, w.mon, w.out, 16) if np.isfinite(sc["best_max_load"]) else []
    return dict(index=i, max_load=[float(v) for v in sc["max_load"]],
                best_variant=int(sc["best_variant"]), overload_sum=float(sc["overload_sum"]),
                worst_branch=int(sc["worst_branch"]), worst_outage=int(sc["worst_outage"]),
                n_island=int(sc["n_island"]), status=int(sc["status"]),
                worst16=[[float(v), int(b), int(o)] for v, b, o in worst])


def main():
    global _W
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    t0 = time.time()
    _W = G.workload_uneven(0, n_cand=N_CAND)
    idx = sample_indices()
    print(f"workload generated in {time.time() - t0:.0f} s", flush=True)
    import multiprocessing as mp
    t1 = time.time()
    res = []
    with mp.get_context("fork").Pool(a.procs) as pool:
        for k, r in enumerate(pool.imap(_one, idx)):
            res.append(r)
            if k % 16 == 15:
                print(f"{k + 1} of {len(idx)} candidates, {time.time() - t1:.0f} s", flush=True)
    wall = time.time() - t1
    json.dump(dict(workload="uneven-10000bus", n_cand=N_CAND, sample_seed=SAMPLE_SEED,
                   fingerprint=fingerprint(_W, idx), oracle_wall_s=round(wall, 1),
                   oracle_procs=a.procs, candidates=res), open(OUT, "w"), indent=0)
    print(f"wrote {OUT}: {len(res)} candidates, oracle {wall:.0f} s on {a.procs} processes")


if __name__ == "__main__":
    main()
