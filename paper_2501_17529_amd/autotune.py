"""Launch-shape autotuner for the N-1 scan, with a JSON cache.

For one batch shape (grid sizes, candidates, variants, precision, device
architecture) it times dcflow_n1_score under every launch shape the library
offers (variants per pass-1 workgroup, monitored rows per LDS chunk and per
work item, persistent or one-workgroup-per-item launch), keeps only shapes whose
scores agree with the library's default, and caches the fastest.  The cache
file is DCFLOW_AUTOTUNE_CACHE or ~/.cache/dcflow/autotune.json.

Timing uses HIP events on the stream the kernels run on; nothing here computes
scores itself.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import dcflow as D

VC_SETS = {"fp32": (16, 8, 4, 1), "fp64": (16, 8, 4, 1)}


def cache_path() -> str:
    p = os.environ.get("DCFLOW_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "dcflow", "autotune.json")


def _arch() -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "unknown")


def shape_key(batch: "D.Batch", n_var: int, prec: str) -> str:
    v = batch.plan.view
    kmax = int(np.max(np.diff(batch.ca.off))) if batch.n_cand else 0
    rec = 0 if batch.get_tuning().get("worst_record", 0) < 0 else 1
    return (f"{_arch()}|{prec}|n_cand={batch.n_cand}|n_var={n_var}|n_mon={v.n_mon}|"
            f"n_out={v.n_out}|ld_o={v.ld_o}|n_multi={v.n_multi_out}|kmax={kmax}|rec={rec}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(batch: "D.Batch", n_var: int, prec: str):
    """The launch shapes worth timing for this batch."""
    mon_pad = (batch.plan.view.n_mon + 63) // 64 * 64
    vcs = [0] + [v for v in VC_SETS["fp64" if prec == "fp64" else "fp32"]
                 if v <= max(1, n_var) and v > 1]
    rcs = sorted({0} | {r for r in (64, 128, 256, 512) if r <= mon_pad})
    # row bands matter only when the seed block outgrows L2
    seed = mon_pad * batch.plan.view.ld_o * (8 if prec == "fp64" else 4)
    bands = [0] + ([b for b in (64, 128, 256, 512, 1024) if b < mon_pad] if seed > (2 << 20) else [])
    out = []
    for vc in vcs:
        for rc in rcs:
            for band in bands:
                if band and rc and rc > band:
                    continue  # the chunk is capped at the band: same as rc = band
                for pe in (0, 1):
                    out.append(dict(scan_vc=vc, scan_rchunk=rc, persistent=pe, scan_band=band))
    return out


def _time_scan(batch, flows, n_var, prec, out, reps):
    import torch
    s = torch.cuda.current_stream()
    batch.n1_score(flows, n_var, prec, out=out)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        batch.n1_score(flows, n_var, prec, out=out)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_scan(batch: "D.Batch", flows, n_var: int, prec: str, reps: int = 10,
              use_cache: bool = True, verbose: bool = False):
    """Picks (and applies to `batch`) the fastest scan launch shape; returns
    (config dict, {config string: ms})."""
    import torch
    path = cache_path()
    key = shape_key(batch, n_var, prec)
    cache = _load(path) if use_cache else {}
    # the batch's other settings (step chunks, the record, the guard) are kept
    base = batch.get_tuning()
    if key in cache:
        cfg = cache[key]["config"]
        batch.set_tuning(**dict(base, **cfg))
        return cfg, cache[key].get("times_ms", {})
    nb = max(batch.n_cand, 1) * D.SCORE_DTYPE.itemsize
    ref_out = torch.empty(nb, dtype=torch.uint8, device="cuda")
    batch.set_tuning(**dict(base, scan_vc=0, scan_rchunk=0, persistent=0, scan_band=0))
    batch.n1_score(flows, n_var, prec, out=ref_out)
    torch.cuda.synchronize()
    ref = D.Batch.scores_to_numpy(ref_out, batch.n_cand)
    out = torch.empty_like(ref_out)
    times = {}
    best, best_t = None, float("inf")
    for cfg in candidates(batch, n_var, prec):
        batch.set_tuning(**dict(base, **cfg))
        try:
            t = _time_scan(batch, flows, n_var, prec, out, reps)
        except D.DcflowError:
            # a shape whose LDS block does not fit this batch (wide contingency sets)
            times[json.dumps(cfg, sort_keys=True)] = None
            continue
        got = D.Batch.scores_to_numpy(out, batch.n_cand)
        same = (np.array_equal(got["max_load"], ref["max_load"])
                and np.array_equal(got["best_variant"], ref["best_variant"])
                and np.array_equal(got["worst_branch"], ref["worst_branch"])
                and np.array_equal(got["worst_outage"], ref["worst_outage"]))
        name = json.dumps(cfg, sort_keys=True)
        times[name] = round(t, 5) if same else None
        if verbose:
            print(f"autotune {name}: {t:.4f} ms{'' if same else ' (results differ: dropped)'}")
        if same and t < best_t:
            best, best_t = cfg, t
    if best is None:
        best = dict(scan_vc=0, scan_rchunk=0, persistent=0, scan_band=0)
    batch.set_tuning(**dict(base, **best))
    if use_cache:
        cache = _load(path)
        cache[key] = {"config": best, "times_ms": times}
        _store(path, cache)
    return best, times
