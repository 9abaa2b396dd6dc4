"""Benchmark of the batched DC-loadflow screen on one MI355X.

One step = the whole hot path over one batch of the medium workload
(1,000-bus / 1,600-branch synthetic grid, 4,096 topology candidates with 1-3
bus splits plus 0-2 outages, 16 load-perturbed injection variants each, N-1
over 500 contingency branches that are also the monitored set):
dcflow_eval_topologies -> dcflow_eval_injections -> dcflow_n1_score, with the
candidate records and injections already resident in device memory.

value = N-1 loadflows per second of the plain FP64 path (the paper's
precision), loadflows = candidates x variants x contingencies per step.  The
mixed paths (FP32 and BF16X6 injection GEMM with the FP32 N-1 scan and its
FP64 error guard) are timed the same way and reported beside it, each with its
rooflines, its difference to the FP64 path over the whole batch and its error
against the oracle on the sampled candidates.  The other workloads (30-bus,
10,000-bus uneven ranks at 65,536 candidates, 2,000-bus control brute force,
the learned proposal), the end-to-end rate and a repeated-run protocol are
extra keys of the same line.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N-1 loadflows/s on 1 MI355X at ≤1e-4 rating error, mixed vs plain FP64 path"
PEAK_VALU_FMA_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12   # non-packed FMA issue, fp32 and fp64
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scan_medium_traffic.txt")


# ------------------------------------------------------------------ CPU baseline

def host_cores():
    """The host's CPUs as this process sees them: the logical CPU count, the CPUs
    it may run on (affinity), the cgroup CPU quota if one is set, and the model.
    'usable' = the smallest of those limits: every core the job can use."""
    logical = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = logical
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(period)
    except (OSError, ValueError):
        pass
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = affinity if quota is None else max(1, min(affinity, int(quota + 0.5)))
    return dict(logical=logical, affinity=affinity, cgroup_quota=quota, model=model,
                usable=usable)


def _warm(_):
    """Imports the oracle's modules in a pool process before the timed region."""
    import threadpoolctl  # noqa: F401
    from oracle import dcflow_oracle  # noqa: F401
    return 0


def _oracle_worker(args):
    from threadpoolctl import threadpool_limits
    from oracle import dcflow_oracle as O
    n_bus, f, t, b, slack, elems, x, mon, out, rating, controls, gens, multi, keep = args
    kw = dict(gens=gens, multi=multi)
    if controls:
        kw.update(controls=controls, ctrl=x[:, n_bus:])
        x = x[:, :n_bus]
    with threadpool_limits(limits=1):
        sc = O.score_candidate(n_bus, f, t, b, slack, elems, x, mon, out, rating, **kw)
    n_extra = (0 if gens is None else len(gens[0])) + (0 if multi is None else len(multi))
    # what the error report needs: per-variant maxima, islanding count, status and
    # the N-0 flows of the kept rows
    res = dict(max_load=sc["max_load"], n_island=sc["n_island"], status=sc["status"])
    if keep is not None and "p0" in sc["flows"]:
        res["p0"] = sc["flows"]["p0"][:, keep]
    return x.shape[0] * (len(out) + n_extra), res


def cpu_baseline(w, n_sample: int, max_var: int = 0, keep_rows=None):
    """The oracle (dense LU per candidate) on the first n_sample candidates (and
    their first max_var variants, if given), process-parallel over candidates on
    every usable host core, one BLAS thread per process.  Returns (baseline dict,
    per-candidate oracle results for the error report)."""
    import multiprocessing as mp
    from oracle import dcflow_oracle as O
    g = w.grid
    rating = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, w.rating_scale,
                       w.rating_offset)
    cores = host_cores()["usable"]
    def xs(i):
        x = w.inj[i] if not w.inj_shared else w.inj
        return x[:max_var] if max_var else x
    # with fewer candidates than cores, each candidate's variants are split into
    # chunks (each chunk repeats the candidate's factorisation, as the oracle does)
    n_var = xs(0).shape[0] if n_sample else 0
    per = max(1, -(-cores // max(1, n_sample)))          # chunks per candidate
    step = max(1, -(-n_var // per))
    jobs, owner = [], []
    for i in range(n_sample):
        x = xs(i)
        for v0 in range(0, x.shape[0], step):
            jobs.append((g.n_bus, g.f, g.t, g.b, g.slack, w.cands.elements(i), x[v0:v0 + step],
                         w.mon, w.out, rating, getattr(w, "controls", None),
                         getattr(w, "gens", None), getattr(w, "multi", None), keep_rows))
            owner.append(i)
    # fresh interpreters (this process may already hold the GPU); started and warmed
    # up before the clock runs
    ctx = mp.get_context("spawn")
    nproc = min(cores, max(1, len(jobs)))
    with ctx.Pool(nproc) as pool:
        pool.map(_warm, range(nproc), chunksize=1)
        t0 = time.perf_counter()
        parts = pool.map(_oracle_worker, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    # the chunks of a candidate back together (variants in order)
    outs = []
    for i in range(n_sample):
        mine = [parts[j] for j in range(len(jobs)) if owner[j] == i]
        res = dict(mine[0][1])
        res["max_load"] = np.concatenate([np.atleast_1d(m[1]["max_load"]) for m in mine])
        if "p0" in res:
            res["p0"] = np.concatenate([m[1]["p0"] for m in mine], axis=0)
        outs.append((sum(m[0] for m in mine), res))
    lf = sum(o[0] for o in outs)
    base = dict(value=lf / dt, unit="loadflows/s", cores=nproc,
                kind="oracle",
                sample=f"first {n_sample} of {w.cands.n_cand} candidates of the same workload"
                       + (f", first {max_var} of {w.n_var} variants" if max_var else "")
                       + f" ({lf} loadflows, {dt:.1f} s wall)",
                host=host_cores())
    return base, [o[1] for o in outs], rating


# ------------------------------------------------------------------ GPU timing

def _source_hash():
    h = hashlib.sha256()
    for name in ("score.hip", "dcflow_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2501_17529_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def run_path(D, torch, plan, w, prec, steps, warmup, tune=True, graph=True, persistent=False,
             tune_cache=None, agg_i=True, tuning=None):
    nv = w.n_var
    bt = D.Batch(plan, w.cands, nv)
    if persistent:
        bt.set_tuning(persistent=1)
    if tuning:
        bt.set_tuning(**tuning)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows, _ = bt.flow_buffer(nv, prec)
    out = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()   # a non-null stream: graphs are captured from it
    res = {}
    with torch.cuda.stream(stream):
        def step(ev=None):
            if ev:
                ev[0].record(stream)
            bt.eval_topologies()
            if ev:
                ev[1].record(stream)
            bt.eval_injections(x, nv, w.inj_shared, prec, flows=flows)
            if ev:
                ev[2].record(stream)
            bt.n1_score(flows, nv, prec, out=out)
            if ev:
                ev[3].record(stream)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if tune:
            from paper_2501_17529_amd import autotune
            if tune_cache:
                os.environ["DCFLOW_AUTOTUNE_CACHE"] = tune_cache
            cfg, times = autotune.tune_scan(bt, flows, nv, prec, use_cache=bool(tune_cache))
            res["tuning"] = cfg
            step()
        # eager steps, phase by phase
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(evs[i])
        torch.cuda.synchronize()
        res["wall_eager"] = time.perf_counter() - t0
        res["phase_ms"] = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]),
                                     e[2].elapsed_time(e[3])] for e in evs]).mean(axis=0)
        sc_eager = D.Batch.scores_to_numpy(out, bt.n_cand)
        res["wall"] = res["wall_eager"]
        if graph:
            # the whole step captured once, replayed with one launch per step; for
            # per-candidate injections the step's candidate chunks (GEMM of one
            # chunk beside the scan of the previous) are chosen by timing replays
            base_cfg = bt.get_tuning()
            chunk_ms = {}
            for ch in ((1, 2, 4, 8) if tune and not w.inj_shared else (base_cfg["step_chunks"],)):
                bt.set_tuning(**dict(base_cfg, step_chunks=ch))
                bt.capture(x, nv, w.inj_shared, prec, flows, out, stream)
                for _ in range(2):
                    bt.replay(stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(5):
                    bt.replay(stream)
                e1.record(stream)
                e1.synchronize()
                chunk_ms[ch] = e0.elapsed_time(e1) / 5
            best = min(chunk_ms, key=chunk_ms.get)
            res["step_chunks"] = best
            res["step_chunk_ms"] = chunk_ms
            bt.set_tuning(**dict(base_cfg, step_chunks=best))
            bt.capture(x, nv, w.inj_shared, prec, flows, out, stream)
            for _ in range(warmup):
                bt.replay(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                bt.replay(stream)
            torch.cuda.synchronize()
            res["wall_graph"] = time.perf_counter() - t0
            sc = D.Batch.scores_to_numpy(out, bt.n_cand)
            for k in ("max_load", "best_variant", "worst_branch", "worst_outage"):
                assert np.array_equal(sc[k], sc_eager[k]), f"graph replay differs in {k}"
            res["wall"] = res["wall_graph"]
        if agg_i:
            # agg_i of the winners after the step (metric-first), outside the timed step:
            # the global top 16 and the two-level list (3 per case, top 16); first with
            # the record off (sweeping the winners' tiles), then from the column-maximum
            # record the winner pass keeps by default (and n1_score's time either way)
            def timed(fn, reps):
                fn()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    fn()
                e1.record(stream)
                e1.synchronize()
                return e0.elapsed_time(e1) / reps

            calls = (("global_top16", lambda: bt.n1_worst(flows, nv, prec, out, 16)),
                     ("per_case3_top16", lambda: bt.n1_worst_per_case(flows, nv, prec, out, 3, 16)))
            agg = {"sweep": {}, "record": {}}
            lists = {}
            base_cfg = bt.get_tuning()
            score = lambda: bt.n1_score(flows, nv, prec, out=out)
            bt.set_tuning(**dict(base_cfg, worst_record=-1))
            agg["n1_score_without_record_ms"] = timed(score, 5)
            for name, fn in calls:
                agg["sweep"][name] = timed(fn, 3)
                lists[name] = fn().cpu().numpy().copy()
            bt.set_tuning(**dict(base_cfg, worst_record=0))
            agg["n1_score_ms"] = timed(score, 5)
            for name, fn in calls:
                agg["record"][name] = timed(fn, 3)
                assert np.array_equal(fn().cpu().numpy(), lists[name]), \
                    f"agg_i from the record differs ({name})"
            bt.set_tuning(**base_cfg)
            score()
            torch.cuda.synchronize()  # the maxima below are read on another stream
            res["agg_i_ms"] = agg
    res["scores"] = sc_eager
    res["batch"] = bt
    res["flows"] = flows
    res["vmax"] = bt.variant_max(nv).cpu().numpy().copy()
    return res


def ti_sweep(sizes, n_cand, top_k, steps, prec):
    """|T_i| sweep with the two running modes of the injection loop (synthetic
    analogue of the paper's Fig. 2 comparison on the medium grid).  The candidates
    stay fixed; variant v of a candidate regroups its split substations' injections
    between the busbars (injection topologies) over shared nodal injections.
      metric-first: per-variant maxima, t_i*, then agg_i (top_k worst cases) for
                    t_i* only;
      output-first: the same plus agg_i for every variant, one worst-case pass per
                    variant (the winner's list included).
    Prints one JSON line per |T_i|."""
    import torch
    import gridgen as G
    from paper_2501_17529_amd import dcflow as D
    w = G.workload_medium(0, n_cand=n_cand, n_var=1)
    plan = D.Plan.from_workload(w)
    n_out = len(w.out)
    for nv in sizes:
        rng = np.random.default_rng(100 + nv)
        bt = D.Batch(plan, w.cands, nv)
        pnv = torch.from_numpy(G.busbar_injection_topologies(w.grid, w.cands, rng, nv)).cuda()
        bt.set_busbar_injections(pnv, nv)
        x = torch.from_numpy(np.repeat(G.balanced(w.grid.p, w.grid.slack)[None], nv, 0)).cuda()
        flows, _ = bt.flow_buffer(nv, prec)
        sc = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        cases = torch.empty(bt.n_cand * top_k * D.CASE_DTYPE.itemsize, dtype=torch.uint8,
                            device="cuda")

        def front():
            bt.eval_topologies()
            bt.eval_injections(x, nv, True, prec, flows=flows)
            bt.n1_score(flows, nv, prec, out=sc)

        front()
        torch.cuda.synchronize()
        # score records naming each variant as the one to list (status kept, so
        # disconnected candidates stay skipped)
        per_v = []
        for v in range(nv):
            s_v = sc.clone()
            iv = s_v.view(torch.int32).view(bt.n_cand, D.SCORE_DTYPE.itemsize // 4)
            iv[:, 4] = torch.where(iv[:, 4] >= 0, v, iv[:, 4])
            per_v.append(s_v)

        def metric_first():
            front()
            bt.n1_worst(flows, nv, prec, sc, top_k, out=cases)

        def output_first():
            front()
            for v in range(nv):
                bt.n1_worst(flows, nv, prec, per_v[v], top_k, out=cases)

        res = {}
        for name, fn in (("metric_first", metric_first), ("output_first", output_first)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) / steps * 1e3
        n_lf = bt.n_cand * nv * n_out
        print(json.dumps({
            "ti": nv, "candidates": bt.n_cand, "top_k": top_k, "prec": prec,
            "metric_first_ms": res["metric_first"], "output_first_ms": res["output_first"],
            "metric_first_loadflows_per_s": n_lf / (res["metric_first"] / 1e3),
            "output_first_loadflows_per_s": n_lf / (res["output_first"] / 1e3),
            "metric_first_us_per_injection": res["metric_first"] * 1e3 / (bt.n_cand * nv),
            "output_first_us_per_injection": res["output_first"] * 1e3 / (bt.n_cand * nv),
        }), flush=True)
        del bt, flows, per_v, pnv, x


def rank_sweep(ks, n_cand, steps, prec):
    """Disconnection sweep (synthetic analogue of the paper's comparison of repeated
    LODF and MODF over the number of disconnections): n_cand candidates of k
    remedial outages each (drawn among the medium grid's non-bridges), |T_i| = 1,
    N-1 over its 500 contingencies.  The k outages of a candidate are joined into
    one k x k correction (the MODF form).  Prints one JSON line per k: the branch
    module (eval_topologies) and the whole step."""
    import torch
    import gridgen as G
    from paper_2501_17529_amd import dcflow as D
    w = G.workload_medium(0, n_cand=1, n_var=1)
    plan = D.Plan.from_workload(w)
    rng = np.random.default_rng(11)
    pool = G.non_bridges(w.grid, rng, 800)
    x = torch.from_numpy(G.balanced(w.grid.p, w.grid.slack)[None]).cuda()
    for k in ks:
        lists = [[(G.KIND_OUTAGE, int(l), 0, 0.0) for l in rng.choice(pool, size=k, replace=False)]
                 for _ in range(n_cand)]
        bt = D.Batch(plan, G.Candidates.from_lists(lists), 1)
        flows, _ = bt.flow_buffer(1, prec)
        out = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

        def branch():
            bt.eval_topologies()

        def step():
            bt.eval_topologies()
            bt.eval_injections(x, 1, True, prec, flows=flows)
            bt.n1_score(flows, 1, prec, out=out)

        res = {}
        for name, fn in (("branch_module", branch), ("step", step)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) / steps * 1e3
        sc = D.Batch.scores_to_numpy(out, bt.n_cand)
        print(json.dumps({
            "disconnections": k, "candidates": bt.n_cand, "prec": prec,
            "branch_module_ms": res["branch_module"], "step_ms": res["step"],
            "branch_module_us_per_topology": res["branch_module"] * 1e3 / bt.n_cand,
            "islanded_candidates": int((sc["status"] & 1).sum()),
        }), flush=True)
        del bt, flows


WORKLOADS = {
    "medium": ("medium-1000bus: 1,000 buses / 1,600 branches, 4,096 candidates (1-3 bus splits + "
               "0-2 outages), 16 injection variants each, N-1 over 500 contingencies = monitored "
               "branches"),
    "uneven": ("uneven-10000bus: 10,000 buses / 15,500 branches, {n} candidates of rank uniform "
               "in 1..8, 1 injection each, every branch monitored, N-1 over 2,000 contingencies"),
    "brute": ("brute-2000bus: 2,000 buses / 3,100 branches with 20 phase shifters and 4 HVDC "
              "links, {n} topologies x 4,096 shared control/load combinations (one GEMM over the "
              "combinations, control columns folded into K), every branch monitored, N-1 over "
              "1,000 contingencies"),
    "tiny": ("tiny-30bus: 30 buses / 41 branches, 100 single-split candidates, 1 injection, N-1 "
             "over all 41 branches"),
}

# MI355X peaks (TFLOP/s).  VALU: 256 CU x 4 SIMD x 16 lanes x 2 flops (one FMA) x 2.4 GHz for
# the unpacked FP32 and the FP64 FMA alike; MFMA: the published dense figures.
PEAK = {"valu": PEAK_VALU_FMA_TFLOPS, "mfma_fp64": 78.6, "mfma_fp32": 157.3, "mfma_bf16": 2500.0}
HBM_GBS = 8000.0
PREC_DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x6": "f32 scan, bf16x6 GEMM", "bf16": "bf16"}


def ranks(w):
    return np.diff(np.asarray(w.cands.off))


# VALU lane instructions per N-1 element of one variant that the sweep cannot do
# without: one FMA for p = F~ + L~ y and its share of the running maximum of |p|
# (FP32: a three-input max with absolute-value operands takes two elements; FP64
# has no such instruction: one two-input max per element, |.| being free).
SWEEP_OPS = {"fp64": 2.0, "fp32": 1.5, "bf16x6": 1.5}


def scan_roofline(w, prec, scan_ms, traffic=None):
    """The N-1 scan (a5) against a combined VALU + matrix-core bound.  The sweep:
    every (monitored row, contingency) element of every variant costs SWEEP_OPS
    VALU lane instructions at the issue rate of 256 CU x 64 lanes x 2.4 GHz (its
    FMA is 2 of the flops counted).  The LODF' tile build: k FMAs per element of a
    candidate of rank k on the matrix cores of the scan's precision, once for the
    variants' maxima and once for the winner (once when there is one variant).
    t_ideal = sweep ops / issue rate + build flops / MFMA peak; frac = t_ideal / t;
    achieved = (sweep FMA flops + build flops) / t and peak = the same / t_ideal."""
    n_ctg = len(w.out) + (0 if w.gens is None else len(w.gens[0]))
    per_pair = float(len(w.mon)) * n_ctg
    n_el = per_pair * w.cands.n_cand * w.n_var
    builds = 1 if w.n_var == 1 else 2
    build_flops = 2.0 * per_pair * float(ranks(w).sum()) * builds
    sweep_flops = 2.0 * n_el
    issue = PEAK_VALU_FMA_TFLOPS / 2 * 1e12          # lane instructions per second
    mfma = PEAK["mfma_fp64"] if prec == "fp64" else PEAK["mfma_fp32"]
    t_ideal = SWEEP_OPS["fp64" if prec == "fp64" else "fp32"] * n_el / issue \
        + build_flops / (mfma * 1e12)
    t = scan_ms / 1e3
    flops = sweep_flops + build_flops
    return {"bound": "alu", "kernel": f"n1_score {prec} (k_scan_max + k_scan_win"
            + (" + error guard" if prec != "fp64" else "") + ")",
            "achieved": flops / t / 1e12, "peak": flops / t_ideal / 1e12, "unit": "TFLOP/s",
            "frac": t_ideal / t, "traffic": traffic, "flops_per_call": flops,
            "t_ideal_ms": t_ideal * 1e3, "sweep_ops_per_element": SWEEP_OPS[
                "fp64" if prec == "fp64" else "fp32"],
            "build_flops": build_flops, "ms_per_call": scan_ms}


def gemm_roofline(w, plan, prec, inj_ms):
    """The injection step (a4): per-candidate injections are one GEMM of the kept
    PTDF rows with every (candidate, variant) column, against the matrix-core peak
    of its precision (BF16X6: six BF16 products per output); shared injections
    (the brute-force workload) are one small GEMM and a broadcast of the flows to
    every topology, bound by writing those flows."""
    v = plan.view
    n_inj = v.n_inj
    if w.inj_shared:
        nbytes = float(w.cands.n_cand) * w.n_var * v.n_er * (8 if prec == "fp64" else 4)
        achieved = nbytes / (inj_ms / 1e3) / 1e9
        return {"bound": "hbm", "kernel": f"eval_injections {prec} (shared GEMM + k_bcast)",
                "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s", "frac": achieved / HBM_GBS,
                "traffic": None, "bytes_per_call": nbytes, "ms_per_call": inj_ms}
    cols = float(w.cands.n_cand) * w.n_var
    mult = 6.0 if prec == "bf16x6" else 1.0
    flops = 2.0 * v.n_er * n_inj * cols * mult
    peak = {"fp64": PEAK["mfma_fp64"], "fp32": PEAK["mfma_fp32"]}.get(prec, PEAK["mfma_bf16"])
    achieved = flops / (inj_ms / 1e3) / 1e12
    return {"bound": "mfma", "kernel": f"eval_injections {prec} (k_sense + GEMM)",
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None, "flops_per_call": flops, "ms_per_call": inj_ms}


def oracle_error(w, plan, r, oracle_res):
    """Error of a path against the oracle on the sampled candidates (the first
    len(oracle_res)): per-variant maxima, islanding counts and the N-0 flows of the
    kept rows, in rating units (kept rows outside the monitored set: p.u.)."""
    if not oracle_res:
        return None
    sc = r["scores"]
    nv = w.n_var
    bt = r["batch"]
    fl = bt.flows_view(r["flows"], nv)
    n_er = plan.view.n_er
    er_mon = len(w.mon)
    from oracle import dcflow_oracle as O
    g = w.grid
    rating = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, w.rating_scale,
                       w.rating_offset)
    rr = np.concatenate([rating, np.ones(n_er - er_mon)])
    vm_err, fl_err, n_isl_bad = 0.0, 0.0, 0
    for i, o in enumerate(oracle_res):
        if not np.all(np.isfinite(o["max_load"])):
            continue
        vm_err = max(vm_err, float(np.abs(r["vmax"][i][:len(o["max_load"])] - o["max_load"]).max()))
        n_isl_bad += int((int(sc["status"][i]) >> 8) != o["n_island"])
        if "p0" in o:
            gf = fl[i].double().cpu().numpy()[:len(o["p0"]), :n_er]
            fl_err = max(fl_err, float((np.abs(gf - o["p0"]) / rr).max()))
    return {"candidates": len(oracle_res), "variant_max_abs": vm_err,
            "n0_flows_rel_rating": fl_err, "island_count_mismatches": n_isl_bad}


def kept_rows(w):
    mon = [int(x) for x in w.mon]
    ms = set(mon)
    return np.asarray(mon + [int(o) for o in w.out if int(o) not in ms], np.int64)


def path_summary(w, plan, r, prec, steps, n_lf, oracle_res, traffic=None, ref=None):
    ms = r["wall"] / steps * 1e3
    ph = r["phase_ms"]
    out = {"value": n_lf / (ms / 1e3), "ms_per_step": ms, "dtype": PREC_DTYPE[prec],
           "phase_ms": {"eval_topologies": float(ph[0]), "eval_injections": float(ph[1]),
                        "n1_score": float(ph[2])},
           "roofline": {"scan": scan_roofline(w, prec, float(ph[2]), traffic),
                        "injections": gemm_roofline(w, plan, prec, float(ph[1]))},
           "tuning": r.get("tuning"), "step_chunks": r.get("step_chunks"),
           "agg_i_ms": r.get("agg_i_ms"),
           "step_mode": "hip graph replay" if "wall_graph" in r else "eager"}
    if prec != "fp64":
        out["guarded_candidates"] = int(((r["scores"]["status"] & 8) != 0).sum())
    if ref is not None:
        d = np.abs(r["scores"]["max_load"] - ref["scores"]["max_load"])
        d = d[np.isfinite(d)]
        out["vs_fp64_path"] = {"max_load_absdiff_max": float(d.max()) if len(d) else 0.0,
                               "candidates_over_1e-4": int((d > 1e-4).sum()),
                               "max_load_absdiff_median": float(np.median(d)) if len(d) else 0.0}
    out["oracle_error"] = oracle_error(w, plan, r, oracle_res)
    return out


def protocol(bt_replay, runs, min_s, n_lf):
    """Repeated timed runs of graph replays, each at least min_s seconds."""
    import torch
    vals = []
    for _ in range(runs):
        n = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            for _ in range(20):
                bt_replay()
            n += 20
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if dt >= min_s:
                break
        vals.append(n_lf * n / dt)
    return {"runs": runs, "seconds_per_run": min_s, "mean": float(np.mean(vals)),
            "median": float(np.median(vals)), "min": float(np.min(vals)),
            "max": float(np.max(vals)), "unit": "loadflows/s"}


def end_to_end(D, torch, w, prec):
    """One cold pass including the one-time base build, the host-to-device copies
    of the grid, candidates and injections, the step and the copy of the scores
    back (pageable host memory, as a caller would hold it)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = D.Plan.from_workload(w)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bt = D.Batch(plan, w.cands, w.n_var)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bt.eval_topologies()
    flows = bt.eval_injections(x, w.n_var, w.inj_shared, prec)
    out = bt.n1_score(flows, w.n_var, prec)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sc = D.Batch.scores_to_numpy(out, bt.n_cand)
    t4 = time.perf_counter()
    n_lf = w.cands.n_cand * w.n_var * len(w.out)
    tot = t4 - t0
    res = {"prec": prec, "build_s": t1 - t0, "h2d_s": t2 - t1, "step_s": t3 - t2,
           "d2h_s": t4 - t3, "total_s": tot, "loadflows_per_s": n_lf / tot,
           "h2d_bytes": int(x.numel() * 8), "candidates_scored": int(len(sc))}
    del bt, flows, x, out, plan
    return res


def section_tiny(D, torch, steps):
    import gridgen as G
    w = G.workload_tiny(0)
    plan = D.Plan.from_workload(w)
    r = run_path(D, torch, plan, w, "fp64", steps, 3, tune=False, agg_i=False)
    ms = r["wall"] / steps * 1e3
    n_lf = w.cands.n_cand * w.n_var * len(w.out)
    return {"workload": WORKLOADS["tiny"], "prec": "fp64", "ms_per_step": ms,
            "us_per_candidate": ms * 1e3 / w.cands.n_cand, "value": n_lf / (ms / 1e3),
            "unit": "loadflows/s", "step_mode": "hip graph replay",
            "note": "launch-latency bound: 100 candidates fill a fraction of one launch"}


def section_uneven(D, torch, n_cand, steps, cpu_n, out_log):
    """The 10,000-bus uneven-rank batch at its full size on one GPU: each path is
    captured into a HIP graph (its replay checked against the eager scores) and
    timed in replay, with the row bands the autotuner picks on this batch."""
    import gridgen as G
    t0 = time.perf_counter()
    w = G.workload_uneven(0, n_cand=n_cand)
    gen_s = time.perf_counter() - t0
    out_log(f"uneven: {n_cand} candidates generated in {gen_s:.0f} s")
    cpu, ores = (None, [])
    if cpu_n:
        cpu, ores, _ = cpu_baseline(w, cpu_n, keep_rows=kept_rows(w))
        out_log(f"uneven: oracle sample done ({cpu['sample']})")
    t0 = time.perf_counter()
    plan = D.Plan.from_workload(w)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    n_lf = w.cands.n_cand * w.n_var * len(w.out)
    res, paths = {}, {}
    tun = {"fp64": dict(scan_band=0), "fp32": dict(scan_band=512), "bf16x6": dict(scan_band=512)}
    for prec in ("fp64", "fp32", "bf16x6"):
        r = run_path(D, torch, plan, w, prec, steps, 1, tune=False, graph=True, agg_i=False,
                     tuning=tun[prec])
        paths[prec] = path_summary(w, plan, r, prec, steps, n_lf, ores,
                                   ref=res.get("fp64"))
        paths[prec]["tuning"] = tun[prec]
        out_log(f"uneven {prec}: {paths[prec]['ms_per_step']:.1f} ms per step")
        # keep the FP64 scores for the comparison; free the batch and flows
        res[prec] = {"scores": r["scores"]}
        del r
        torch.cuda.empty_cache()
    ml = res["fp64"]["scores"]["max_load"]
    k = ranks(w)
    return {"workload": WORKLOADS["uneven"].format(n=f"{n_cand:,}"), "candidates": n_cand,
            "rank_counts": {int(q): int((k == q).sum()) for q in range(1, 9)},
            "generate_s": gen_s, "build_ptdf_s": build_s, "loadflows_per_step": n_lf,
            "value": paths["fp64"]["value"], "dtype": "f64", "paths": paths,
            "fp64_max_load_range": [float(np.min(ml)), float(np.max(ml[np.isfinite(ml)]))],
            "cpu_baseline": cpu,
            "device_bytes_note": "one batch of 65,536 candidates holds about 80 GB of factors "
                                 "(U FP64 37 GB, U/r FP32 18 GB, W 7 GB, BF16 parts 4 GB) plus "
                                 "8 GB of FP64 flows and 5 GB of injections"}


def section_brute(D, torch, n_topo, steps, cpu_n, out_log):
    import gridgen as G
    w = G.workload_brute(0, n_topo=n_topo)
    cpu, ores = (None, [])
    if cpu_n:
        cpu, ores, _ = cpu_baseline(w, cpu_n, max_var=128)
        out_log(f"brute: oracle sample done ({cpu['sample']})")
    plan = D.Plan.from_workload(w)
    n_lf = w.cands.n_cand * w.n_var * len(w.out)
    res, paths = {}, {}
    for prec in ("fp32", "bf16x6", "fp64"):
        r = run_path(D, torch, plan, w, prec, steps, 1, tune=False, graph=False, agg_i=False)
        paths[prec] = path_summary(w, plan, r, prec, steps, n_lf, [],
                                   ref=None)
        res[prec] = {"scores": r["scores"]}
        if ores:
            # the oracle sample holds the first 128 combinations of each sampled topology
            errs = [float(np.abs(r["vmax"][i][:len(o["max_load"])] - o["max_load"]).max())
                    for i, o in enumerate(ores) if np.all(np.isfinite(o["max_load"]))]
            paths[prec]["oracle_error"] = {"topologies": len(ores), "combinations": 128,
                                           "variant_max_abs": max(errs) if errs else None}
        out_log(f"brute {prec}: {paths[prec]['ms_per_step']:.1f} ms per step")
        del r
        torch.cuda.empty_cache()
    for prec in ("fp32", "bf16x6"):
        d = np.abs(res[prec]["scores"]["max_load"] - res["fp64"]["scores"]["max_load"])
        d = d[np.isfinite(d)]
        paths[prec]["vs_fp64_path"] = {"max_load_absdiff_max": float(d.max()),
                                       "candidates_over_1e-4": int((d > 1e-4).sum())}
    return {"workload": WORKLOADS["brute"].format(n=f"{n_topo:,}"), "topologies": n_topo,
            "loadflows_per_step": n_lf, "value": paths["fp64"]["value"], "dtype": "f64",
            "paths": paths, "cpu_baseline": cpu}


def section_proposal(D, torch, reps=5):
    """The learned proposal on the medium grid: per held-out load snapshot, features
    of every single-split action, standardisation, fused BF16 inference, top-512
    and the exact screen of those 512, against the exhaustive exact screen of every
    action; and one training epoch (forward, backward, Adam) over 2 snapshots'
    actions.  Timing only (random-initialised weights; the gain is a GPU test)."""
    import gridgen as G
    from paper_2501_17529_amd import proposal as PR
    w = G.workload_medium(0, n_cand=4, n_var=1)
    g = w.grid
    plan = D.Plan.from_workload(w)
    rng = np.random.default_rng(9)
    xs = G.perturbed_injections(g, rng, (3,), 0.2)
    bus, mask, side = PR.enumerate_actions(g)
    na = len(bus)
    prop = PR.Proposal(plan, seed=1)
    x_dev, flows, glob = prop.snapshot_summary(xs)
    snap2 = np.repeat(np.arange(2, dtype=np.int32), na)
    act2 = np.tile(np.arange(na), 2)
    feat_t = prop.features(x_dev, flows, glob, snap2, bus[act2], mask[act2], side[act2])
    yt = torch.zeros(feat_t.shape[0], dtype=torch.float32, device="cuda")
    prop.set_standardization(feat_t, yt + 1.0)
    prop.standardize(feat_t)
    prop.pack()
    s = 2

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    st = {}

    def feats():
        st["f"] = prop.features(x_dev, flows, glob, np.full(na, s, np.int32), bus, mask, side)
        prop.standardize(st["f"])
    t_feat = timed(feats)
    t_inf = timed(lambda: st.__setitem__("y", prop.infer(st["f"])))
    t_top = timed(lambda: st.__setitem__("top", PR.topk_smallest(st["y"], 512)))
    top = st["top"].cpu().numpy()
    c512 = PR.action_candidates(bus[top], mask[top], side[top], xs[s])
    call = PR.action_candidates(bus, mask, side, xs[s])
    t_ver = timed(lambda: PR.exact_scores(plan, c512, xs[s]))
    t_exh = timed(lambda: PR.exact_scores(plan, call, xs[s]))
    t_epoch = timed(lambda: prop.train(feat_t, yt, epochs=1, batch=1024))
    n_train = (feat_t.shape[0] // 1024) * 1024
    flops_fwd = 2.0 * (96 * 256 + 256 * 256 + 256)
    return {"actions": na, "features_ms": t_feat, "infer_ms": t_inf, "topk512_ms": t_top,
            "verify512_ms": t_ver, "exhaustive_ms": t_exh,
            "proposal_pipeline_ms": t_feat + t_inf + t_top + t_ver,
            "infer_tflops": flops_fwd * na / (t_inf / 1e3) / 1e12,
            "train_epoch_ms": t_epoch, "train_samples": n_train,
            "train_tflops": 3 * flops_fwd * n_train / (t_epoch / 1e3) / 1e12,
            "note": "exact-solver calls include their host-side batch set-up; the proposal's "
                    "gain is measured in exact evaluations by the GPU test"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="medium")
    ap.add_argument("--cands", type=int, default=0, help="candidates (default: 4,096 medium, "
                    "65,536 uneven, 1,024 brute)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample size (default: 128 medium, 16 uneven, 1 brute)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", choices=["all", "fp32", "fp64", "bf16x6", "bf16"], default="all")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="the medium workload only: no other configurations, no repeated-run "
                         "protocol, no end-to-end pass")
    ap.add_argument("--protocol-runs", type=int, default=5)
    ap.add_argument("--protocol-s", type=float, default=10.0)
    ap.add_argument("--tune-cache", default="", metavar="PATH",
                    help="autotuner cache file: shapes found there are reused without a sweep "
                         "(so that a profiled run times the same launch shapes as the bench run)")
    ap.add_argument("--n1-extras", default="", metavar="G,Q",
                    help="add G generator outages and Q multi-outage cases (2-4 contingency "
                         "branches each) to the N-1 set of the workload")
    ap.add_argument("--rank-sweep", default="", metavar="KS",
                    help="only run the disconnection sweep for the comma-separated numbers of "
                         "remedial outages per candidate (1..8)")
    ap.add_argument("--ti-sweep", default="", metavar="SIZES",
                    help="only run the |T_i| sweep, metric-first vs output-first, for the "
                         "comma-separated numbers of injection topologies per candidate")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three plain device copies of MIB MiB (HBM counter scale)")
    ap.add_argument("--plan-builds", type=int, default=0, metavar="N",
                    help="only build the workload's plan N times in a row and print the wall "
                         "time of each (one-time FP64 base, host set-up included)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path here "
              "(candidates would shard across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

    def log(msg):
        print(f"[bench {time.perf_counter() - t_start:6.1f} s] {msg}", file=sys.stderr, flush=True)

    if a.copy_calibration:
        import torch
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 3}))
        return

    if a.plan_builds:
        import torch
        import gridgen as G
        from paper_2501_17529_amd import dcflow as D
        torch.cuda.init()
        wl = {"medium": lambda: G.workload_medium(0, n_cand=16),
              "uneven": lambda: G.workload_uneven(0, n_cand=16),
              "brute": lambda: G.workload_brute(0, n_topo=2, n_comb=4),
              "tiny": lambda: G.workload_tiny(0)}[a.workload]()
        times = []
        for _ in range(a.plan_builds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = D.Plan.from_workload(wl)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            del plan
        print(json.dumps({"workload": a.workload, "n_bus": int(wl.grid.n_bus),
                          "n_branch": int(wl.grid.n_branch), "plan_build_ms": times}))
        return

    if a.rank_sweep:
        rank_sweep([int(v) for v in a.rank_sweep.split(",")], a.cands or 4096, a.steps,
                   "fp32" if a.prec == "all" else a.prec)
        return
    if a.ti_sweep:
        ti_sweep([int(v) for v in a.ti_sweep.split(",")], a.cands or 512, 16, a.steps,
                 "fp32" if a.prec == "all" else a.prec)
        return

    import gridgen as G
    if a.workload != "medium":
        # one of the other configurations alone, as its own line
        import torch
        from paper_2501_17529_amd import dcflow as D
        torch.cuda.init()
        if a.workload == "uneven":
            sec = section_uneven(D, torch, a.cands or 65536, a.steps,
                                 0 if a.no_cpu_baseline else (a.cpu_sample or 16), log)
        elif a.workload == "brute":
            sec = section_brute(D, torch, a.cands or 1024, a.steps,
                                0 if a.no_cpu_baseline else (a.cpu_sample or 1), log)
        else:
            sec = section_tiny(D, torch, a.steps)
        sec["wall_s"] = time.perf_counter() - t_start
        print(json.dumps(sec), flush=True)
        return

    w = G.workload_medium(0, n_cand=a.cands or 4096)
    precs = ["fp64", "fp32", "bf16x6"] if a.prec == "all" else [a.prec]
    sample = a.cpu_sample or 128
    if a.n1_extras:
        n_g, n_q = (int(v) for v in a.n1_extras.split(","))
        rng = np.random.default_rng(77)
        w.gens = G.generator_outages(w.grid, rng, n_g) if n_g else None
        w.multi = G.multi_outage_cases(w.grid, w.out, rng, n_q) if n_q else None
    cpu, ores = None, []
    if not a.no_cpu_baseline:
        cpu, ores, _ = cpu_baseline(w, min(sample, w.cands.n_cand), keep_rows=kept_rows(w))
        log(f"medium: oracle sample done ({cpu['sample']})")

    import torch
    from paper_2501_17529_amd import dcflow as D
    torch.cuda.init()
    t0 = time.perf_counter()
    plan = D.Plan.from_workload(w)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0

    n_extra = (0 if w.gens is None else len(w.gens[0])) + (0 if w.multi is None else len(w.multi))
    n_lf = w.cands.n_cand * w.n_var * (len(w.out) + n_extra)
    traffic = None
    if not a.n1_extras and os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("source_hash") == _source_hash():
            traffic = tf
    res, paths = {}, {}
    for prec in precs:
        res[prec] = run_path(D, torch, plan, w, prec, a.steps, a.warmup,
                             tune=not a.no_autotune, tune_cache=a.tune_cache or None,
                             graph=not a.no_graph)
        tr = traffic.get("bytes_per_launch") if traffic and traffic.get("prec") == prec else None
        paths[prec] = path_summary(w, plan, res[prec], prec, a.steps, n_lf, ores, traffic=tr,
                                   ref=res.get("fp64"))
        log(f"medium {prec}: {paths[prec]['ms_per_step']:.3f} ms per step")
    main_prec = precs[0]
    r = res[main_prec]
    mp_ = paths[main_prec]
    proto = None
    if not a.quick and a.protocol_runs > 0 and "wall_graph" in r:
        bt = r["batch"]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            proto = protocol(lambda: bt.replay(stream), a.protocol_runs, a.protocol_s, n_lf)
        log(f"protocol: mean {proto['mean']:.3e} loadflows/s")
    g = w.grid
    line = {
        "metric": METRIC, "value": mp_["value"], "unit": "loadflows/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": mp_["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": PREC_DTYPE[main_prec], "data": "synthetic",
        "config": {"workload": WORKLOADS["medium"],
                   "n_bus": g.n_bus, "n_branch": g.n_branch, "candidates": w.cands.n_cand,
                   "variants": w.n_var, "contingencies": len(w.out), "monitored": len(w.mon),
                   "loadflows_per_step": n_lf, "parallelism": "single GPU",
                   **({"generator_outages": len(w.gens[0]) if w.gens is not None else 0,
                       "multi_outage_cases": len(w.multi) if w.multi is not None else 0}
                      if a.n1_extras else {})},
        # the dominant kernel of the headline path: its N-1 scan
        "roofline": None if a.n1_extras else {
            k: v for k, v in mp_["roofline"]["scan"].items()
            if k in ("bound", "kernel", "achieved", "peak", "unit", "frac", "traffic")},
        "paths": paths,
        "build_ptdf_s": build_s,
    }
    for p in precs:
        for key in ("batch", "flows"):
            res[p].pop(key, None)
    del res
    torch.cuda.empty_cache()
    if not a.quick:
        line["end_to_end"] = end_to_end(D, torch, w, main_prec)
        log("end-to-end pass done")
    line["protocol"] = proto
    if not a.quick:
        cfgs = {}
        cfgs["tiny"] = section_tiny(D, torch, a.steps)
        log("tiny done")
        cfgs["proposal"] = section_proposal(D, torch)
        log("proposal done")
        cfgs["brute"] = section_brute(D, torch, 1024, 2, 0 if a.no_cpu_baseline else 1, log)
        cfgs["uneven"] = section_uneven(D, torch, 65536, 2, 0 if a.no_cpu_baseline else 16, log)
        line["configs"] = cfgs
    line["cpu_baseline"] = cpu
    line["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
