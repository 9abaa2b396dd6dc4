"""Benchmark of the batched DC-loadflow screen on one MI355X.

One step = the whole hot path over one batch of the medium workload
(1,000-bus / 1,600-branch synthetic grid, 4,096 topology candidates with 1-3
bus splits plus 0-2 outages, 16 load-perturbed injection variants each, N-1
over 500 contingency branches that are also the monitored set):
dcflow_eval_topologies -> dcflow_eval_injections -> dcflow_n1_score, with the
candidate records and injections already resident in device memory.

value = N-1 loadflows per second of the mixed path (FP32 MFMA GEMM and FP32
N-1 scan, FP64 k x k solves / LODF denominators / LODF' tile build);
loadflows = candidates x variants x contingencies per step.  The plain FP64
path is timed the same way and reported beside it.

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


def _oracle_worker(args):
    from threadpoolctl import threadpool_limits
    from oracle import dcflow_oracle as O
    n_bus, f, t, b, slack, elems, x, mon, out, rating, controls, gens, multi = args
    kw = dict(gens=gens, multi=multi)
    if controls:
        kw.update(controls=controls, ctrl=x[:, n_bus:])
        x = x[:, :n_bus]
    with threadpool_limits(limits=1):
        O.score_candidate(n_bus, f, t, b, slack, elems, x, mon, out, rating, **kw)
    n_extra = (0 if gens is None else len(gens[0])) + (0 if multi is None else len(multi))
    return x.shape[0] * (len(out) + n_extra)


def cpu_baseline(w, n_sample: int, max_var: int = 0):
    """The oracle (dense LU per candidate) on the first n_sample candidates (and
    their first max_var variants, if given), process-parallel over candidates,
    one BLAS thread per process."""
    import multiprocessing as mp
    from oracle import dcflow_oracle as O
    g = w.grid
    rating = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, w.rating_scale,
                       w.rating_offset)
    cores = host_cores()["usable"]
    def xs(i):
        x = w.inj[i] if not w.inj_shared else w.inj
        return x[:max_var] if max_var else x
    jobs = [(g.n_bus, g.f, g.t, g.b, g.slack, w.cands.elements(i), xs(i), w.mon, w.out, rating,
             getattr(w, "controls", None), getattr(w, "gens", None), getattr(w, "multi", None))
            for i in range(n_sample)]
    ctx = mp.get_context("fork")     # forked before this process touches the GPU
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        lf = sum(pool.map(_oracle_worker, jobs, chunksize=1))
    dt = time.perf_counter() - t0
    return dict(value=lf / dt, unit="loadflows/s", cores=cores, kind="oracle",
                host=host_cores(),
                sample=f"first {n_sample} of {w.cands.n_cand} candidates of the same workload"
                       + (f", first {max_var} of {w.n_var} variants" if max_var else "")
                       + f" ({lf} loadflows, {dt:.1f} s wall)")


# ------------------------------------------------------------------ GPU timing

def _source_hash():
    h = hashlib.sha256()
    for name in ("score.hip", "dcflow_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2501_17529_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def run_path(D, torch, plan, w, prec, steps, warmup, tune=True, graph=True, persistent=False,
             tune_cache=None):
    nv = w.n_var
    bt = D.Batch(plan, w.cands, nv)
    if persistent:
        bt.set_tuning(persistent=1)
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
        # agg_i of the winners after the step (metric-first), outside the timed step:
        # the global top 16 and the two-level list (3 per case, top 16)
        agg = {}
        for name, fn in (("global_top16", lambda: bt.n1_worst(flows, nv, prec, out, 16)),
                         ("per_case3_top16",
                          lambda: bt.n1_worst_per_case(flows, nv, prec, out, 3, 16))):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                fn()
            e1.record(stream)
            e1.synchronize()
            agg[name] = e0.elapsed_time(e1) / 3
        res["agg_i_ms"] = agg
    res["scores"] = sc_eager
    res["batch"] = bt
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
    "uneven": ("uneven-10000bus, one GPU's share: 10,000 buses / 15,500 branches, {n} candidates "
               "of rank uniform in 1..8 (of the 65,536-candidate batch), 1 injection each, every "
               "branch monitored, N-1 over 2,000 contingencies, persistent launch"),
    "brute": ("brute-2000bus: 2,000 buses / 3,100 branches with 20 phase shifters and 4 HVDC "
              "links, {n} topologies x 4,096 shared control/load combinations (one GEMM over the "
              "combinations, control columns folded into K), every branch monitored, N-1 over "
              "1,000 contingencies"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="medium")
    ap.add_argument("--cands", type=int, default=0, help="candidates (default: 4,096 medium, "
                    "8,192 uneven, 1,024 brute)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample size (default: 128 medium, 2 uneven, 1 brute)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", choices=["all", "fp32", "fp64", "bf16x6", "bf16"], default="all")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
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
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path here "
              "(candidates would shard across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)

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

    if a.rank_sweep:
        rank_sweep([int(v) for v in a.rank_sweep.split(",")], a.cands or 4096, a.steps,
                   "fp32" if a.prec == "all" else a.prec)
        return
    if a.ti_sweep:
        ti_sweep([int(v) for v in a.ti_sweep.split(",")], a.cands or 512, 16, a.steps,
                 "fp32" if a.prec == "all" else a.prec)
        return

    import gridgen as G
    if a.workload == "medium":
        w = G.workload_medium(0, n_cand=a.cands or 4096)
        precs = ["fp32", "fp64", "bf16x6"] if a.prec == "all" else [a.prec]
        sample = a.cpu_sample or 128
    elif a.workload == "uneven":
        w = G.workload_uneven(0, n_cand=a.cands or 8192)
        precs = ["fp32", "bf16x6"] if a.prec == "all" else [a.prec]
        sample = a.cpu_sample or 2
    else:
        w = G.workload_brute(0, n_topo=a.cands or 1024)
        precs = ["fp32", "bf16x6"] if a.prec == "all" else [a.prec]
        sample = a.cpu_sample or 1
    if a.n1_extras:
        n_g, n_q = (int(v) for v in a.n1_extras.split(","))
        rng = np.random.default_rng(77)
        w.gens = G.generator_outages(w.grid, rng, n_g) if n_g else None
        w.multi = G.multi_outage_cases(w.grid, w.out, rng, n_q) if n_q else None
    max_var = 128 if a.workload == "brute" else 0   # the oracle holds all N-1 flows at once
    cpu = None if a.no_cpu_baseline else cpu_baseline(w, min(sample, w.cands.n_cand), max_var)

    import torch
    from paper_2501_17529_amd import dcflow as D
    torch.cuda.init()
    t0 = time.perf_counter()
    plan = D.Plan.from_workload(w)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0

    n_extra = (0 if w.gens is None else len(w.gens[0])) + (0 if w.multi is None else len(w.multi))
    n_lf = w.cands.n_cand * w.n_var * (len(w.out) + n_extra)
    res = {}
    for prec in precs:
        # (brute: a sweep of launch shapes at 4,096 variants would take minutes; the
        # library's default shape is timed)
        res[prec] = run_path(D, torch, plan, w, prec, a.steps, a.warmup,
                             tune=not a.no_autotune and a.workload != "brute",
                             tune_cache=a.tune_cache or None,
                             graph=not a.no_graph, persistent=a.workload == "uneven")
    main_prec = precs[0]
    r = res[main_prec]
    ms = r["wall"] / a.steps * 1e3
    value = n_lf / (ms / 1e3)

    # roofline of the dominant kernel (the N-1 scan, both passes): 2 flops (one FMA) per N-1
    # element, (V + 1) variant sweeps (the winner is re-scanned once; with one variant the
    # winner pass is the only sweep) over E_m x O per candidate
    scan_ms = float(r["phase_ms"][2])
    sweeps = w.n_var + 1 if w.n_var > 1 else 1
    flops = 2.0 * w.cands.n_cand * sweeps * len(w.mon) * len(w.out)
    achieved = flops / (scan_ms / 1e3) / 1e12
    traffic = None
    if a.workload == "medium" and not a.n1_extras and os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("source_hash") == _source_hash() and tf.get("prec") == main_prec:
            traffic = tf.get("bytes_per_launch")
    g = w.grid
    line = {
        "metric": METRIC, "value": value, "unit": "loadflows/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": main_prec, "data": "synthetic",
        "config": {"workload": WORKLOADS[a.workload].format(n=f"{w.cands.n_cand:,}"),
                   "n_bus": g.n_bus, "n_branch": g.n_branch, "candidates": w.cands.n_cand,
                   "variants": w.n_var, "contingencies": len(w.out), "monitored": len(w.mon),
                   "loadflows_per_step": n_lf, "parallelism": "single GPU",
                   **({"generator_outages": len(w.gens[0]) if w.gens is not None else 0,
                       "multi_outage_cases": len(w.multi) if w.multi is not None else 0}
                      if a.n1_extras else {})},
        # (with --n1-extras the score also runs the multi-outage kernels: no roofline)
        "roofline": None if a.n1_extras else {
            "bound": "alu", "kernel": "k_scan (per-variant N-1 maxima + winner pass)",
            "achieved": achieved, "peak": PEAK_VALU_FMA_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_FMA_TFLOPS, "traffic": traffic},
        "phase_ms": {p: {"eval_topologies": float(v["phase_ms"][0]),
                         "eval_injections": float(v["phase_ms"][1]),
                         "n1_score": float(v["phase_ms"][2])} for p, v in res.items()},
        "build_ptdf_s": build_s,
        "step_mode": "hip graph replay" if "wall_graph" in r else "eager",
        "eager_ms_per_step": r["wall_eager"] / a.steps * 1e3,
        "scan_tuning": {p: v.get("tuning") for p, v in res.items()},
        "step_chunks": {p: v.get("step_chunks") for p, v in res.items()},
        "step_chunk_ms": {p: v.get("step_chunk_ms") for p, v in res.items()},
        "agg_i_ms": {p: v.get("agg_i_ms") for p, v in res.items()},
    }
    for p, v in res.items():
        if p == main_prec:
            continue
        msp = v["wall"] / a.steps * 1e3
        line[f"{p}_path"] = {"value": n_lf / (msp / 1e3), "ms_per_step": msp}
        if p != "bf16":
            line[f"{main_prec}_vs_{p}_max_load_absdiff"] = float(
                np.abs(r["scores"]["max_load"] - v["scores"]["max_load"]).max())
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
