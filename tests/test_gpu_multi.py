"""Multi-outage N-1 cases on the GPU (Def. eq_modf; Sec. III-C branch-module
step 5 and injection-module step 8c): per candidate and case the MODF system of
the changed grid, then the cases' flows over every monitored row, in the score
and in the worst-case lists, against the oracle's re-solved networks.  Covers
busbar-like cases that island, cases with branches the candidate removed,
generator outages beside them, one variant, row bands and candidate chunks."""
import numpy as np
import pytest

import gridgen as G

from _gpu_common import (TOL, compare, compare_worst, gpu_available, oracle_rating,
                         oracle_scores, run_gpu, say)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _workload(seed=61, n_cand=28, n_var=6, n_multi=40, n_gen=6, n_mon=130):
    rng = np.random.default_rng(seed)
    g = G.make_grid(120, 190, seed)
    out = np.sort(rng.choice(190, size=90, replace=False)).astype(np.int32)
    lists = []
    for _ in range(n_cand):
        k = int(rng.integers(1, 9))
        ns = min(int(rng.binomial(k, 0.5)), 6)
        lists.append(G.sample_candidate(g, rng, ns, k - ns))
    # remedial outages of contingency branches, so that some cases lose a branch
    for j in range(4):
        lists.append([(G.KIND_OUTAGE, int(out[3 * j]), 0, 0.0),
                      (G.KIND_OUTAGE, int(out[3 * j + 1]), 0, 0.0)])
    lists.append([])
    cands = G.Candidates.from_lists(lists)
    mon = np.sort(rng.choice(190, size=n_mon, replace=False)).astype(np.int32)
    multi = G.multi_outage_cases(g, out, rng, n_multi)
    for j in range(4):   # cases holding the removed branches
        multi.append([int(out[3 * j]), int(out[3 * j + 1]), int(out[3 * j + 2])])
    gens = G.generator_outages(g, rng, n_gen)
    inj = G.perturbed_injections(g, rng, (len(lists), n_var), 0.2)
    return G.Workload("multi", g, mon, out, cands, inj, False, gens=gens, multi=multi)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_multi_outages_against_oracle(prec):
    w = _workload()
    r = oracle_rating(w)
    gpu = run_gpu(w, prec)
    idx = list(range(w.cands.n_cand))
    orc = oracle_scores(w, idx, r)
    err = compare(w, gpu, orc, r, idx, prec)
    n_gen = len(w.gens[0])
    multi_worst = [i for i in idx if orc[i]["worst_outage"] <= -2 - n_gen]
    assert multi_worst, "no multi-outage case is ever the worst"
    n_isl = sum(o["n_island"] for o in orc)
    assert n_isl > 0
    # where the oracle's worst case is unique by more than 4 tol, the GPU names it
    # (a multi case holding a contingency whose partner barely matters ties with it)
    sc = gpu["scores"]
    tol = TOL[prec]
    n_unique = 0
    for i in multi_worst:
        o = orc[i]
        if sc[i]["best_variant"] != o["best_variant"]:
            continue
        if int((o["loads_best"] >= o["loads_best"].max() - 4 * tol).sum()) == 1:
            n_unique += 1
            assert (sc[i]["worst_outage"], sc[i]["worst_branch"]) == (
                o["worst_outage"], o["worst_branch"]), i
    assert n_unique > 0
    say(f"multi-outage cases {prec}: worst |d max_load| {err:.2e}, {len(multi_worst)} "
        f"candidates decided by a multi case, {n_isl} islanding cases")


def test_multi_outages_one_variant():
    w = _workload(seed=62, n_var=1)
    r = oracle_rating(w)
    gpu = run_gpu(w, "fp64")
    idx = list(range(w.cands.n_cand))
    compare(w, gpu, oracle_scores(w, idx, r), r, idx, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_outage_worst_cases(prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = _workload(seed=63)
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    assert plan.view.n_multi_out == len(w.multi)
    bt = D.Batch(plan, w.cands, nv)
    bt.eval_topologies()
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows = bt.eval_injections(x, nv, False, prec)
    r = oracle_rating(w)
    idx = list(range(w.cands.n_cand))
    orc = oracle_scores(w, idx, r)
    top_k = 12
    n_multi_listed = 0
    lim = -2 - len(w.gens[0])
    for band in (0, 64):
        bt.set_tuning(scan_band=band)
        sc_dev = bt.n1_score(flows, nv, prec)
        cases = bt.n1_worst(flows, nv, prec, sc_dev, top_k)
        torch.cuda.synchronize()
        sc = D.Batch.scores_to_numpy(sc_dev, bt.n_cand)
        cs = D.Batch.cases_to_numpy(cases, bt.n_cand, top_k)
        for i in idx:
            if sc[i]["best_variant"] != orc[i]["best_variant"]:
                continue
            compare_worst(w, cs[i], sc[i], orc[i], top_k, prec, ctx=f"cand {i} band {band}")
            n_multi_listed += int((cs[i]["outage"] <= lim).sum())
    assert n_multi_listed > 0
    say(f"multi-outage worst cases {prec}: {n_multi_listed} multi entries listed")


def test_multi_outages_in_step_chunks():
    """The chunked step (candidate ranges) gives the scores of the plain calls bit
    for bit with multi-outage cases."""
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = _workload(seed=64)
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    bt.eval_topologies()
    flows = bt.eval_injections(x, nv, False, "fp32")
    ref = D.Batch.scores_to_numpy(bt.n1_score(flows, nv, "fp32"), bt.n_cand).copy()
    for ch in (1, 3):
        bt.set_tuning(step_chunks=ch)
        fl2, _ = bt.flow_buffer(nv, "fp32")
        out = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        bt.step(x, nv, False, "fp32", fl2, out)
        torch.cuda.synchronize()
        got = D.Batch.scores_to_numpy(out, bt.n_cand)
        for k in ("max_load", "overload_sum", "best_variant", "worst_branch", "worst_outage",
                  "status"):
            assert np.array_equal(got[k], ref[k]), (ch, k)


def test_medium_batch_with_extra_cases_sampled():
    """The medium batch (4,096 candidates x 16 variants, 500 contingencies) with 100
    generator outages and 100 multi-outage cases, in the launch shapes the bench
    uses (autotuned FP32 scan, persistent queue allowed): 16 sampled candidates
    against the oracle."""
    import torch
    from paper_2501_17529_amd import autotune
    from paper_2501_17529_amd import dcflow as D
    w = G.workload_medium(0)
    rng = np.random.default_rng(77)
    w.gens = G.generator_outages(w.grid, rng, 100)
    w.multi = G.multi_outage_cases(w.grid, w.out, rng, 100)
    nv = w.n_var
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    bt.eval_topologies()
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows = bt.eval_injections(x, nv, False, "fp32")
    autotune.tune_scan(bt, flows, nv, "fp32", reps=2, use_cache=False)
    out = bt.n1_score(flows, nv, "fp32")
    torch.cuda.synchronize()
    gpu = dict(scores=D.Batch.scores_to_numpy(out, bt.n_cand),
               vmax=bt.variant_max(nv).cpu().numpy(), flows=None)
    r = oracle_rating(w)
    idx = sorted(int(i) for i in np.random.default_rng(3).choice(w.cands.n_cand, 16, replace=False))
    orc = []
    for j, i in enumerate(idx):   # a few seconds of oracle per candidate
        orc += oracle_scores(w, [i], r)
        if j % 4 == 3:
            say(f"oracle: {j + 1} of {len(idx)} sampled candidates")
    err = compare(w, gpu, orc, r, idx, "fp32", check_flows=False)
    say(f"medium batch with 100 generator and 100 multi-outage cases: worst |d max_load| "
        f"{err:.2e} over 16 sampled candidates, tuning {bt.get_tuning()}")


def test_multi_outages_graph_replay():
    """A captured step with generator and multi-outage cases replays to the eager
    scores, with eager work on the same buffers between the replays."""
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = _workload(seed=65)
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows, _ = bt.flow_buffer(nv, "fp32")
    out = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    keys = ("max_load", "overload_sum", "best_variant", "worst_branch", "worst_outage", "status")
    with torch.cuda.stream(s):
        bt.eval_topologies()
        bt.eval_injections(x, nv, False, "fp32", flows=flows)
        bt.n1_score(flows, nv, "fp32", out=out)
        torch.cuda.synchronize()
        eager = D.Batch.scores_to_numpy(out, bt.n_cand).copy()
        bt.capture(x, nv, False, "fp32", flows, out, s)
        torch.cuda.synchronize()
        for rep in range(3):
            out.zero_()
            bt.replay(s)
            torch.cuda.synchronize()
            got = D.Batch.scores_to_numpy(out, bt.n_cand)
            for k in keys:
                assert np.array_equal(got[k], eager[k]), (rep, k)
            other = torch.empty_like(out)
            bt.n1_score(flows, nv, "fp32", out=other)
            torch.cuda.synchronize()
