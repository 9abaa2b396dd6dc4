"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the CPU oracle on the same seeded inputs."""
import sys

import numpy as np

from oracle import dcflow_oracle as O

TOL = {"fp64": 1e-6, "fp32": 1e-4, "bf16x6": 1e-4}   # max |dp| / rating


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def kept_rows(mon, out):
    mon = [int(x) for x in mon]
    s = set(mon)
    return np.asarray(mon + [int(o) for o in out if int(o) not in s], np.int64)


def run_gpu(w, prec, rating=None, cands=None, inj=None, inj_shared=None):
    import torch
    from paper_2501_17529_amd import dcflow as D
    cands = w.cands if cands is None else cands
    inj = w.inj if inj is None else inj
    shared = w.inj_shared if inj_shared is None else inj_shared
    plan = D.Plan.from_workload(w, rating=rating)
    nv = inj.shape[-2]
    bt = D.Batch(plan, cands, nv)
    bt.eval_topologies()
    x = torch.from_numpy(np.ascontiguousarray(inj)).cuda()
    flows = bt.eval_injections(x, nv, shared, prec)
    out = bt.n1_score(flows, nv, prec)
    torch.cuda.synchronize()
    sc = D.Batch.scores_to_numpy(out, bt.n_cand)
    vmax = bt.variant_max(nv).cpu().numpy()
    fl = bt.flows_view(flows, nv).double().cpu().numpy()
    return dict(plan=plan, batch=bt, scores=sc, vmax=vmax, flows=fl)


def compare(w, gpu, oracle_res, rating, idx, prec, check_flows=True):
    """Element-wise comparison of GPU scores and flows with the oracle."""
    tol = TOL[prec]
    sc = gpu["scores"]
    er = kept_rows(w.mon, w.out)
    mon_pos = np.arange(len(w.mon))
    worst_err = 0.0
    for ci, i in enumerate(idx):
        o = oracle_res[ci]
        s = sc[i]
        ctx = f"cand {i} ({prec})"
        if o["status"] & O.ST_DISCONNECTED:
            assert s["status"] & 1, ctx
            assert np.isinf(s["max_load"]) and s["best_variant"] == -1, ctx
            continue
        assert (s["status"] & 0x7) == o["status"], (ctx, s["status"], o["status"])
        assert (s["status"] >> 8) == o["n_island"], (ctx, s["status"] >> 8, o["n_island"])
        # per-variant maxima
        vm = gpu["vmax"][i]
        err = np.abs(vm - o["max_load"]).max()
        worst_err = max(worst_err, err)
        assert err <= tol, (ctx, "variant max", err)
        # best variant: unique unless another variant is within 2 tol
        ml = o["max_load"]
        if s["best_variant"] != o["best_variant"]:
            assert abs(ml[s["best_variant"]] - ml[o["best_variant"]]) <= 2 * tol, ctx
        assert abs(s["max_load"] - ml[s["best_variant"]]) <= tol, ctx
        # worst case: the reported (outage, branch) must carry a load within 2 tol of the max
        if s["best_variant"] == o["best_variant"]:
            loads = o["loads_best"]
            row = int(np.flatnonzero(np.asarray(w.mon) == s["worst_branch"])[0])
            if s["worst_outage"] == -1:    # N-0 (generator outages are -2 - g)
                lv = loads[0, row]
            else:
                cpos = np.flatnonzero(o["scored_out"] == s["worst_outage"])
                assert len(cpos) == 1, ctx
                lv = loads[1 + cpos[0], row]
            assert abs(lv - loads.max()) <= 2 * tol, (ctx, lv, loads.max())
            cnt = int((loads > 1.0 - 2 * tol).sum()) + 1
            assert abs(s["overload_sum"] - o["overload_sum"]) <= tol * cnt, (
                ctx, s["overload_sum"], o["overload_sum"])
        if check_flows:
            p0 = o["flows"]["p0"]             # [V, m]
            g = gpu["flows"][i][:, : len(er)]  # [V, n_er]
            rr = np.concatenate([rating, np.full(len(er) - len(w.mon), 1.0)])
            e = np.abs(g - p0[:, er]) / rr
            assert e.max() <= tol, (ctx, "N-0 flows", e.max())
    return worst_err


def oracle_scores(w, idx, rating, variants=None):
    """Oracle scores of candidates idx (all variants, or the listed ones); with
    controls, the injection vectors' tail holds the control values."""
    g = w.grid
    res = []
    for i in idx:
        x = w.inj if w.inj_shared else w.inj[int(i)]
        if variants is not None:
            x = x[np.asarray(variants)]
        kw = {"gens": getattr(w, "gens", None), "multi": getattr(w, "multi", None)}
        if getattr(w, "controls", None):
            kw.update(controls=w.controls, ctrl=x[:, g.n_bus:])
            x = x[:, :g.n_bus]
        res.append(O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, w.cands.elements(int(i)),
                                     x, w.mon, w.out, rating, **kw))
    return res


def oracle_rating(w):
    g = w.grid
    return O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, w.rating_scale, w.rating_offset)


def compare_worst(w, cases, score, oracle_sc, top_k, prec, ctx=""):
    """One candidate's worst-case list from the GPU against the oracle's: the
    sorted loads agree within the tolerance rank by rank; every listed case is a
    scored case whose oracle load matches; no case repeats; the first entry is
    the score record's maximum and worst case, bit for bit.  Near-equal loads
    may come in either order."""
    tol = TOL[prec]
    want = O.worst_cases(oracle_sc, w.mon, w.out, top_k)
    used = cases[cases["branch"] >= 0]
    assert len(used) == len(want), (ctx, len(used), len(want))
    if not len(want):
        assert np.all(cases["load"] == -1.0), ctx
        return 0.0
    np.testing.assert_allclose(used["load"], [v for v, _, _ in want], atol=tol, rtol=0,
                               err_msg=f"{ctx}: ranked loads")
    assert np.all(np.diff(used["load"]) <= 0), (ctx, "not sorted")
    pairs = list(zip(used["branch"].tolist(), used["outage"].tolist()))
    assert len(set(pairs)) == len(pairs), (ctx, "repeated case")
    # oracle load of every listed case
    mon_pos = {int(b): i for i, b in enumerate(w.mon)}
    cases_o = [-1] + [int(o) for o in oracle_sc["scored_out"]]
    row_of = {o: ci for ci, o in enumerate(cases_o)}
    for (b, o), v in zip(pairs, used["load"]):
        assert o in row_of, (ctx, "not a scored case", b, o)
        lo = oracle_sc["loads_best"][row_of[o], mon_pos[b]]
        assert abs(lo - v) <= tol, (ctx, b, o, lo, v)
    assert used["load"][0] == score["max_load"], (ctx, used["load"][0], score["max_load"])
    assert (used["branch"][0], used["outage"][0]) == (score["worst_branch"], score["worst_outage"]), ctx
    return float(np.abs(used["load"] - np.array([v for v, _, _ in want])).max())
