"""Injection brute force with phase shifters and HVDC links: the 2,000-bus /
3,100-branch grid with 20 shifters and 4 HVDC links, every branch monitored,
1,000 contingencies, all 4,096 control/load combinations for a sample of the
topologies (the unchanged grid and 7 of the 1,024), shared combinations as one
GEMM with the control columns folded into K.  Sampled (topology, combination)
pairs are checked against the oracle's DC model with controls one by one, all
pairs by invariants."""
import numpy as np
import pytest

import gridgen as G

from _gpu_common import TOL, gpu_available, kept_rows, oracle_rating, oracle_scores, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def brute():
    from paper_2501_17529_amd import dcflow as D
    import torch
    w0 = G.workload_brute(0, n_topo=7, n_comb=4096)
    lists = [[]] + [w0.cands.elements(i) for i in range(w0.cands.n_cand)]
    w = G.Workload(w0.name, w0.grid, w0.mon, w0.out, G.Candidates.from_lists(lists), w0.inj, True,
                   meta=w0.meta, controls=w0.controls)
    plan = D.Plan.from_workload(w)
    torch.cuda.synchronize()
    r = oracle_rating(w)
    combos = [0, 1, 777, 2048, 4095]
    tops = [0, 3, 6]
    say(f"brute: oracle on topologies {tops}, combinations {combos}")
    res = {i: o for i, o in zip(tops, oracle_scores(w, tops, r, variants=combos))}
    return w, plan, r, combos, tops, res


def test_control_columns_match_the_model(brute):
    """The plan's control columns equal the flow change of one unit of each
    control in the oracle's model (unchanged grid)."""
    from oracle import dcflow_oracle as O
    w, plan, r, combos, tops, res = brute
    g = w.grid
    n = g.n_bus
    h = plan.ptdf(controls=True).cpu().numpy()
    assert h.shape[1] == n + len(w.controls["pst"]) + len(w.controls["hvdc"])
    nc = len(w.controls["pst"]) + len(w.controls["hvdc"])
    for q in range(nc):
        ctrl = np.zeros((1, nc))
        ctrl[0, q] = 1.0
        cf = O.candidate_flows(n, g.f, g.t, g.b, g.slack, [], np.zeros((1, n)), [],
                               w.controls, ctrl)
        np.testing.assert_allclose(h[:, n + q], cf["p0"][0], atol=1e-11, err_msg=f"control {q}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_brute_force_sample(brute, prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    w, plan, r, combos, tops, res = brute
    nv = w.inj.shape[0]
    bt = D.Batch(plan, w.cands, nv)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    bt.eval_topologies()
    flows = bt.eval_injections(x, nv, True, prec)
    out = bt.n1_score(flows, nv, prec)
    torch.cuda.synchronize()
    sc = D.Batch.scores_to_numpy(out, bt.n_cand)
    vm = bt.variant_max(nv).cpu().numpy()
    say(f"brute {prec}: max_load {sc['max_load'].min():.3f}..{sc['max_load'].max():.3f}")
    assert np.all(np.isfinite(vm)) and np.all((sc["status"] & 0x7) == 0)
    np.testing.assert_array_equal(sc["best_variant"], np.argmin(vm, axis=1))
    np.testing.assert_array_equal(sc["max_load"], vm[np.arange(bt.n_cand), sc["best_variant"]])
    tol = TOL[prec]
    er = kept_rows(w.mon, w.out)
    fl = bt.flows_view(flows, nv)
    worst = 0.0
    for i in tops:
        o = res[i]
        err = np.abs(vm[i, combos] - o["max_load"]).max()
        worst = max(worst, err)
        assert err <= tol, (prec, i, err)
        got = fl[i, combos].double().cpu().numpy()[:, : len(er)]
        p0 = o["flows"]["p0"][:, er]
        fe = np.abs(got - p0) / r[: len(er)]
        assert fe.max() <= tol, (prec, i, "flows", fe.max())
    say(f"brute {prec}: worst |d max_load| on the sample = {worst:.3e}")
