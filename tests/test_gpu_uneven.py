"""Uneven-rank configuration at one GPU's share: the 10,000-bus / 15,500-branch
grid, 8,192 candidates of rank uniform in 1..8 (an eighth of the 65,536-candidate
batch), every branch monitored, 2,000 contingencies, one injection per
candidate, run as one persistent launch per pass.  The whole share runs on the
GPU; three sampled candidates are checked against the oracle one by one (a
dense 10,000-bus solve each), every candidate by invariants."""
import numpy as np
import pytest

import gridgen as G

from _gpu_common import compare, compare_worst, gpu_available, oracle_rating, oracle_scores, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

N_SHARE = 8192


@pytest.fixture(scope="module")
def uneven():
    from paper_2501_17529_amd import dcflow as D
    import torch
    say("uneven share: generating 10,000-bus grid and 8,192 candidates")
    w = G.workload_uneven(0, n_cand=N_SHARE)
    say("uneven share: plan build")
    plan = D.Plan.from_workload(w)
    torch.cuda.synchronize()
    r = oracle_rating(w)
    idx = [int(i) for i in np.random.default_rng(17).choice(N_SHARE, size=3, replace=False)]
    say(f"uneven share: oracle on candidates {idx}")
    res = oracle_scores(w, idx, r)
    return w, plan, r, idx, res


@pytest.mark.parametrize("prec", ["bf16x6", "fp32"])
def test_uneven_share(uneven, prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    w, plan, r, idx, res = uneven
    k = np.diff(w.cands.off)
    assert k.min() == 1 and k.max() == 8
    bt = D.Batch(plan, w.cands, 1)
    bt.set_tuning(persistent=1)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    bt.eval_topologies()
    flows = bt.eval_injections(x, 1, False, prec)
    out = bt.n1_score(flows, 1, prec)
    torch.cuda.synchronize()
    sc = D.Batch.scores_to_numpy(out, bt.n_cand)
    say(f"uneven share {prec}: max_load range {sc['max_load'].min():.3f}..{sc['max_load'].max():.3f}")
    # invariants over the whole share
    assert np.all(np.isfinite(sc["max_load"])) and np.all(sc["max_load"] > 0)
    assert np.all((sc["status"] & 0x7) == 0)
    assert np.all(sc["best_variant"] == 0)
    assert np.all(sc["overload_sum"] >= 0)
    assert np.all(np.isin(sc["worst_branch"], w.mon))
    assert np.all((sc["worst_outage"] == -1) | np.isin(sc["worst_outage"], w.out))
    vm = bt.variant_max(1).cpu().numpy()[:, 0]
    np.testing.assert_array_equal(vm, sc["max_load"])
    # the sampled candidates against the oracle, element by element (flows of every kept row)
    gpu = dict(scores=sc, vmax=bt.variant_max(1).cpu().numpy(),
               flows={i: bt.flows_view(flows, 1)[i].double().cpu().numpy() for i in idx})
    err = compare(w, gpu, res, r, idx, prec)
    say(f"uneven share {prec}: worst |d max_load| on the sample = {err:.3e}")
    # one work item per candidate (every monitored row in one band): same scores
    mon_pad = (len(w.mon) + 63) // 64 * 64
    bt.set_tuning(persistent=1, scan_band=mon_pad)
    out2 = bt.n1_score(flows, 1, prec)
    torch.cuda.synchronize()
    sc2 = D.Batch.scores_to_numpy(out2, bt.n_cand)
    for key in ("max_load", "worst_branch", "worst_outage", "status"):
        np.testing.assert_array_equal(sc2[key], sc[key], err_msg=key)
    np.testing.assert_allclose(sc2["overload_sum"], sc["overload_sum"], rtol=1e-9, atol=1e-12)
    # agg_i of the winners (row bands merged), sampled against the oracle
    cases = D.Batch.cases_to_numpy(bt.n1_worst(flows, 1, prec, out, 16), bt.n_cand, 16)
    assert np.all(cases["load"][:, 0] == sc["max_load"])
    for ci, i in enumerate(idx):
        compare_worst(w, cases[i], sc[i], res[ci], 16, prec, f"uneven {prec} cand {i}")
