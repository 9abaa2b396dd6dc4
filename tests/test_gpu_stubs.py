"""Stub folding end to end on the GPU (Sec. IV-A): the library's scores of split
candidates on the folded grid, with moved stubs turned into per-variant
new-busbar injections (dcflow_set_busbar_injections), equal its scores on the
unfolded grid over the kept branches."""
import numpy as np
import pytest

import gridgen as G
from oracle import dcflow_oracle as O

from _gpu_common import gpu_available, say
from test_stub_fold import fold_candidate

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_folded_grid_scores_match(prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    rng = np.random.default_rng(9)
    g = G.attach_stubs(G.make_grid(150, 230, 9), rng, 40)
    cands = [G.sample_candidate(g, rng, int(rng.integers(1, 4)), int(rng.integers(0, 2)))
             for _ in range(64)]
    split = np.zeros(g.n_bus, bool)
    for els in cands:
        for k, d, _, _ in els:
            if k == G.KIND_SPLIT:
                split[d] = True
    fo = D.fold_stubs(g.n_bus, g.f, g.t, g.slack, protect=split)
    keep = fo["branch_new"] >= 0
    kept = np.flatnonzero(keep)
    nv = 4
    x = G.perturbed_injections(g, rng, (nv,), 0.2)
    sf = D.stub_flows(fo, g.f, g.t, x)
    xf = D.fold_injections(fo, x)
    pairs = [(els, fold_candidate(g, fo, keep, els, sf, nv)) for els in cands]
    pairs = [(a, b) for a, (b, ok, _) in pairs if ok]
    assert len(pairs) >= 32
    n_moved = sum(fold_candidate(g, fo, keep, a, sf, nv)[2] for a, _ in pairs)
    assert n_moved > 0
    rating = np.ones(len(kept))

    def scores(n_bus, f, t, b, slack, mon, lists, xx, pnv):
        cs = G.Candidates.from_lists([[(k, d, m, 0.0) for k, d, m, _ in els] for els in lists])
        plan = D.Plan(n_bus, f, t, b, mon, mon, np.zeros(n_bus), slack, rating=rating)
        bt = D.Batch(plan, cs, nv)
        if pnv is not None:
            bt.set_busbar_injections(torch.from_numpy(np.ascontiguousarray(pnv)).cuda(), nv)
        bt.eval_topologies()
        xt = torch.from_numpy(np.ascontiguousarray(xx)).cuda()
        fl = bt.eval_injections(xt, nv, True, prec)
        out = bt.n1_score(fl, nv, prec)
        vm = bt.variant_max(nv).cpu().numpy().copy()
        torch.cuda.synchronize()
        return D.Batch.scores_to_numpy(out, bt.n_cand).copy(), vm

    full_sc, full_vm = scores(g.n_bus, g.f, g.t, g.b, g.slack, kept, [a for a, _ in pairs], x,
                              None)
    pnv = np.concatenate([np.stack([np.asarray(pn, float) * np.ones(nv) for _, _, _, pn in b])
                          if b else np.zeros((0, nv)) for _, b in pairs])
    f2, t2 = fo["bus_new"][g.f[keep]], fo["bus_new"][g.t[keep]]
    fold_sc, fold_vm = scores(fo["n_bus"], f2, t2, g.b[keep], fo["slack"], np.arange(len(kept)),
                              [b for _, b in pairs], xf, pnv)
    tol = 1e-9 if prec == "fp64" else 1e-4
    err = np.abs(fold_vm - full_vm).max()
    assert err <= tol, err
    np.testing.assert_array_equal(fold_sc["status"], full_sc["status"])
    # the folded-grid scores against the oracle on the unfolded grid (every kept
    # branch monitored and a contingency, unit ratings)
    oerr = 0.0
    for i in range(0, len(pairs), 4):
        els = [(k, d, m, 0.0) for k, d, m, _ in pairs[i][0]]
        o = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, els, x, kept, kept, rating)
        oerr = max(oerr, float(np.abs(fold_vm[i] - o["max_load"]).max()))
        assert (fold_sc["status"][i] >> 8) == o["n_island"], i
    assert oerr <= (1e-6 if prec == "fp64" else 1e-4), oerr
    say(f"stub folding {prec}: {fo['n_bus']} of {g.n_bus} buses, {len(kept)} of "
        f"{g.n_branch} branches kept, {n_moved} moved stubs, max |d max_load| {err:.2e}, "
        f"against the oracle {oerr:.2e}")
