"""Stub folding (dcflow_fold_stubs and its host helpers; Sec. IV-A): radial stubs
replaced by their injections at the bus they hang from.  Against the DC flows of
the oracle on the unfolded and the folded grids: the flows of every kept branch
agree, a folded branch carries the sum of the injections beyond it, and the N-1
scores of split candidates agree when the split buses are protected."""
import numpy as np
import pytest

import gridgen as G
from oracle import dcflow_oracle as O


@pytest.fixture(scope="module")
def D():
    from paper_2501_17529_amd import dcflow
    return dcflow


def fold_candidate(g, fo, keep, els, sf, n_var):
    """A candidate's elements on the folded grid: split masks remapped to the
    folded incident lists (kept branches keep their relative order), and a moved
    stub turned into its injection on the new busbar (per-variant p_new from the
    stub flows sf [n_var][n_branch]), outages renumbered.  Returns (elements,
    valid, stubs moved); not valid when the new busbar would keep no branch, or
    all of them, or an outage removes a folded branch."""
    els2, ok, n_moved = [], True, 0
    for k, d, m, pn in els:
        if k != G.KIND_SPLIT:   # an outage: renumbered (a folded branch's outage islands)
            ok = ok and bool(keep[d])
            els2.append((k, int(fo["branch_new"][d]), m, pn))
            continue
        inc = [int(l) for l in g.incident(d)]
        inc2 = [l for l in inc if keep[l]]
        moved = [inc[q] for q in range(len(inc)) if (m >> q) & 1]
        pnew = np.full(n_var, float(pn))
        for l in moved:
            if not keep[l]:      # a stub: its injection (the sum beyond it) goes to B
                beyond = int(g.t[l]) if int(g.f[l]) == d else int(g.f[l])
                pnew += sf[:, l] if int(g.f[l]) == beyond else -sf[:, l]
                n_moved += 1
        m2 = sum(1 << inc2.index(l) for l in moved if keep[l])
        ok = ok and m2 != 0 and m2 != (1 << len(inc2)) - 1
        els2.append((k, int(fo["bus_new"][d]), m2, pnew))
    return els2, ok, n_moved


def _folded_grid(g, fold):
    keep = fold["branch_new"] >= 0
    return (fold["n_bus"], fold["bus_new"][g.f[keep]], fold["bus_new"][g.t[keep]], g.b[keep],
            fold["slack"], keep)


def test_path_by_hand(D):
    # slack 0 - 1 - 2 - 3 with a triangle 0 - 4 - 5 - 0; injections 1, 2, 3 on the path
    f = [0, 1, 2, 0, 4, 5]
    t = [1, 2, 3, 4, 5, 0]
    fo = D.fold_stubs(6, f, t, 0)
    assert list(fo["bus_new"]) == [0, 0, 0, 0, 1, 2]
    assert list(fo["branch_new"]) == [-1, -1, -1, 0, 1, 2]
    assert list(fo["up_branch"]) == [-1, 0, 1, 2, -1, -1]
    x = np.array([[-6.0, 1.0, 2.0, 3.0, 0.0, 0.0]])
    np.testing.assert_array_equal(D.fold_injections(fo, x), [[0.0, 0.0, 0.0]])
    np.testing.assert_array_equal(D.stub_flows(fo, f, t, x), [[-6, -5, -3, 0, 0, 0]])
    # protecting bus 2 keeps 0-1-2 (and so bus 1, now of degree two) and folds bus 3 only
    fo2 = D.fold_stubs(6, f, t, 0, protect=np.arange(6) == 2)
    assert list(fo2["branch_new"]) == [0, 1, -1, 2, 3, 4]
    assert list(fo2["up_branch"]) == [-1, -1, -1, 2, -1, -1]


def test_slack_and_parallel_branches_stay(D):
    # the slack at a leaf stays; a bus on two parallel branches has degree two and stays
    f = [0, 1, 2, 3, 1, 1]
    t = [1, 2, 3, 1, 4, 4]
    fo = D.fold_stubs(5, f, t, 0)
    assert fo["n_bus"] == 5 and fo["n_branch"] == 6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_folded_flows_equal_unfolded(D, seed):
    rng = np.random.default_rng(seed)
    g = G.attach_stubs(G.make_grid(80, 120, seed), rng, 15)
    fo = D.fold_stubs(g.n_bus, g.f, g.t, g.slack)
    assert fo["n_bus"] <= 80 and fo["n_branch"] < g.n_branch
    x = G.perturbed_injections(g, rng, (3,), 0.3)
    p_full = O.dc_flows(g.n_bus, g.f, g.t, g.b, g.slack, x)
    n2, f2, t2, b2, s2, keep = _folded_grid(g, fo)
    p_fold = O.dc_flows(n2, f2, t2, b2, s2, D.fold_injections(fo, x))
    np.testing.assert_allclose(p_fold, p_full[:, keep], atol=1e-10)
    np.testing.assert_allclose(D.stub_flows(fo, g.f, g.t, x)[:, ~keep], p_full[:, ~keep],
                               atol=1e-10)
    # every folded branch is a bridge of the original grid
    assert np.all(O.bridges(g.n_bus, g.f, g.t)[~keep])


def test_scores_equal_with_protected_split_buses(D):
    """N-1 screening of split candidates on the folded grid equals that on the
    unfolded one over the kept branches (folded branches are bridges: their N-1
    cases island either way).  A split that moves a stub to the new busbar moves
    the stub's injection there instead: the branch topology becomes an injection
    topology (per-variant p_new), which is what folding is for."""
    rng = np.random.default_rng(5)
    g = G.attach_stubs(G.make_grid(60, 95, 5), rng, 25)
    cands = [G.sample_candidate(g, rng, int(rng.integers(1, 3)), 0) for _ in range(16)]
    split = np.zeros(g.n_bus, bool)
    for els in cands:
        for k, d, _, _ in els:
            split[d] = True
    fo = D.fold_stubs(g.n_bus, g.f, g.t, g.slack, protect=split)
    n2, f2, t2, b2, s2, keep = _folded_grid(g, fo)
    kept = np.flatnonzero(keep)
    x = G.perturbed_injections(g, rng, (2,), 0.2)
    xf = D.fold_injections(fo, x)
    sf = D.stub_flows(fo, g.f, g.t, x)          # [V, n_branch]
    r = np.full(len(kept), 1.0)
    n_moved_stub = n_cmp = 0
    for els in cands:
        els2, ok, nm = fold_candidate(g, fo, keep, els, sf, x.shape[0])
        n_moved_stub += nm
        if not ok:
            continue  # the new busbar would keep no branch (or all): not a split any more
        full = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, els, x, kept, kept, r)
        fold = O.score_candidate(n2, f2, t2, b2, s2, els2, xf, np.arange(len(kept)),
                                 np.arange(len(kept)), r)
        np.testing.assert_allclose(fold["max_load"], full["max_load"], atol=1e-10)
        assert fold["n_island"] == full["n_island"]
        n_cmp += 1
    assert n_cmp >= 8 and n_moved_stub > 0


def test_fold_errors(D):
    with pytest.raises(D.DcflowError):
        D.fold_stubs(3, [0, 1], [1, 3], 0)       # terminal out of range
    with pytest.raises(D.DcflowError):
        D.fold_stubs(3, [0, 1], [1, 1], 0)       # self loop
