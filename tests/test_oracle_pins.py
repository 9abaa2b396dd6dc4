"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, physical invariants, brute force and the paper's own formulas."""
import itertools

import numpy as np
import pytest

import gridgen as G
from oracle import dcflow_oracle as O
from oracle import paper_formulas as PF


def _incidence_balance(n, f, t, alive, flows, p):
    """Net outflow minus injection at every node."""
    bal = np.zeros((flows.shape[0], n))
    fa, ta = f[alive], t[alive]
    for v in range(flows.shape[0]):
        np.add.at(bal[v], fa, flows[v, alive])
        np.add.at(bal[v], ta, -flows[v, alive])
    return bal - p


# ------------------------------------------------------------ closed forms

def test_triangle_ptdf_closed_form():
    # equal reactances: a unit transfer splits 2/3 on the direct edge, 1/3 on the detour
    f = np.array([1, 1, 2])
    t = np.array([0, 2, 0])
    b = np.ones(3) * 7.0
    h = O.ptdf(3, f, t, b, 0)
    np.testing.assert_allclose(h[:, 0], 0.0, atol=0)
    np.testing.assert_allclose(h[:, 1], [2 / 3, 1 / 3, 1 / 3], atol=1e-15)
    np.testing.assert_allclose(h[:, 2], [1 / 3, -1 / 3, 2 / 3], atol=1e-15)


def test_triangle_score_by_hand():
    # unit susceptances, +1 at bus 1 and +0.5 at bus 2 withdrawn at slack 0.
    # N-0 = (5/6, 1/6, 2/3).  Losing edge 0 routes bus 1 over 1->2->0: (0, 1, 1.5);
    # losing edge 1: (1, 0, 0.5); losing edge 2: (1.5, -0.5, 0).
    f = np.array([1, 1, 2])
    t = np.array([0, 2, 0])
    b = np.ones(3)
    x = np.array([[-1.5, 1.0, 0.5]])
    r = np.array([1.0, 1.0, 1.2])
    mon = out = np.arange(3)
    sc = O.score_candidate(3, f, t, b, 0, [], x, mon, out, r)
    np.testing.assert_allclose(sc["flows"]["p0"][0], [5 / 6, 1 / 6, 2 / 3], atol=1e-15)
    assert sc["best_max_load"] == pytest.approx(1.5, abs=1e-14)
    assert sc["overload_sum"] == pytest.approx(0.25 + 0.5, abs=1e-14)
    assert sc["n_island"] == 0
    assert (sc["worst_outage"], sc["worst_branch"]) == (2, 0)


def test_triangle_worst_cases_by_hand():
    # the triangle above: N-0 loads (5/6, 1/6, 5/9); losing edge 0: (0, 1, 1.25); edge 1:
    # (1, 0, 5/12); edge 2: (1.5, 0.5, 0).  Two loads of exactly 1 tie: the case of edge
    # 0 comes first.
    f = np.array([1, 1, 2])
    t = np.array([0, 2, 0])
    x = np.array([[-1.5, 1.0, 0.5]])
    r = np.array([1.0, 1.0, 1.2])
    mon = out = np.arange(3)
    sc = O.score_candidate(3, f, t, np.ones(3), 0, [], x, mon, out, r)
    got = O.worst_cases(sc, mon, out, 7)
    want = [(1.5, 0, 2), (1.25, 2, 0), (1.0, 1, 0), (1.0, 0, 1), (5 / 6, 0, -1), (5 / 9, 2, -1),
            (0.5, 1, 2)]
    np.testing.assert_allclose([v for v, _, _ in got], [v for v, _, _ in want], atol=1e-14)
    # the two loads of 1 are equal only up to rounding: either order is right
    assert [(b, o) for _, b, o in got[:2]] == [(0, 2), (2, 0)]
    assert {(b, o) for _, b, o in got[2:4]} == {(1, 0), (0, 1)}
    assert [(b, o) for _, b, o in got[4:]] == [(0, -1), (2, -1), (1, 2)]
    assert O.worst_cases(sc, mon, out, 1)[0][1:] == (sc["worst_branch"], sc["worst_outage"])


@pytest.mark.parametrize("seed", [3, 4])
def test_worst_cases_match_bruteforce(seed):
    """The k worst cases of the winner, by re-factorising per contingency."""
    w = G.workload_tiny(seed)
    g = w.grid
    r = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, w.rating_scale, w.rating_offset)
    rng = np.random.default_rng(seed)
    for i in rng.choice(w.cands.n_cand, size=5, replace=False):
        el = w.cands.elements(int(i))
        x = w.inj if w.inj_shared else w.inj[int(i)]
        sc = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, el, x, w.mon, w.out, r)
        got = O.worst_cases(sc, w.mon, w.out, 12)
        p1, isl = O.n1_flows_bruteforce(g.n_bus, g.f, g.t, g.b, g.slack, el, x, w.out)
        v = sc["best_variant"]
        p0 = sc["flows"]["p0"][v]
        ent = [(abs(p0[l]) / r[li], li, int(l), -1) for li, l in enumerate(w.mon)]
        for c, o in enumerate(w.out):
            if isl[c]:
                continue
            ent += [(abs(p1[v, c, l]) / r[li], (c + 1) * len(w.mon) + li, int(l), int(o))
                    for li, l in enumerate(w.mon)]
        ent.sort(key=lambda e: (-e[0], e[1]))
        np.testing.assert_allclose([e[0] for e in got], [e[0] for e in ent[:12]], atol=1e-10)
        # ties within rounding may swap places: compare the cases as sets up to the last load
        last = ent[11][0]
        strict = [(e[2], e[3]) for e in ent[:12] if e[0] > last + 1e-9]
        assert strict == [(b, o) for v_, b, o in got[:len(strict)]]


def _random_tree(n, seed):
    rng = np.random.default_rng(seed)
    par = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)])
    f = np.arange(1, n)
    t = par[1:]
    flip = rng.random(n - 1) < 0.5
    f2 = np.where(flip, t, f)
    t2 = np.where(flip, f, t)
    return par, f2, t2, rng


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_radial_tree_closed_form(seed):
    n = 25
    par, f, t, rng = _random_tree(n, seed)
    p = rng.normal(size=n)
    p[0] = -p[1:].sum()
    # subtree sums (slack = root 0): the edge (i, par i) carries sum of P below i, towards par
    sub = p.copy()
    for i in range(n - 1, 0, -1):
        sub[par[i]] += sub[i]
    expect = np.where(f == np.arange(1, n), sub[1:], -sub[1:])
    for b in (np.ones(n - 1), rng.lognormal(-2.5, 0.5, n - 1)):
        fl = O.dc_flows(n, f, t, b, 0, p)[0]
        np.testing.assert_allclose(fl, expect, atol=1e-12)


def test_parallel_lines_lodf_is_one():
    # two identical lines 0-1 plus a line 1-2: losing one doubles the other
    f = np.array([0, 0, 1])
    t = np.array([1, 1, 2])
    b = np.array([4.0, 4.0, 2.0])
    x = np.array([[1.5, 0.5, -2.0]])
    cf = O.candidate_flows(3, f, t, b, 0, [], x, [0, 1, 2])
    assert cf["state"].tolist() == [0, 0, 2]          # line 1-2 is a bridge
    assert cf["lodf"][1, 0] == pytest.approx(1.0, abs=1e-14)
    assert cf["lodf"][0, 1] == pytest.approx(1.0, abs=1e-14)
    assert cf["den"][0] == pytest.approx(0.5, abs=1e-14)


def test_unicyclic_grid():
    # 5-cycle 0..4 plus pendant buses 5 (on 2) and 6 (on 5); x random
    rng = np.random.default_rng(4)
    f = np.array([0, 1, 2, 3, 4, 2, 5])
    t = np.array([1, 2, 3, 4, 0, 5, 6])
    b = rng.lognormal(-2.5, 0.5, 7)
    n = 7
    p = rng.normal(size=n)
    p[0] = -p[1:].sum()
    out = np.arange(7)
    cf = O.candidate_flows(n, f, t, b, 0, [], p, out)
    assert cf["state"].tolist() == [0, 0, 0, 0, 0, 2, 2]
    for c in range(5):
        # losing a cycle edge leaves a tree: flows are the subtree sums
        keep = np.array([e for e in range(7) if e != c])
        p1_tree = O.dc_flows(n, f[keep], t[keep], np.ones(6), 0, p)[0]   # reactance-free
        p1 = cf["p0"][0] + cf["lodf"][:, c] * cf["p0"][0, c]
        np.testing.assert_allclose(p1[keep], p1_tree, atol=1e-11)
        assert abs(p1[c]) < 1e-14


# ---------------------------------------------------------- invariants

def _mixed_workload(seed, n=60, m=95, n_cand=20):
    rng = np.random.default_rng(seed)
    g = G.make_grid(n, m, seed)
    cands = []
    for _ in range(n_cand):
        ns = int(rng.integers(0, 4))
        no = int(rng.integers(0 if ns else 1, 3))
        cands.append(G.sample_candidate(g, rng, ns, no))
    return g, cands, rng


@pytest.mark.parametrize("seed", [0, 1])
def test_kirchhoff_balance(seed):
    g, cands, rng = _mixed_workload(seed)
    x = G.perturbed_injections(g, rng, (3,), 0.3)
    for els in cands:
        for k, (kind, d, m, _p) in enumerate(els):
            if kind == G.KIND_SPLIT:
                els[k] = (kind, d, m, float(rng.normal()))    # move some injection too
        cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, [])
        n2, f2, t2, alive, splits = O.rebuild(g.n_bus, g.f, g.t, els)
        p = O.candidate_injections(n2, x, splits, g.slack)
        bal = _incidence_balance(n2, f2, t2, alive, cf["p0"], p)
        assert np.abs(bal).max() < 1e-11
        assert np.all(cf["p0"][:, ~alive] == 0)


def test_slack_absorbs_imbalance():
    g, cands, rng = _mixed_workload(3, n_cand=3)
    x = G.perturbed_injections(g, rng, (2,), 0.1)
    y = x.copy()
    y[:, g.slack] += 5.0
    for els in cands:
        a = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, [])["p0"]
        c = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, y, [])["p0"]
        np.testing.assert_allclose(a, c, atol=1e-12)


def test_lodf_matches_bruteforce_tiny_workload():
    w = G.workload_tiny(0)
    g = w.grid
    for i in range(w.cands.n_cand):
        els = w.cands.elements(i)
        cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, w.inj, w.out)
        p1b, isl = O.n1_flows_bruteforce(g.n_bus, g.f, g.t, g.b, g.slack, els, w.inj, w.out)
        assert np.array_equal(isl, cf["state"] == 2)
        ok = np.flatnonzero(cf["state"] == 0)
        p1 = cf["p0"][:, None, :] + cf["lodf"].T[None] * cf["p0"][:, w.out][:, :, None]
        np.testing.assert_allclose(p1[:, ok], p1b[:, ok], atol=1e-11)


@pytest.mark.parametrize("seed", [0, 1])
def test_lodf_matches_bruteforce_with_outages_and_splits(seed):
    g, cands, rng = _mixed_workload(seed, n_cand=8)
    x = G.perturbed_injections(g, rng, (2,), 0.3)
    out = np.arange(g.n_branch)
    for els in cands:
        cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out)
        p1b, isl = O.n1_flows_bruteforce(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out)
        st = cf["state"]
        assert np.array_equal(isl & (st != 1), st == 2)
        ok = np.flatnonzero(st != 2)
        p1 = cf["p0"][:, None, :] + cf["lodf"].T[None] * cf["p0"][:, out][:, :, None]
        np.testing.assert_allclose(p1[:, ok], p1b[:, ok], atol=1e-10)


def test_bridges_match_bruteforce():
    rng = np.random.default_rng(7)
    for trial in range(30):
        n = int(rng.integers(3, 12))
        m = int(rng.integers(n - 1, 2 * n))
        f = rng.integers(0, n, m)
        t = (f + rng.integers(1, n, m)) % n
        br = O.bridges(n, f, t)
        base = O.connected(n, f, t)
        for e in range(m):
            keep = np.arange(m) != e
            if base:
                assert br[e] == (not O.connected(n, f[keep], t[keep]))


def test_single_edge_split_equals_outage():
    g, _, rng = _mixed_workload(5, n_cand=0)
    x = G.perturbed_injections(g, rng, (2,), 0.3)
    for a in np.flatnonzero(g.degree() >= 3)[:10]:
        inc = g.incident(int(a))
        for bit in range(1, len(inc)):
            split = [(G.KIND_SPLIT, int(a), 1 << bit, 0.0)]
            outage = [(G.KIND_OUTAGE, int(inc[bit]), 0, 0.0)]
            n2, f2, t2, al, _ = O.rebuild(g.n_bus, g.f, g.t, outage)
            if not O.connected(g.n_bus, f2[al], t2[al]):
                continue
            s = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, split, x, [])["p0"]
            o = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, outage, x, [])["p0"]
            np.testing.assert_allclose(s, o, atol=1e-12)


def test_complement_mask_gives_same_flows():
    g, _, rng = _mixed_workload(6, n_cand=0)
    x = G.perturbed_injections(g, rng, (1,), 0.3)
    for a in np.flatnonzero(g.degree() >= 3)[:12]:
        el = G.random_split(g, rng, int(a))
        d = len(g.incident(int(a)))
        comp = ((1 << d) - 1) ^ el[2]
        pn = 0.3
        one = [(G.KIND_SPLIT, int(a), el[2], pn)]
        two = [(G.KIND_SPLIT, int(a), comp, float(x[0, a]) - pn)]
        r1 = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, one, x, [])
        if not r1["connected"]:
            continue
        r2 = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, two, x, [])
        if int(a) == g.slack:
            continue   # the slack stays with busbar A, so the labels are not symmetric
        np.testing.assert_allclose(r1["p0"], r2["p0"], atol=1e-11)


def test_element_order_invariance():
    g, cands, rng = _mixed_workload(8, n_cand=10)
    x = G.perturbed_injections(g, rng, (3,), 0.2)
    out = np.arange(g.n_branch)
    r = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, out)
    for els in cands:
        if len(els) < 2:
            continue
        perm = list(reversed(els))
        a = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out, out, r)
        c = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, perm, x, out, out, r)
        np.testing.assert_allclose(a["max_load"], c["max_load"], rtol=1e-12)
        assert a["n_island"] == c["n_island"]


def test_disconnected_candidate_flagged():
    # a split that moves every branch but one of a degree-3 bus whose kept branch ...
    f = np.array([0, 1, 1, 2])
    t = np.array([1, 2, 3, 3])
    b = np.ones(4)
    # split bus 0 (degree 1 is not splittable) -> use outage of bridge 0-1 instead
    sc = O.score_candidate(4, f, t, b, 0, [(G.KIND_OUTAGE, 0, 0, 0.0)],
                           np.zeros((2, 4)), [1, 2], [1, 2], np.ones(2))
    assert sc["status"] & O.ST_DISCONNECTED
    assert np.all(np.isinf(sc["max_load"]))


# ------------------------------------------------ the paper's own formulas

def test_paper_lodf_definition_matches_rebuild():
    g = G.make_grid(20, 32, 11)
    h = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
    lodf = PF.lodf_matrix(h, g.f, g.t)
    cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, [], g.p, np.arange(g.n_branch))
    ok = cf["state"] == 0
    np.testing.assert_allclose(lodf[:, ok], cf["lodf"][:, ok], atol=1e-11)


def test_paper_modf_equals_sequential_lodf_and_rebuild():
    g = G.make_grid(20, 32, 12)
    h = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
    rng = np.random.default_rng(0)
    done = 0
    for _ in range(50):
        outs = rng.choice(g.n_branch, size=int(rng.integers(1, 5)), replace=False)
        al = np.ones(g.n_branch, bool)
        al[outs] = False
        if not O.connected(g.n_bus, g.f[al], g.t[al]):
            continue
        ref = O.ptdf(g.n_bus, g.f[al], g.t[al], g.b[al], g.slack)
        hm = PF.ptdf_after_modf(h, g.f, g.t, outs)
        hs = h
        for o in outs:
            hs = PF.ptdf_after_outage(hs, g.f, g.t, o)
        np.testing.assert_allclose(hm[al], ref, atol=1e-11)
        np.testing.assert_allclose(hs[al], ref, atol=1e-11)
        np.testing.assert_allclose(hm[~al], 0.0, atol=1e-11)   # row fix: no flow on outages
        done += 1
    assert done > 10


def test_paper_bsdf_matches_rebuild_including_slack_split():
    g = G.make_grid(16, 27, 3)
    h = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
    rng = np.random.default_rng(1)
    checked = set()
    for a in np.flatnonzero(g.degree() >= 3):
        inc = g.incident(int(a))
        for _ in range(3):
            el = G.random_split(g, rng, int(a))
            n2, f2, t2, al, _ = O.rebuild(g.n_bus, g.f, g.t, [el])
            if not O.connected(n2, f2, t2):
                continue
            moved = [int(inc[i]) for i in range(len(inc)) if (el[2] >> i) & 1]
            hp = PF.bsdf_split(h, g.f, g.t, g.b, int(a), moved, g.slack)
            np.testing.assert_allclose(hp, O.ptdf(n2, f2, t2, g.b, g.slack), atol=1e-11)
            checked.add(int(a))
    assert g.slack in checked


def test_repeated_bsdf_equals_joint_rebuild():
    # Eq. bsdf_application applied split after split equals the rebuilt grid
    g = G.make_grid(18, 30, 5)
    rng = np.random.default_rng(2)
    h0 = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
    n_ok = 0
    for _ in range(20):
        els = G.sample_candidate(g, rng, 2, 0)
        h = h0
        f2, t2 = g.f.copy(), g.t.copy()
        for (kind, a, m, _p) in els:
            inc = g.incident(a)
            moved = [int(inc[i]) for i in range(len(inc)) if (m >> i) & 1]
            # split on the current topology (the second split sees the first)
            h = PF.bsdf_split(h, f2, t2, g.b, a, moved, g.slack)
            newbus = h.shape[1] - 1
            for br in moved:
                if f2[br] == a:
                    f2[br] = newbus
                else:
                    t2[br] = newbus
        n2, rf, rt, _, _ = O.rebuild(g.n_bus, g.f, g.t, els)
        np.testing.assert_allclose(h, O.ptdf(n2, rf, rt, g.b, g.slack), atol=1e-10)
        n_ok += 1
    assert n_ok == 20


def test_fig1_packing_counts_fixture():
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fig1_packing.json")))
    ks = [len(c) for c in fx["candidates"]]
    assert sum(ks) == fx["naive_applications"]
    assert max(ks) * len(ks) == fx["padded_simd_applications"]
    # shared-prefix tree: distinct prefixes of the sorted split lists
    prefixes = {tuple(sorted(c)[:i + 1]) for c in fx["candidates"] for i in range(len(c))}
    assert len(prefixes) == fx["tree_applications"]


# ------------------------------------------------ controls (phase shifters, HVDC)

def test_pst_parallel_lines_closed_form():
    """Two parallel lines 0-1 (b1 carries a phase shifter of angle a), injection P
    at bus 1, slack 0: p_A = -(b1 P + b1 b2 a)/(b1 + b2), p_B = -(b2 P - b1 b2 a)/(b1 + b2)
    (a loop flow b1 b2 a/(b1 + b2) circulates)."""
    f, t = np.array([0, 0]), np.array([1, 1])
    b1, b2, P, a_deg = 4.0, 6.0, 0.7, 7.0
    b = np.array([b1, b2])
    a = np.deg2rad(a_deg)
    cf = O.candidate_flows(2, f, t, b, 0, [], np.array([[0.0, P]]), [],
                           controls=dict(pst=[0]), ctrl=np.array([[a_deg]]))
    p = cf["p0"][0]
    assert abs(p[0] - (-(b1 * P + b1 * b2 * a) / (b1 + b2))) < 1e-13
    assert abs(p[1] - (-(b2 * P - b1 * b2 * a) / (b1 + b2))) < 1e-13


def test_hvdc_on_a_tree_closed_form():
    """On a path graph an HVDC transfer of P from bus i to bus j loads every branch
    between them with P (in the direction j -> i in the AC network), the rest 0."""
    n = 6
    f, t = np.arange(n - 1), np.arange(1, n)
    b = np.linspace(1.0, 3.0, n - 1)
    P = 0.9   # level 3 at 0.3 p.u. per level
    cf = O.candidate_flows(n, f, t, b, 0, [], np.zeros((1, n)), [],
                           controls=dict(hvdc=[(1, 4)], hvdc_scale=0.3), ctrl=np.array([[3.0]]))
    p = cf["p0"][0]
    # bus 1 gives P, bus 4 takes P: the AC network returns P from 4 to 1 over branches 1..3
    np.testing.assert_allclose(p, [0.0, -P, -P, -P, 0.0], atol=1e-13)


def test_n1_with_controls_matches_bruteforce():
    """LODF superposition on N-0 flows with phase shifters and HVDC links equals
    re-solving every post-contingency network with the control model: with
    phase-shifter branches among the contingencies, a candidate that removes a
    shifter's branch (the shifter then does nothing) and candidates whose split
    moves a shifter's branch to the new busbar (the shift acts between its
    post-change terminals), as well as plain splits and outages."""
    w = G.workload_tiny(0)
    g = w.grid
    nb = np.flatnonzero(~O.bridges(g.n_bus, g.f, g.t))
    pst = [int(nb[0]), int(nb[4])]
    controls = dict(pst=pst, hvdc=[(3, 17), (8, 25)], hvdc_scale=0.25)
    rng = np.random.default_rng(2)
    ctrl = np.column_stack([rng.integers(-10, 11, size=(4, 2)), rng.integers(0, 8, size=(4, 2))])
    x = G.perturbed_injections(g, rng, (4,), 0.2)
    out = [int(c) for c in nb][:14]
    assert set(pst) <= set(out)
    a = int(np.flatnonzero(g.degree() >= 3)[2])

    def moving(branch, bus, extra_bit):
        # split of `bus` moving `branch` (and the incident branch of bit extra_bit)
        inc = list(O.incident_branches(g.f, g.t, bus))
        return (G.KIND_SPLIT, bus, (1 << inc.index(branch)) | (1 << extra_bit), 0.1)

    cands = [[], [(G.KIND_OUTAGE, out[5], 0, 0.0)], [(G.KIND_SPLIT, a, 2, 0.4)],
             [(G.KIND_OUTAGE, pst[1], 0, 0.0)],
             [moving(pst[1], int(g.t[pst[1]]), 0), (G.KIND_OUTAGE, out[6], 0, 0.0)],
             [moving(pst[0], int(g.t[pst[0]]), 0)], [moving(pst[1], int(g.f[pst[1]]), 0)]]
    n_checked = 0
    for els in cands:
        cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out, controls, ctrl)
        if not cf["connected"]:
            continue
        p1, isl = O.n1_flows_bruteforce(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out, controls,
                                        ctrl)
        for ci, c in enumerate(out):
            if cf["state"][ci] != 0:
                continue
            sup = cf["p0"] + cf["lodf"][:, ci][None, :] * cf["p0"][:, c][:, None]
            sup[:, c] = 0.0
            np.testing.assert_allclose(sup, p1[:, ci, :], atol=1e-10)
            n_checked += c in pst
    assert n_checked >= 8  # shifter contingencies checked across the candidates


def test_per_variant_busbar_injections_match_fixed_ones():
    """Injection topologies: a candidate whose split moves a different share of the
    substation's injection to the new busbar in each variant gives, variant by
    variant, the flows of the same candidate with that share as its fixed p_new;
    Kirchhoff's law holds at the new busbar with the moved injection."""
    w = G.workload_tiny(5)
    g = w.grid
    rng = np.random.default_rng(5)
    i = next(j for j in range(w.cands.n_cand) if any(e[0] == G.KIND_SPLIT for e in w.cands.elements(j)))
    el = w.cands.elements(i)
    x = np.repeat(np.atleast_2d(w.inj if w.inj_shared else w.inj[i])[:1], 6, axis=0)
    shares = rng.normal(0.0, 0.7, size=6)
    elv = [(k, b, m, shares if k == G.KIND_SPLIT else 0.0) for (k, b, m, _) in el]
    cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, elv, x, w.out)
    for v in range(6):
        elf = [(k, b, m, float(shares[v]) if k == G.KIND_SPLIT else 0.0) for (k, b, m, _) in el]
        one = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, elf, x[v:v + 1], w.out)
        np.testing.assert_allclose(cf["p0"][v], one["p0"][0], atol=1e-12)
    # balance at the new busbar: its branches carry the moved injection away
    n2, f2, t2, alive, splits = O.rebuild(g.n_bus, g.f, g.t, elv)
    a, bnew, pn = splits[0]
    for v in range(6):
        out_b = sum(cf["p0"][v][l] for l in range(len(f2)) if alive[l] and f2[l] == bnew) - \
            sum(cf["p0"][v][l] for l in range(len(f2)) if alive[l] and t2[l] == bnew)
        assert abs(out_b - pn[v]) < 1e-10


# ------------------------------------------------------- generator outages

def test_triangle_generator_outage_by_hand():
    # unit susceptances; bus 1 injects 1, bus 2 is a net load of 0.5 that holds a
    # 0.4 generator, the slack 0 another of 0.3.  N-0 = (1/2, 1/2, 0).  Losing the bus-2
    # generator adds -0.4 PTDF[:, 2] = -0.4 (1/3, -1/3, 2/3): (11/30, 19/30, -4/15);
    # losing the slack's changes nothing.  With ratings (1, 1/2, 1) the bus-2 case
    # gives the maximum 19/15 on edge 1.
    f = np.array([1, 1, 2])
    t = np.array([0, 2, 0])
    x = np.array([[-0.5, 1.0, -0.5]])
    r = np.array([1.0, 0.5, 1.0])
    gens = (np.array([0, 2]), np.array([0.3, 0.4]))
    sc = O.score_candidate(3, f, t, np.ones(3), 0, [], x, np.arange(3), [], r, gens=gens)
    np.testing.assert_allclose(sc["flows"]["gcol"][:, 1], [1 / 3, -1 / 3, 2 / 3], atol=1e-15)
    np.testing.assert_allclose(sc["flows"]["gcol"][:, 0], 0.0, atol=0)
    np.testing.assert_allclose(sc["loads_best"][2], [11 / 30, 19 / 15, 4 / 15], atol=1e-15)
    assert sc["best_max_load"] == pytest.approx(19 / 15, abs=1e-14)
    assert (sc["worst_branch"], sc["worst_outage"]) == (1, -3)
    assert sc["overload_sum"] == pytest.approx(4 / 15, abs=1e-14)
    got = O.worst_cases(sc, np.arange(3), np.zeros(0, np.int64), 6)
    want = [(19 / 15, 1, -3), (1.0, 1, -1), (1.0, 1, -2), (0.5, 0, -1), (0.5, 0, -2),
            (11 / 30, 0, -3)]
    np.testing.assert_allclose([v for v, _, _ in got], [v for v, _, _ in want], atol=1e-14)
    # the slack generator's case equals N-0 bit for bit, so the ties are ordered by case
    assert [(b, o) for _, b, o in got] == [(b, o) for _, b, o in want]


@pytest.mark.parametrize("seed", [0, 1])
def test_generator_outages_match_bruteforce(seed):
    """-P_g PTDF'[:, bus] on the candidate network equals solving that network
    again without the generator's output, for a generator at every bus (split
    buses, whose generator stays on busbar A, and the slack included)."""
    g, cands, rng = _mixed_workload(seed, n_cand=10)
    x = G.perturbed_injections(g, rng, (2,), 0.3)
    gens = (np.arange(g.n_bus), 0.2 + rng.uniform(0.0, 1.0, g.n_bus))
    out = np.arange(0, g.n_branch, 7)
    n_split = 0
    for els in cands:
        for k, (kind, d, m, _p) in enumerate(els):
            if kind == G.KIND_SPLIT:
                els[k] = (kind, d, m, float(rng.normal()))    # move some injection too
                n_split += 1
        cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out, gens=gens)
        if not cf["connected"]:
            continue
        p1b, isl = O.n1_flows_bruteforce(g.n_bus, g.f, g.t, g.b, g.slack, els, x, out, gens=gens)
        assert not isl[len(out):].any()
        pg = cf["p0"][:, None, :] - gens[1][None, :, None] * cf["gcol"].T[None]
        np.testing.assert_allclose(pg, p1b[:, len(out):], atol=1e-10)
        np.testing.assert_allclose(cf["gcol"][:, g.slack], 0.0, atol=0)
    assert n_split > 0


def test_generator_outages_in_the_score():
    """The score's maximum covers the generator cases: it equals the largest load
    over N-0, the non-islanding branch contingencies and the generator outages,
    each taken from the brute-force re-solves; generator cases are reported as
    -2 - g."""
    w = G.workload_tiny(3)
    g = w.grid
    rng = np.random.default_rng(3)
    gens = G.generator_outages(g, rng, 8)
    assert len(gens[0]) == 8 and np.all(gens[1] > 0)
    r = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, 1.0, 0.05)
    x = G.perturbed_injections(g, rng, (3,), 0.2)
    n_gen_worst = 0
    for i in range(12):
        els = w.cands.elements(i)
        sc = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, els, x, w.mon, w.out, r,
                               gens=gens)
        if sc["best_variant"] < 0:
            continue
        p1b, isl = O.n1_flows_bruteforce(g.n_bus, g.f, g.t, g.b, g.slack, els, x, w.out,
                                         gens=gens)
        p0 = sc["flows"]["p0"]
        loads = [np.abs(p0[:, w.mon]) / r]
        loads += [np.abs(p1b[:, c, w.mon]) / r for c in np.flatnonzero(~isl)]
        want = np.max(np.stack(loads, 1), axis=(1, 2))
        np.testing.assert_allclose(sc["max_load"], want, atol=1e-10)
        n_gen_worst += sc["worst_outage"] <= -2
        assert -2 - len(gens[0]) < sc["worst_outage"] < g.n_branch
    assert n_gen_worst >= 1     # a generator case is the worst one at least once


# ------------------------------------------------------- multi-outage cases

def test_multi_outage_by_hand():
    # buses 0 (slack), 1, 2; two unit lines 1-0 (branches 0, 1) and the detour
    # 1 -> 2 -> 0 (branches 2, 3); +1 at bus 1.  N-0: 0.4 on each direct line, 0.2 on
    # the detour.  Tripping {0, 1} sends everything over the detour (1, 1); {0, 2}
    # leaves line 1 alone (1) and bus 2 hanging on branch 3 (0); {2, 3} islands bus 2.
    # Rating 0.9 on branch 3 makes (branch 3, case {0, 1}) the unique maximum 1/0.9.
    f = np.array([1, 1, 1, 2])
    t = np.array([0, 0, 2, 0])
    x = np.array([[-1.0, 1.0, 0.0]])
    r = np.array([1.0, 1.0, 1.0, 0.9])
    mon = out = np.arange(4)
    multi = [[0, 1], [0, 2], [2, 3]]
    pm, isl = O.multi_outage_flows(3, f, t, np.ones(4), 0, [], x, multi)
    np.testing.assert_allclose(pm[0, 0], [0, 0, 1, 1], atol=1e-15)
    np.testing.assert_allclose(pm[0, 1], [0, 1, 0, 0], atol=1e-15)
    assert list(isl) == [False, False, True]
    sc = O.score_candidate(3, f, t, np.ones(4), 0, [], x, mon, out, r, multi=multi)
    np.testing.assert_allclose(sc["flows"]["p0"][0], [0.4, 0.4, 0.2, 0.2], atol=1e-15)
    assert sc["best_max_load"] == pytest.approx(1 / 0.9, abs=1e-14)
    assert (sc["worst_branch"], sc["worst_outage"]) == (3, -2)
    assert sc["n_island"] == 1
    got = O.worst_cases(sc, mon, out, 4)
    assert [(b, o) for _, b, o in got] == [(3, -2), (2, -2), (1, -3), (1, 0)]
    np.testing.assert_allclose([v for v, _, _ in got], [1 / 0.9, 1.0, 1.0, 2 / 3], atol=1e-14)
    # a remedial outage of branch 0: case {0, 1} trips branch 1 alone, with the same flows
    sc2 = O.score_candidate(3, f, t, np.ones(4), 0, [(G.KIND_OUTAGE, 0, 0, 0.0)], x, mon, out,
                            r, multi=multi)
    assert sc2["best_max_load"] == pytest.approx(1 / 0.9, abs=1e-14)
    assert (sc2["worst_branch"], sc2["worst_outage"]) in {(3, 1), (3, -2)}


@pytest.mark.parametrize("seed", [0, 1])
def test_multi_outage_matches_paper_modf(seed):
    """Re-solving the candidate network without a case's branches equals the
    paper's MODF (Def. eq_modf) applied to the candidate network's PTDF: p0 + MODF
    p0[S] (branches the candidate removed left out of S)."""
    g, cands, rng = _mixed_workload(seed, n_cand=10)
    x = G.perturbed_injections(g, rng, (2,), 0.3)
    out = np.arange(0, g.n_branch, 3)
    multi = G.multi_outage_cases(g, out, rng, 12)
    n_checked = n_isl = 0
    for els in cands:
        n2, f2, t2, alive, splits = O.rebuild(g.n_bus, g.f, g.t, els)
        fa, ta, ba = f2[alive], t2[alive], np.asarray(g.b)[alive]
        if not O.connected(n2, fa, ta):
            continue
        pm, isl = O.multi_outage_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, multi)
        p0 = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x, [])["p0"]
        h = O.ptdf(n2, fa, ta, ba, g.slack)
        idx = -np.ones(len(f2), np.int64)
        idx[alive] = np.arange(int(alive.sum()))
        for qi, case in enumerate(multi):
            s_alive = [int(idx[c]) for c in case if alive[c]]
            if isl[qi]:
                n_isl += 1
                continue
            if not s_alive:
                np.testing.assert_allclose(pm[:, qi], p0, atol=1e-12)
                continue
            md = PF.modf(h, fa, ta, s_alive)
            want = p0[:, alive] + (md @ p0[:, alive][:, s_alive].T).T
            np.testing.assert_allclose(pm[:, qi][:, alive], want, atol=1e-10)
            n_checked += 1
    assert n_checked > 50 and n_isl > 0


def test_multi_outage_order_with_generators():
    """Case order: branch contingencies, then generator outages (-2 - g), then
    multi-outage cases (-2 - G - q); every listed case carries its own load."""
    w = G.workload_tiny(4)
    g = w.grid
    rng = np.random.default_rng(4)
    gens = G.generator_outages(g, rng, 5)
    multi = G.multi_outage_cases(g, w.out, rng, 10)
    r = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, 1.0, 0.05)
    seen_multi = 0
    for i in range(10):
        els = w.cands.elements(i)
        sc = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, els, w.inj, w.mon, w.out, r,
                               gens=gens, multi=multi)
        if sc["best_variant"] < 0:
            continue
        ids = sc["scored_out"]
        nb = int((ids >= 0).sum())
        assert np.all(ids[:nb] >= 0)
        assert np.all(ids[nb:nb + 5] == -2 - np.arange(5))
        assert np.all(ids[nb + 5:] <= -7)
        pm, isl = O.multi_outage_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, w.inj, multi)
        for v, b, o in O.worst_cases(sc, w.mon, w.out, 16):
            if o <= -7:
                q = -7 - o
                assert not isl[q]
                li = int(np.flatnonzero(w.mon == b)[0])
                assert v == pytest.approx(abs(pm[0, q, b]) / r[li], abs=1e-12)
                seen_multi += 1
    assert seen_multi > 0


def test_two_level_worst_cases_by_hand():
    # the triangle of test_triangle_worst_cases_by_hand: losing edge 2 loads (1.5, 0.5, 0),
    # edge 0 (0, 1, 1.25), edge 1 (1, 0, 5/12), N-0 (5/6, 1/6, 5/9).  One place per case:
    # each case's maximum, ordered by load.
    f = np.array([1, 1, 2])
    t = np.array([0, 2, 0])
    x = np.array([[-1.5, 1.0, 0.5]])
    r = np.array([1.0, 1.0, 1.2])
    mon = out = np.arange(3)
    sc = O.score_candidate(3, f, t, np.ones(3), 0, [], x, mon, out, r)
    got = O.worst_cases_per_case(sc, mon, out, 1, 7)
    assert [(b, o) for _, b, o in got] == [(0, 2), (2, 0), (0, 1), (0, -1)]
    np.testing.assert_allclose([v for v, _, _ in got], [1.5, 1.25, 1.0, 5 / 6], atol=1e-14)
    two = O.worst_cases_per_case(sc, mon, out, 2, 3)
    assert [(b, o) for _, b, o in two[:2]] == [(0, 2), (2, 0)]


@pytest.mark.parametrize("seed", [0, 1])
def test_two_level_worst_cases_reduce_to_global(seed):
    """With per_case >= k the two levels give the global top-k; with a smaller cap
    no case holds more than per_case places and every listed load is at least the
    load of any case's first left-out entry that could have entered."""
    w = G.workload_tiny(seed)
    g = w.grid
    rng = np.random.default_rng(seed)
    gens = G.generator_outages(g, rng, 4)
    multi = G.multi_outage_cases(g, w.out, rng, 5)
    r = O.ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon, 1.0, 0.05)
    for i in range(6):
        sc = O.score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, w.cands.elements(i), w.inj,
                               w.mon, w.out, r, gens=gens, multi=multi)
        assert O.worst_cases_per_case(sc, w.mon, w.out, 16, 16) == \
            O.worst_cases(sc, w.mon, w.out, 16)
        capped = O.worst_cases_per_case(sc, w.mon, w.out, 2, 16)
        if not capped:
            continue
        outs = [o for _, _, o in capped]
        assert max(outs.count(o) for o in set(outs)) <= 2
        assert len(capped) == min(16, 2 * sc["loads_best"].shape[0])
        assert all(a[0] >= b[0] for a, b in zip(capped, capped[1:]))
