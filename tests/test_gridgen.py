"""Seeded synthetic inputs: determinism and structural guarantees."""
import numpy as np

import gridgen as G


def test_grid_is_deterministic_and_connected():
    a = G.make_grid(200, 320, 5)
    b = G.make_grid(200, 320, 5)
    for k in ("f", "t", "x", "b", "p", "pos"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.n_branch == 320
    assert G.is_connected(a.n_bus, a.f, a.t)
    assert abs(a.p.sum()) < 1e-12
    assert np.all(a.f != a.t)
    pairs = {(min(u, v), max(u, v)) for u, v in zip(a.f, a.t)}
    assert len(pairs) == a.n_branch          # no parallel branches


def test_tiny_workload_shape():
    w = G.workload_tiny(0)
    assert (w.grid.n_bus, w.grid.n_branch, w.cands.n_cand) == (30, 41, 100)
    assert np.all(np.diff(w.cands.off) == 1)
    assert np.all(w.cands.kind == G.KIND_SPLIT)
    assert w.inj.shape == (1, 30) and w.inj_shared


def test_candidates_are_connected_and_canonical():
    w = G.workload_medium(0, n_cand=64, n_var=2, n_out=50)
    g = w.grid
    k = np.diff(w.cands.off)
    assert k.min() >= 1 and k.max() <= 5
    for i in range(w.cands.n_cand):
        els = w.cands.elements(i)
        n2, f, t, alive = G.candidate_topology(g, els)
        assert G.is_connected(n2, f, t, alive)
        buses = [d for (kd, d, m, p) in els if kd == G.KIND_SPLIT]
        assert len(buses) == len(set(buses))
        for (kd, d, m, p) in els:
            if kd == G.KIND_SPLIT:
                deg = len(g.incident(d))
                assert m & 1 == 0 and m != 0 and m < (1 << deg)
    # contingencies are non-bridges of the base grid
    for c in w.out:
        al = np.ones(g.n_branch, bool)
        al[c] = False
        assert G.is_connected(g.n_bus, g.f, g.t, al)
    # injections balanced per variant
    assert np.abs(w.inj.sum(axis=-1)).max() < 1e-9


def test_workload_seed_reproducible():
    a = G.workload_medium(3, n_cand=16, n_var=2, n_out=20)
    b = G.workload_medium(3, n_cand=16, n_var=2, n_out=20)
    for k in ("off", "kind", "id", "mask", "p_new"):
        assert np.array_equal(getattr(a.cands, k), getattr(b.cands, k))
    assert np.array_equal(a.inj, b.inj) and np.array_equal(a.out, b.out)
