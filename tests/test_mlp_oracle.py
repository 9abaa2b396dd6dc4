"""Pins of the FP64 reference MLP: finite differences, the first Adam step in
closed form, and a hand-checked feature vector."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(rng, d_in=12, h=16)
    x = rng.normal(size=(9, 12))
    t = rng.normal(size=9)
    g = M.backward(p, x, t)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp = M.loss(p, x, t)
            flat[i] = old - eps
            lm = M.loss(p, x, t)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, an)


def test_first_adam_step_closed_form():
    # with zero moments, step 1 moves each parameter by lr * g / (|g| + eps') ~ lr * sign(g)
    rng = np.random.default_rng(1)
    p = M.init_params(rng, d_in=5, h=4)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    before = {k: x.copy() for k, x in p.items()}
    M.adam_step(p, g, m, v, 1, lr=0.01, eps=1e-8)
    for k in p:
        expect = before[k] - 0.01 * g[k] / (np.abs(g[k]) + 1e-8)
        np.testing.assert_allclose(p[k], expect, rtol=1e-12, atol=1e-15)


def test_feature_vector_by_hand():
    # triangle 1->0, 1->2, 2->0; action: split bus 1 moving its second branch (id 1)
    f = np.array([1, 1, 2])
    t = np.array([0, 2, 0])
    flows = np.array([0.5, -0.25, 0.75])
    r = np.array([1.0, 2.0, 4.0])
    p = np.array([-1.0, 0.25, 0.75])
    rho = np.array([0.0, 0.6, 0.2])
    x = M.action_features(3, f, t, flows, r, p, 1, 0b10, True, (0.3, 0.9), rho, 2.0)
    assert x.shape == (M.D_IN,)
    assert (x[0], x[1], x[2], x[3]) == (2.0, 0.25, 1.0, 0.6)
    # slot 0 = branch 0 (leaves bus 1 towards 0): flow 0.5 / 1, sigma 0.6 - 0.0
    np.testing.assert_allclose(x[4:9], [0.5, 0.0, 1.0, 0.6, 0.6 * 0.5 / 2.0])
    # slot 1 = branch 1 (leaves bus 1 towards 2), moved: flow -0.25 / 2, sigma 0.6 - 0.2
    np.testing.assert_allclose(x[9:14], [-0.125, 1.0, 1.0, 0.4, 0.4 * -0.25 / 2.0])
    assert np.all(x[14:4 + M.D_MAX * M.N_SLOT_FEAT] == 0)
    np.testing.assert_allclose(x[74:76], [0.3, 0.9])
    assert np.all(x[76:] == 0)


def test_critical_row_is_post_contingency_sensitivity():
    # the critical row equals the PTDF row of l* in the grid without c* (brute force)
    from oracle import dcflow_oracle as O
    import gridgen as G
    g = G.make_grid(14, 22, 2)
    h = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
    nb = np.flatnonzero(~O.bridges(g.n_bus, g.f, g.t))
    l_star, c_star = int(nb[0]), int(nb[3])
    keep = np.arange(g.n_branch) != c_star
    h2 = O.ptdf(g.n_bus, g.f[keep], g.t[keep], g.b[keep], g.slack)
    row = M.critical_row(h, g.f, g.t, l_star, c_star)
    np.testing.assert_allclose(row, h2[np.flatnonzero(keep) == l_star][0], atol=1e-12)
    np.testing.assert_allclose(M.critical_row(h, g.f, g.t, l_star, -1), h[l_star])


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    p = M.init_params(rng, d_in=8, h=32)
    x = rng.normal(size=(256, 8))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] ** 2
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    l0 = M.loss(p, x, t)
    for step in range(1, 301):
        M.adam_step(p, M.backward(p, x, t), m, v, step, lr=3e-3)
    assert M.loss(p, x, t) < 0.2 * l0


def _tiny():
    import gridgen as G
    from oracle import dcflow_oracle as O
    w = G.workload_tiny(0)
    g = w.grid
    f, t, b = np.asarray(g.f), np.asarray(g.t), np.asarray(g.b)
    r = O.ratings(g.n_bus, f, t, b, g.slack, g.p, w.mon)
    r_of = np.zeros(len(f))
    r_of[np.asarray(w.mon)] = r
    return w, g, f, t, b, r, r_of


def test_split_pair_loads_match_bsdf_route():
    """Plain rebuild vs the paper's split factor (Def. eq_bsdf, Eq.
    bsdf_application) followed by the LODF of the post-split PTDF: the same
    post-split N-1 loads by two independent routes, slack-bus splits included."""
    from oracle import dcflow_oracle as O
    from oracle import paper_formulas as PF
    w, g, f, t, b, r, r_of = _tiny()
    n, sl = g.n_bus, g.slack
    h = O.ptdf(n, f, t, b, sl)
    rng = np.random.default_rng(11)
    p = g.p + 0.1 * rng.normal(size=n)
    mon, out = np.asarray(w.mon), np.asarray(w.out)
    deg = g.degree()
    buses = [sl] + [int(a) for a in np.flatnonzero(deg >= 3)[:6] if a != sl]
    checked = 0
    for a in buses:
        inc = np.flatnonzero((f == a) | (t == a))
        for mask in (2, (1 << len(inc)) - 2):
            for side in (0, 1):
                moved = [int(inc[q]) for q in range(len(inc)) if (mask >> q) & 1]
                pairs = [(int(mon[3]), -1), (int(mon[5]), int(out[7])), (int(mon[1]), int(inc[0])),
                         (int(inc[-1]), int(out[2]))]
                pairs = [(l, c) for l, c in pairs if l != c]
                got, ok = M.split_pair_loads(n, f, t, b, sl, p, a, mask, side, pairs, r_of)
                if not ok:
                    continue
                hs = PF.bsdf_split(h, f, t, b, a, moved, slack=sl)   # [m][n + 1], node B = n
                pe = np.concatenate([p, [0.0]])
                pn = p[a] if side else 0.0
                pe[a] -= pn
                pe[n] += pn
                p0 = hs @ pe
                f2 = f.copy()
                t2 = t.copy()
                for l in moved:
                    if f[l] == a:
                        f2[l] = n
                    else:
                        t2[l] = n
                ref = []
                for (l, c) in pairs:
                    v = p0[l]
                    if c >= 0:
                        dlt = hs[:, f2[c]] - hs[:, t2[c]]
                        den = 1.0 - dlt[c]
                        if abs(den) > 1e-9:
                            v = p0[l] + dlt[l] / den * p0[c]
                    ref.append(abs(v) / r_of[l])
                np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12)
                checked += 1
    assert checked >= 10


def test_base_pairs_match_brute_force():
    from oracle import dcflow_oracle as O
    w, g, f, t, b, r, r_of = _tiny()
    n, sl = g.n_bus, g.slack
    mon, out = np.asarray(w.mon), np.asarray(w.out)
    p = g.p
    pairs = M.base_pairs(n, f, t, b, sl, p, mon, out, r, k=8)
    p1, isl = O.n1_flows_bruteforce(n, f, t, b, sl, [], p, out)
    p0 = O.dc_flows(n, f, t, b, sl, p)[0]
    cand = [(abs(p0[l]) / r_of[l], (0, i), int(l), -1) for i, l in enumerate(mon)]
    for ci, c in enumerate(out):
        if isl[ci]:
            continue
        for i, l in enumerate(mon):
            cand.append((abs(p1[0, ci, l]) / r_of[l], (ci + 1, i), int(l), int(c)))
    cand.sort(key=lambda z: (-z[0], z[1]))
    for (l, c, v), ref in zip(pairs, cand[:8]):
        assert abs(v - ref[0]) <= 1e-9 * max(1.0, ref[0])
        assert (l, c) == (ref[2], ref[3])


def test_improvement_label():
    assert M.improvement_label(np.inf, 2.0) == 0.0
    assert M.improvement_label(3.0, 2.0) == 0.0
    assert abs(M.improvement_label(1.0, 2.0) - np.log(0.5)) < 1e-15


def test_pair_slots_of_the_feature_vector():
    w, g, f, t, b, r, r_of = _tiny()
    x = M.action_features(g.n_bus, f, t, np.zeros(len(f)), np.ones(len(f)), g.p, 3, 2, False,
                          (0.5, 0.7), np.zeros(g.n_bus), 1.0, pair_loads=np.arange(8.0) / 8.0)
    np.testing.assert_array_equal(x[M.X_PAIRS:M.X_PAIRS + 8], np.arange(8.0) / 8.0)
    assert x[M.X_PAIRS + 8] == 7.0 / 8.0 and x[M.X_PAIRS + 9] == 0.0
    y = M.action_features(g.n_bus, f, t, np.zeros(len(f)), np.ones(len(f)), g.p, 3, 2, False,
                          (0.5, 0.7), np.zeros(g.n_bus), 1.0, pair_loads=np.ones(8), connected=False)
    assert not y[M.X_PAIRS:M.X_PAIRS + 9].any() and y[M.X_PAIRS + 9] == 1.0


def test_round_bf16_by_hand_and_against_torch():
    """Round-to-nearest-even onto the 8-bit significand: hand values at and
    around the halfway points, then agreement with torch's CPU conversion."""
    import torch
    r = M.round_bf16
    one = 1.0
    assert r(one) == 1.0
    assert r(1 + 2 ** -8) == 1.0                      # tie, 1.0 is even
    assert r(1 + 3 * 2 ** -8) == 1 + 2 ** -6          # tie, rounds up to the even neighbour
    assert r(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7   # above the tie
    assert r(-(1 + 2 ** -8 + 2 ** -20)) == -(1 + 2 ** -7)
    assert r(0.0) == 0.0 and np.isnan(r(np.nan))
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-6, 6, size=20000),
                        np.float32(1.0) + np.arange(-300, 300) * np.float32(2 ** -16)])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(r(v), ref)


def test_bf16_forward_exact_on_representable_values():
    """With integer inputs and weights in {-1, 0, 1} (second layer over 64) every
    operand and first-layer activation is a bfloat16 value, so BF16 inference
    equals the FP64 forward; a weight moved by less than half a bfloat16 step
    changes the FP64 forward but not the BF16 one."""
    rng = np.random.default_rng(1)
    p = M.init_params(rng)
    p["w1"] = rng.integers(-1, 2, size=p["w1"].shape).astype(np.float64)
    p["w1"][0, :] = 1.0
    p["w2"] = rng.integers(-1, 2, size=p["w2"].shape).astype(np.float64) / 64.0
    x = rng.integers(-2, 3, size=(5, M.D_IN)).astype(np.float64)
    x[:, 0] = 1.0
    y, _ = M.forward(p, x)
    assert np.array_equal(M.forward_bf16(p, x), y)
    q = {k: v.copy() for k, v in p.items()}
    q["w1"][0, :] = 1.0 + 2 ** -12
    assert np.array_equal(M.forward_bf16(q, x), y)
    assert not np.array_equal(M.forward(q, x)[0], y)
