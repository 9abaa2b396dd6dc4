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
