"""FP64 reference of the learned proposal network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the solver library.

The network ranks single-bus-split actions so that the exact solver evaluates
the most promising first (an addition to the paper, whose optimiser that
proposes candidates is out of its scope, Sec. III-A).  This module restates it
plainly so the GPU kernels can be checked:

  * per-action features from the base-case flows of a load snapshot, among
    them the exact post-split N-1 loads of the snapshot's K_PAIRS worst
    (branch, contingency) pairs of the unchanged grid, by plain rebuild;
  * a 3-layer perceptron d_in -> 256 -> 256 -> 1 with ReLU;
  * mean squared error on standardised labels, its gradients by the chain rule;
  * one Adam step (Kingma & Ba, 2015) with bias correction.

Parity of the gradients is pinned by central finite differences.
"""
from __future__ import annotations

import numpy as np

D_MAX = 14            # incident-branch slots per action
N_SLOT_FEAT = 5       # oriented flow / r, moved bit, present bit, sigma, sigma * flow / r*
K_PAIRS = 8           # tracked (branch, contingency) pairs per snapshot
N_FEAT = 4 + D_MAX * N_SLOT_FEAT + 2 + K_PAIRS + 2   # 86
D_IN = 96             # padded input width
X_PAIRS = 4 + D_MAX * N_SLOT_FEAT + 2                # first pair-load slot (76)


def critical_row(h, f, t, l_star, c_star):
    """Sensitivity of the critical post-contingency flow to nodal injections:
    PTDF[l*, :] + LODF[l*, c*] PTDF[c*, :] (Def. eq_lodf, Eq. lodf_delta applied
    to the PTDF); c* = -1 means the N-0 case (row l* alone)."""
    if c_star < 0:
        return h[l_star].copy()
    d = h[:, f[c_star]] - h[:, t[c_star]]
    lw = d[l_star] / (1.0 - d[c_star])
    return h[l_star] + lw * h[c_star]


def base_pairs(n, f, t, b, slack, p, mon, out, rating, k=K_PAIRS):
    """The k largest relative loads of the unchanged grid under injections p,
    over N-0 rows and every non-islanding contingency (Sec. III-A loads), as
    (branch l, contingency branch c or -1, load); ties go to the lower
    position in the order N-0 rows first, then contingency-major."""
    from . import dcflow_oracle as O
    o = O.score_candidate(n, f, t, b, slack, [], p, mon, out, rating)
    L = o["loads_best"]            # [1 + scored][n_mon], rows in that order
    sc = o["scored_out"]
    flat = L.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))[:k]
    res = []
    for q in order:
        ci, li = divmod(int(q), len(mon))
        res.append((int(mon[li]), -1 if ci == 0 else int(sc[ci - 1]), float(flat[q])))
    return res


def split_pair_loads(n, f, t, b, slack, p, bus, mask, inj_moves, pairs, rating_of):
    """Exact loads of the tracked pairs after one split of ``bus`` (branches of
    ``mask`` to the new busbar, the bus injection with them if inj_moves):
    the split network is rebuilt and its N-0 flows and LODF computed directly
    (Def. eq_lodf, Eq. lodf_delta).  A pair whose contingency islands the split
    network keeps its N-0 load.  Returns (loads [len(pairs)], connected)."""
    from . import dcflow_oracle as O
    pnew = p[bus] if inj_moves else 0.0
    outs = [c for _, c in pairs if c >= 0]
    cf = O.candidate_flows(n, f, t, b, slack, [(O.KIND_SPLIT, bus, mask, pnew)], p, outs)
    if not cf["connected"]:
        return np.zeros(len(pairs)), False
    p0 = cf["p0"][0]
    res, k = [], 0
    for (l, c) in pairs:
        v = p0[l]
        if c >= 0:
            if cf["state"][k] == 0:
                v = p0[l] + cf["lodf"][l, k] * p0[c]
            k += 1
        res.append(abs(v) / rating_of[l])
    return np.asarray(res), True


def improvement_label(max_load, base_max):
    """Training label: log of the candidate's maximum load relative to the
    unchanged grid's, clipped at 0 (no gain); an islanded candidate gets 0."""
    if not np.isfinite(max_load):
        return 0.0
    return min(np.log(max_load / base_max), 0.0)


def action_features(n_bus, f, t, flows, rating_all, p, bus, mask, inj_moves, glob2, rho, r_star,
                    pair_loads=None, connected=True):
    """Feature vector of one split action (float64 [D_IN]).

    flows: base-case flows of the snapshot on every branch; rating_all: per
    branch normaliser; p: snapshot injections; glob2: (max N-0 load, max N-1
    load) of the snapshot's unchanged grid; rho: critical_row(...) of its worst
    case, r_star the normaliser of that case's monitored branch."""
    inc = np.flatnonzero((np.asarray(f) == bus) | (np.asarray(t) == bus))
    x = np.zeros(D_IN)
    x[0] = len(inc)
    x[1] = p[bus]
    x[2] = 1.0 if inj_moves else 0.0
    x[3] = rho[bus]
    for q, br in enumerate(inc[:D_MAX]):
        leaves = f[br] == bus
        far = t[br] if leaves else f[br]
        fo = (1.0 if leaves else -1.0) * flows[br]
        sig = rho[bus] - rho[far]
        base = 4 + q * N_SLOT_FEAT
        x[base + 0] = fo / rating_all[br]
        x[base + 1] = 1.0 if (mask >> q) & 1 else 0.0
        x[base + 2] = 1.0
        x[base + 3] = sig
        x[base + 4] = sig * fo / r_star
    x[4 + D_MAX * N_SLOT_FEAT + 0] = glob2[0]
    x[4 + D_MAX * N_SLOT_FEAT + 1] = glob2[1]
    if pair_loads is not None:
        if connected:
            x[X_PAIRS:X_PAIRS + K_PAIRS] = pair_loads
            x[X_PAIRS + K_PAIRS] = np.max(pair_loads)
        else:
            x[X_PAIRS + K_PAIRS + 1] = 1.0
    return x


def init_params(rng, d_in=D_IN, h=256):
    """He-uniform initialisation, FP64."""
    def lin(fan_in, fan_out):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, (fan_in, fan_out)), np.zeros(fan_out)
    w1, b1 = lin(d_in, h)
    w2, b2 = lin(h, h)
    w3, b3 = lin(h, 1)
    return dict(w1=w1, b1=b1, w2=w2, b2=b2, w3=w3, b3=b3)


def forward(params, x):
    """Returns (y [B], cache)."""
    z1 = x @ params["w1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["w2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ params["w3"] + params["b3"])[:, 0]
    return y, (x, z1, h1, z2, h2)


def round_bf16(a):
    """Round to the nearest bfloat16 value, ties to even (the 8-bit-significand
    format: the upper 16 bits of an IEEE binary32), returned as float64.  The
    input is first rounded to binary32 (the width the GPU holds it in)."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep = (u >> 16) & 1                       # last kept bit: the tie goes to even
    r = ((u + 0x7FFF + keep) >> 16) << 16
    nan = np.isnan(np.asarray(a, dtype=np.float32))
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def forward_bf16(params, x):
    """The forward pass as BF16 inference defines it: the inputs and the first two
    weight matrices in bfloat16, the first layer's activations stored in bfloat16
    before the second product, every product summed in wide precision (here
    FP64), biases, the last layer and the output in full precision."""
    xb = round_bf16(x)
    z1 = xb @ round_bf16(params["w1"]) + params["b1"]
    h1 = round_bf16(np.maximum(z1, 0.0))
    z2 = h1 @ round_bf16(params["w2"]) + params["b2"]
    h2 = np.maximum(z2, 0.0)
    return (h2 @ params["w3"] + params["b3"])[:, 0]


def loss(params, x, target):
    y, _ = forward(params, x)
    return float(np.mean((y - target) ** 2))


def backward(params, x, target):
    """Gradients of the mean squared error with respect to every parameter."""
    y, (x, z1, h1, z2, h2) = forward(params, x)
    bsz = x.shape[0]
    dy = (2.0 / bsz) * (y - target)[:, None]          # [B, 1]
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ params["w3"].T
    dz2 = dh2 * (z2 > 0)
    g["w2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["w2"].T
    dz1 = dh1 * (z1 > 0)
    g["w1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; ``step`` counts from 1."""
    for k in params:
        m[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] ** 2
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
