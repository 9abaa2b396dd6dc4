"""Learned proposal for single-bus-split actions (an addition to the paper).

A 96 -> 256 -> 256 -> 1 ReLU perceptron, trained on the GPU by the library's
own kernels on maximum-load labels produced by the exact screen, scores every
single-split action of a load snapshot; the exact screen then verifies the
best-scored ones.  Exhaustive screening stays the fallback and the arbiter.

All arithmetic runs in libdcflow kernels (features, standardisation, forward,
backward, Adam, BF16 inference, top-k, exact screen); this module only
allocates device buffers and sequences the calls.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import dcflow as D

_lib = D._lib
P = ctypes.c_void_p
PAIRS = 8  # tracked (branch, contingency) pairs per snapshot


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _chk(rc, what):
    D._check(rc, what)


def enumerate_actions(grid, max_deg=14):
    """All single-split actions: (bus, canonical mask, side) with bus degree in
    [3, max_deg]; the mask keeps the first incident branch on busbar A; side 1
    moves the bus injection to the new busbar."""
    deg = grid.degree()
    bus, mask, side = [], [], []
    for a in np.flatnonzero((deg >= 3) & (deg <= max_deg)):
        d = int(deg[a])
        for m in range(1, 1 << (d - 1)):
            for sd in (0, 1):
                bus.append(int(a))
                mask.append(m << 1)
                side.append(sd)
    return (np.asarray(bus, np.int32), np.asarray(mask, np.uint32), np.asarray(side, np.int32))


def action_candidates(bus, mask, side, x_snap):
    """Candidate records of single-split actions for one snapshot: the moved
    injection p_new is the bus's snapshot injection when side is 1."""
    n = len(bus)
    off = np.arange(n + 1, dtype=np.int32)
    kind = np.full(n, 1, np.int8)
    p_new = np.where(side != 0, x_snap[bus], 0.0).astype(np.float64)

    class _C:
        pass
    c = _C()
    c.off, c.kind, c.id, c.mask, c.p_new = off, kind, bus.astype(np.int32), mask, p_new
    return c


def exact_scores(plan, cands, x_snap, prec="fp32"):
    """max_load of every candidate under one snapshot (exact screen, V = 1)."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(x_snap[None, :])).cuda()
    sc, _, _ = D.screen(plan, cands, x, 1, True, prec)
    return sc["max_load"].copy()


class Proposal:
    """Device-resident network state: FP32 master weights, Adam moments, BF16
    inference copies and the feature / label standardisation constants."""

    def __init__(self, plan: "D.Plan", seed: int = 0):
        import torch
        self.plan = plan
        self.np_ = _lib.dcflow_mlp_param_count()
        rng = np.random.default_rng(seed)
        p = np.zeros(self.np_, np.float32)
        din, h = 96, 256

        def fill(off, fan_in, size):
            lim = np.sqrt(6.0 / fan_in)
            p[off:off + size] = rng.uniform(-lim, lim, size)
        o_w1 = 0
        o_b1 = o_w1 + din * h
        o_w2 = o_b1 + h
        o_b2 = o_w2 + h * h
        o_w3 = o_b2 + h
        fill(o_w1, din, din * h)
        fill(o_w2, h, h * h)
        fill(o_w3, h, h)
        dev = "cuda"
        self.params = torch.from_numpy(p).to(dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.bf16 = torch.empty(_lib.dcflow_mlp_bf16_bytes(), dtype=torch.uint8, device=dev)
        self.mu = torch.zeros(96, dtype=torch.float32, device=dev)
        self.isd = torch.ones(96, dtype=torch.float32, device=dev)
        self.t_mu = torch.zeros(1, dtype=torch.float32, device=dev)
        self.t_isd = torch.ones(1, dtype=torch.float32, device=dev)
        self.step = 0

    # ------------------------------------------------------------ data
    def snapshot_summary(self, x_snap):
        """Device flows [S][m], per-snapshot (max N-0 load, max N-0/N-1 load) of
        the unchanged grid (the two global features) and its worst case
        (monitored branch, contingency or -1), which anchors the sensitivity
        features."""
        import torch
        S = x_snap.shape[0]
        x = torch.from_numpy(np.ascontiguousarray(x_snap)).cuda()
        flows = torch.empty((S, self.plan.view.n_branch), dtype=torch.float64, device="cuda")
        n0 = torch.empty(S, dtype=torch.float64, device="cuda")
        s = D._stream()
        _chk(_lib.dcflow_snapshot_flows(self.plan.h, _ptr(x), S, _ptr(flows), _ptr(n0), s),
             "dcflow_snapshot_flows")
        # the unchanged grid under every snapshot: S empty candidates, one variant each
        empty = D._CandArgs(np.zeros(S + 1, np.int32), np.zeros(0, np.int8),
                            np.zeros(0, np.int32), np.zeros(0, np.uint32))
        bt = D.Batch(self.plan, empty, 1)
        bt.eval_topologies()
        fl = bt.eval_injections(x.view(S, 1, -1), 1, False, "fp64")
        out = bt.n1_score(fl, 1, "fp64")
        sc = D.Batch.scores_to_numpy(out, S)
        glob = torch.stack([n0, torch.from_numpy(sc["max_load"].copy()).cuda()], dim=1).contiguous()
        worst = np.stack([sc["worst_branch"], sc["worst_outage"]], axis=1).astype(np.int32)
        self.worst_host = worst
        self.worst = torch.from_numpy(np.ascontiguousarray(worst)).cuda()
        # the snapshot's worst (branch, contingency) pairs, tracked through each split
        self.pairs = torch.empty((S, PAIRS, 2), dtype=torch.int32, device="cuda")
        self.pair_loads = torch.empty((S, PAIRS), dtype=torch.float64, device="cuda")
        _chk(_lib.dcflow_snapshot_pairs(self.plan.h, _ptr(flows), S, _ptr(self.pairs),
                                        _ptr(self.pair_loads), s), "dcflow_snapshot_pairs")
        self.glob = glob
        return x, flows, glob

    def features(self, x_dev, flows, glob, snap, bus, mask, side):
        import torch
        n = len(bus)
        feat = torch.empty((n, 96), dtype=torch.float32, device="cuda")
        arrs = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
                for a in (snap.astype(np.int32), bus.astype(np.int32), mask.astype(np.int32),
                          side.astype(np.int32))]
        _chk(_lib.dcflow_action_features(self.plan.h, _ptr(flows), _ptr(x_dev), _ptr(glob),
                                         _ptr(self.worst), _ptr(self.pairs), n,
                                         *[_ptr(a) for a in arrs], _ptr(feat), D._stream()),
             "dcflow_action_features")
        return feat

    def improvement_labels(self, max_load, snap):
        """Training labels of exact-screen maxima (device): the log gain over
        the snapshot's unchanged grid, clipped at 0."""
        import torch
        ml = torch.as_tensor(np.ascontiguousarray(max_load, dtype=np.float64)).cuda()
        sn = torch.as_tensor(np.ascontiguousarray(snap, dtype=np.int32)).cuda()
        out = torch.empty(ml.shape[0], dtype=torch.float32, device="cuda")
        _chk(_lib.dcflow_improvement_labels(_ptr(ml), _ptr(sn), _ptr(self.glob), ml.shape[0],
                                            _ptr(out), D._stream()), "dcflow_improvement_labels")
        return out

    def set_standardization(self, feat, labels):
        """Standardisation constants from the training set (on the device)."""
        s = D._stream()
        n = feat.shape[0]
        _chk(_lib.dcflow_column_stats(_ptr(feat), n, 96, _ptr(self.mu), _ptr(self.isd), s),
             "dcflow_column_stats")
        _chk(_lib.dcflow_column_stats(_ptr(labels), n, 1, _ptr(self.t_mu), _ptr(self.t_isd), s),
             "dcflow_column_stats")

    def standardize(self, feat, labels=None):
        s = D._stream()
        _chk(_lib.dcflow_standardize(_ptr(feat), feat.shape[0], 96, _ptr(self.mu), _ptr(self.isd),
                                     s), "dcflow_standardize")
        if labels is not None:
            _chk(_lib.dcflow_standardize(_ptr(labels), labels.shape[0], 1, _ptr(self.t_mu),
                                         _ptr(self.t_isd), s), "dcflow_standardize")

    # ------------------------------------------------------------ training
    def train(self, feat, labels, epochs=8, batch=1024, lr=1e-3):
        """Minibatch Adam on the mean squared error; feat/labels already
        standardised and in a shuffled order (contiguous minibatches)."""
        import torch
        n = feat.shape[0]
        ws = torch.empty(_lib.dcflow_mlp_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
        s = D._stream()
        losses = []
        for _ in range(epochs):
            for b0 in range(0, n - batch + 1, batch):
                xb = feat[b0:b0 + batch]
                tb = labels[b0:b0 + batch]
                _chk(_lib.dcflow_mlp_grad(_ptr(self.params), _ptr(xb), _ptr(tb), batch,
                                          _ptr(self.grad), _ptr(self.loss), _ptr(ws),
                                          ws.numel(), s), "dcflow_mlp_grad")
                self.step += 1
                _chk(_lib.dcflow_mlp_adam(_ptr(self.params), _ptr(self.grad), _ptr(self.m),
                                          _ptr(self.v), self.step, float(lr), s), "dcflow_mlp_adam")
            losses.append(float(self.loss.item()))
        return losses

    # ------------------------------------------------------------ inference
    def pack(self):
        _chk(_lib.dcflow_mlp_pack_bf16(_ptr(self.params), _ptr(self.bf16), D._stream()),
             "dcflow_mlp_pack_bf16")

    def infer(self, feat):
        import torch
        y = torch.empty(feat.shape[0], dtype=torch.float32, device="cuda")
        _chk(_lib.dcflow_mlp_infer(_ptr(self.params), _ptr(self.bf16), _ptr(feat), feat.shape[0],
                                   _ptr(y), D._stream()), "dcflow_mlp_infer")
        return y

    def forward_fp32(self, feat):
        import torch
        n = feat.shape[0]
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        ws = torch.empty(_lib.dcflow_mlp_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        _chk(_lib.dcflow_mlp_forward(_ptr(self.params), _ptr(feat), n, _ptr(y), _ptr(ws),
                                     ws.numel(), D._stream()), "dcflow_mlp_forward")
        return y


def topk_smallest(scores, k):
    import torch
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    _chk(_lib.dcflow_topk_smallest(_ptr(scores), scores.shape[0], k, _ptr(idx), D._stream()),
         "dcflow_topk_smallest")
    return idx
