"""GPU tests of the orchestration layer: launch shapes (variant groups, row
chunks, row bands, persistent queue) give the same scores as the default launch, a
captured HIP graph of the whole step replays to the eager result (several
replays, with eager work and new injections in between), and the autotuner
records and re-applies its choice."""
import json

import numpy as np
import pytest

import gridgen as G
from oracle import dcflow_oracle as O

from _gpu_common import gpu_available, oracle_rating, oracle_scores, compare, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

KEYS = ("max_load", "best_variant", "worst_branch", "worst_outage", "status")


def _workload(seed=21, n_cand=40, n_var=6):
    """Uneven ranks 1..8 on a small grid, plus an islanded candidate (the new
    busbar keeps no branch after an outage) and the unchanged grid."""
    rng = np.random.default_rng(seed)
    g = G.make_grid(120, 190, seed)
    lists = []
    for i in range(n_cand):
        k = int(rng.integers(1, 9))
        ns = min(int(rng.binomial(k, 0.5)), 6)
        lists.append(G.sample_candidate(g, rng, ns, k - ns))
    a = int(np.flatnonzero(g.degree() >= 3)[0])
    inc = g.incident(a)
    lists.append([(G.KIND_SPLIT, a, 0b010, 0.0), (G.KIND_OUTAGE, int(inc[1]), 0, 0.0)])
    lists.append([])
    cands = G.Candidates.from_lists(lists)
    mon = np.sort(rng.choice(190, size=130, replace=False)).astype(np.int32)
    out = np.sort(rng.choice(190, size=70, replace=False)).astype(np.int32)
    inj = G.perturbed_injections(g, rng, (len(lists), n_var), 0.2)
    return G.Workload("orch", g, mon, out, cands, inj, False)


def _scores(D, bt, flows, nv, prec, out=None):
    import torch
    out = bt.n1_score(flows, nv, prec, out=out)
    torch.cuda.synchronize()
    return D.Batch.scores_to_numpy(out, bt.n_cand)


def _same(a, b, ctx):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{ctx}: {k}")
    np.testing.assert_allclose(a["overload_sum"], b["overload_sum"], rtol=1e-9, atol=1e-12,
                               err_msg=f"{ctx}: overload_sum")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_launch_shapes_agree(prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    from paper_2501_17529_amd import autotune
    w = _workload()
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    bt.eval_topologies()
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows = bt.eval_injections(x, nv, False, prec)
    ref = _scores(D, bt, flows, nv, prec)
    say(f"launch shapes {prec}: {len(autotune.candidates(bt, nv, prec))}")
    # row bands: the scan split into (candidate, band) work items whose partials
    # are combined afterwards (the autotuner offers them only for large seeds)
    banded = [dict(scan_vc=0, scan_rchunk=rc, persistent=pe, scan_band=b)
              for b in (64, 128) for rc in (0, 64) for pe in (0, 1)]
    for cfg in autotune.candidates(bt, nv, prec) + banded:
        bt.set_tuning(**cfg)
        got = bt.get_tuning()
        assert {k: got[k] for k in cfg} == cfg and got["step_chunks"] == 0
        _same(_scores(D, bt, flows, nv, prec), ref, f"{prec} {cfg}")
    # the default launch itself against the oracle
    r = oracle_rating(w)
    idx = [0, 7, 19, len(w.cands.off) - 3, len(w.cands.off) - 2]
    gpu = dict(scores=ref, vmax=bt.variant_max(nv).cpu().numpy(),
               flows=bt.flows_view(flows, nv).double().cpu().numpy())
    compare(w, gpu, oracle_scores(w, idx, r), r, idx, prec)
    assert ref[len(w.cands.off) - 3]["status"] & O.ST_DISCONNECTED


def test_tuning_rejects_bad_values():
    import ctypes
    from paper_2501_17529_amd import dcflow as D
    w = _workload(n_cand=3, n_var=2)
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, 2)
    for bad in ((0, 65, 0, 0), (-1, 0, 0, 0), (0, 0, -1, 0), (0, 0, 0, 96), (0, 0, 0, -64)):
        t = D.Tuning(*bad)
        assert D._lib.dcflow_batch_set_tuning(bt.h, ctypes.byref(t)) == -1
    assert D._lib.dcflow_graph_launch(bt.h, None) == -1   # nothing captured


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_replay_matches_eager(persistent):
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = _workload(seed=22)
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    bt.set_tuning(persistent=persistent)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows, _ = bt.flow_buffer(nv, "fp32")
    out = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bt.eval_topologies()
        bt.eval_injections(x, nv, False, "fp32", flows=flows)
        eager = _scores(D, bt, flows, nv, "fp32", out=out)
        out.zero_()
        bt.capture(x, nv, False, "fp32", flows, out, s)
        torch.cuda.synchronize()
        for rep in range(3):
            out.zero_()
            bt.replay(s)
            torch.cuda.synchronize()
            _same(D.Batch.scores_to_numpy(out, bt.n_cand), eager, f"replay {rep}")
            # eager work on the same buffers between replays
            other = torch.empty_like(out)
            bt.n1_score(flows, nv, "fp32", out=other)
            torch.cuda.synchronize()
        # new injections in the captured buffer: the replay sees them
        rng = np.random.default_rng(23)
        x.copy_(torch.from_numpy(G.perturbed_injections(w.grid, rng, w.inj.shape[:2], 0.3)))
        bt.eval_topologies()
        bt.eval_injections(x, nv, False, "fp32", flows=flows)
        eager2 = _scores(D, bt, flows, nv, "fp32")
        out.zero_()
        bt.replay(s)
        torch.cuda.synchronize()
        _same(D.Batch.scores_to_numpy(out, bt.n_cand), eager2, "replay after new injections")
    say(f"graph replay (persistent={persistent}) matches eager")


def test_autotune_records_and_reuses(tmp_path, monkeypatch):
    import torch
    from paper_2501_17529_amd import dcflow as D
    from paper_2501_17529_amd import autotune
    monkeypatch.setenv("DCFLOW_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    w = _workload(seed=24, n_cand=30, n_var=16)
    nv = 16
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    bt.eval_topologies()
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows = bt.eval_injections(x, nv, False, "fp32")
    ref = _scores(D, bt, flows, nv, "fp32")
    cfg, times = autotune.tune_scan(bt, flows, nv, "fp32")
    got = bt.get_tuning()
    assert {k: got[k] for k in cfg} == cfg
    assert all(v is not None for v in times.values()), times
    data = json.load(open(tmp_path / "tune.json"))
    key = autotune.shape_key(bt, nv, "fp32")
    assert data[key]["config"] == cfg
    bt.set_tuning()
    cfg2, _ = autotune.tune_scan(bt, flows, nv, "fp32")   # cache hit
    got = bt.get_tuning()
    assert cfg2 == cfg and {k: got[k] for k in cfg} == cfg
    _same(_scores(D, bt, flows, nv, "fp32"), ref, "tuned")
    say(f"autotune picked {cfg}")


@pytest.mark.parametrize("chunks", [2, 3, 5])
def test_chunked_step_matches_separate_calls(chunks):
    """dcflow_step in candidate chunks (injections of one chunk beside the scan of
    the previous one on the batch's second stream) gives the same flows and
    scores, bit for bit, as the three calls over the whole batch; also captured
    into a graph and replayed."""
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = _workload(seed=24)
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    bt.eval_topologies()
    ref_flows = bt.eval_injections(x, nv, False, "fp32").clone()
    ref = _scores(D, bt, ref_flows, nv, "fp32")
    bt.set_tuning(step_chunks=chunks)
    assert bt.get_tuning()["step_chunks"] == chunks
    flows, _ = bt.flow_buffer(nv, "fp32")
    out = torch.empty(bt.n_cand * D.SCORE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        flows.zero_()
        bt.step(x, nv, False, "fp32", flows, out, s)
        torch.cuda.synchronize()
        assert torch.equal(flows, ref_flows)
        _same(D.Batch.scores_to_numpy(out, bt.n_cand), ref, f"step chunks={chunks}")
        bt.capture(x, nv, False, "fp32", flows, out, s)
        for rep in range(3):
            out.zero_()
            flows.zero_()
            torch.cuda.synchronize()
            bt.replay(s)
            torch.cuda.synchronize()
            assert torch.equal(flows, ref_flows), rep
            _same(D.Batch.scores_to_numpy(out, bt.n_cand), ref, f"replay {rep} chunks={chunks}")
    say(f"chunked step ({chunks} chunks) matches the separate calls")
