"""agg_i from the winner pass's column-maximum record (tuning worst_record, on by
default): the n1_score winner pass keeps each candidate's column maxima of the
winning variant (Sec. III-A agg_i, metric-first recompute of Sec. IV-B), and
n1_worst / n1_worst_per_case read them instead of sweeping the winner's tiles
again.  The lists must be bit for bit those of the sweep (worst_record < 0): with
one and several scan bands, the FP32 error guard, score records naming another
variant, a chunked step and graph replays; and they must still match the
oracle."""
import numpy as np
import pytest

import gridgen as G

from _gpu_common import compare_worst, gpu_available, oracle_rating, oracle_scores, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _mixed(seed=41, n_cand=40, n_var=6):
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
    mon = np.sort(rng.choice(190, size=150, replace=False)).astype(np.int32)
    out = np.sort(rng.choice(190, size=90, replace=False)).astype(np.int32)
    inj = G.perturbed_injections(g, rng, (len(lists), n_var), 0.2)
    return G.Workload("worst-record", g, mon, out, cands, inj, False)


def _setup(w, prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    nv = w.inj.shape[1]
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, nv)
    bt.eval_topologies()
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    flows = bt.eval_injections(x, nv, w.inj_shared, prec)
    return D, bt, x, flows, nv


def _lists(D, bt, flows, nv, prec, sc_dev, top_k=16, per_case=3):
    import torch
    a = bt.n1_worst(flows, nv, prec, sc_dev, top_k)
    b = bt.n1_worst_per_case(flows, nv, prec, sc_dev, per_case, top_k)
    torch.cuda.synchronize()
    return a.cpu().numpy().copy(), b.cpu().numpy().copy()


def _same(ref, got, what):
    for r, g, name in zip(ref, got, ("global", "per-case")):
        assert np.array_equal(r, g), f"{what}: {name} lists differ from the sweep's"


@pytest.mark.parametrize("prec,tuning", [("fp64", {}), ("fp32", {}), ("bf16x6", {}),
                                         ("fp64", {"scan_band": 64}),
                                         ("fp32", {"scan_band": 64, "persistent": 1}),
                                         ("fp32", {"guard_tol": 1e-9})])
def test_record_gives_the_sweeps_lists(prec, tuning):
    w = _mixed()
    D, bt, x, flows, nv = _setup(w, prec)
    bt.set_tuning(**dict(tuning, worst_record=-1))
    sc_dev = bt.n1_score(flows, nv, prec)
    ref = _lists(D, bt, flows, nv, prec, sc_dev)
    sc_ref = sc_dev.cpu().numpy().copy()
    bt.set_tuning(**dict(tuning, worst_record=1))
    bt.n1_score(flows, nv, prec, out=sc_dev)
    got = _lists(D, bt, flows, nv, prec, sc_dev)
    assert np.array_equal(sc_dev.cpu().numpy(), sc_ref), "the record changed the scores"
    _same(ref, got, f"{prec} {tuning}")
    # and against the oracle (global top 16)
    r = oracle_rating(w)
    idx = [0, 7, len(w.cands.off) - 3, len(w.cands.off) - 2]
    sc = D.Batch.scores_to_numpy(sc_dev, bt.n_cand)
    cases = got[0][: bt.n_cand * 16 * D.CASE_DTYPE.itemsize].view(D.CASE_DTYPE).reshape(bt.n_cand, 16)
    for i, o in zip(idx, oracle_scores(w, idx, r)):
        compare_worst(w, cases[i], sc[i], o, 16, prec, f"record {prec} cand {i}")
    say(f"worst record {prec} {tuning}: lists equal to the sweep's")


def test_record_other_variant_falls_back():
    """Score records edited to name another variant (same array): those candidates
    are swept, the others read the record; the lists equal the sweep's."""
    import torch
    w = _mixed(seed=42)
    D, bt, x, flows, nv = _setup(w, "fp64")
    n = bt.n_cand
    words = D.SCORE_DTYPE.itemsize // 4

    def edit(sc_dev):
        iv = sc_dev.view(torch.int32).view(n, words)
        col = D.SCORE_DTYPE.fields["best_variant"][1] // 4
        sel = torch.zeros(n, dtype=torch.bool, device="cuda")
        sel[::3] = True
        iv[:, col] = torch.where(sel & (iv[:, col] >= 0), (iv[:, col] + 1) % nv, iv[:, col])

    bt.set_tuning(worst_record=-1)
    sc_dev = bt.n1_score(flows, nv, "fp64")
    edit(sc_dev)
    ref = _lists(D, bt, flows, nv, "fp64", sc_dev)
    bt.set_tuning(worst_record=1)
    bt.n1_score(flows, nv, "fp64", out=sc_dev)
    edit(sc_dev)
    got = _lists(D, bt, flows, nv, "fp64", sc_dev)
    _same(ref, got, "edited winners")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_record_chunked_step_and_replay(prec):
    """The record written by a chunked step, and by replays of a captured step."""
    import torch
    w = _mixed(seed=43)
    D, bt, x, flows, nv = _setup(w, prec)
    bt.set_tuning(worst_record=-1)
    sc_dev = bt.n1_score(flows, nv, prec)
    ref = _lists(D, bt, flows, nv, prec, sc_dev)
    bt.set_tuning(worst_record=1, step_chunks=3)
    bt.step(x, nv, False, prec, flows, sc_dev)
    _same(ref, _lists(D, bt, flows, nv, prec, sc_dev), f"{prec} chunked step")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bt.capture(x, nv, False, prec, flows, sc_dev, stream)
        for rep in range(3):
            bt.replay(stream)
            stream.synchronize()
            # an eager evaluation between the replays: the replay restores the record
            bt.eval_topologies()
            bt.eval_injections(x, nv, False, prec, flows=flows)
            torch.cuda.synchronize()
            bt.replay(stream)
            got = _lists(D, bt, flows, nv, prec, sc_dev)
            _same(ref, got, f"{prec} replay {rep}")


def test_record_medium_batch():
    """The bench's medium grid (one scan band in both precisions)."""
    w = G.workload_medium(0, n_cand=384)
    for prec in ("fp64", "fp32"):
        D, bt, x, flows, nv = _setup(w, prec)
        bt.set_tuning(worst_record=-1)
        sc_dev = bt.n1_score(flows, nv, prec)
        ref = _lists(D, bt, flows, nv, prec, sc_dev)
        bt.set_tuning()  # the default keeps the record
        bt.n1_score(flows, nv, prec, out=sc_dev)
        _same(ref, _lists(D, bt, flows, nv, prec, sc_dev), f"medium {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_record_is_read(prec):
    """White-box: with the record's flows pointer and score array, the worst-case
    calls read the record and do not sweep again.  The flows are zeroed in place
    after the score call (outside the calls' contract): a sweep would fill the lists
    with loads of 0, while the record's thresholds (from the real flows) admit no
    hot-column entry (the two-level list keeps only its N-0 case, 3 entries)."""
    import torch
    w = _mixed(seed=44)
    D, bt, x, flows, nv = _setup(w, prec)
    bt.set_tuning(worst_record=1)
    sc_dev = bt.n1_score(flows, nv, prec)
    torch.cuda.synchronize()
    flows.zero_()
    a, b = _lists(D, bt, flows, nv, prec, sc_dev)
    n = bt.n_cand
    sc = D.Batch.scores_to_numpy(sc_dev, n)
    # scored candidates without guarded columns (those are listed from the flows)
    live = (sc["status"] & 13) == 0
    assert live.sum() > 10
    for raw, name, first in ((a, "global", 0), (b, "per-case", 3)):
        cases = raw[: n * 16 * D.CASE_DTYPE.itemsize].view(D.CASE_DTYPE).reshape(n, 16)
        # the record's tau is positive for these candidates: no zero load of a hot
        # column passes it
        assert np.all(cases["load"][live][:, first:] == -1.0), \
            f"{prec} {name}: the record was not read"


def test_record_wide_contingency_set():
    """More than 1,024 contingency columns (ld_o 1,152) on one band of 384 monitored
    rows: k_rec_select does not take them, k_scan_colmax reads the record into LDS.
    The lists equal the sweep's, and the oracle's for sampled candidates."""
    rng = np.random.default_rng(45)
    g = G.make_grid(700, 1300, 45)
    lists = []
    for i in range(12):
        k = int(rng.integers(1, 6))
        ns = min(int(rng.binomial(k, 0.5)), 4)
        lists.append(G.sample_candidate(g, rng, ns, k - ns))
    cands = G.Candidates.from_lists(lists)
    mon = np.sort(rng.choice(1300, size=380, replace=False)).astype(np.int32)
    out = np.sort(rng.choice(1300, size=1100, replace=False)).astype(np.int32)
    inj = G.perturbed_injections(g, rng, (len(lists), 3), 0.2)
    w = G.Workload("worst-record-wide", g, mon, out, cands, inj, False)
    for prec in ("fp64", "fp32"):
        D, bt, x, flows, nv = _setup(w, prec)
        assert bt.plan.view.ld_o > 1024
        bt.set_tuning(worst_record=-1)
        sc_dev = bt.n1_score(flows, nv, prec)
        ref = _lists(D, bt, flows, nv, prec, sc_dev)
        bt.set_tuning(worst_record=1)
        bt.n1_score(flows, nv, prec, out=sc_dev)
        got = _lists(D, bt, flows, nv, prec, sc_dev)
        _same(ref, got, f"wide {prec}")
    r = oracle_rating(w)
    idx = [0, 5]
    sc = D.Batch.scores_to_numpy(sc_dev, bt.n_cand)
    cases = got[0][: bt.n_cand * 16 * D.CASE_DTYPE.itemsize].view(D.CASE_DTYPE).reshape(bt.n_cand, 16)
    for i, o in zip(idx, oracle_scores(w, idx, r)):
        compare_worst(w, cases[i], sc[i], o, 16, "fp32", f"wide cand {i}")
