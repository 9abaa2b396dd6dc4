"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  FP64 mode: max |dp|/rating <= 1e-6; FP32 mode: <= 1e-4."""
import numpy as np
import pytest

import gridgen as G
from oracle import dcflow_oracle as O

from _gpu_common import TOL, compare, gpu_available, oracle_rating, oracle_scores, run_gpu, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _mixed_workload(seed, n=90, m=140, n_cand=48, n_var=5, kmax=8):
    """Small grid, uneven ranks up to kmax, monitored and contingency sets of
    ragged sizes that differ (so E_r = E_m u O is a proper union), bridges among
    the contingencies, a few injections moved onto new busbars."""
    rng = np.random.default_rng(seed)
    g = G.make_grid(n, m, seed)
    lists = []
    for i in range(n_cand):
        k = int(rng.integers(1, kmax + 1))
        ns = int(rng.binomial(k, 0.5))
        ns = min(ns, 6)
        els = G.sample_candidate(g, rng, ns, k - ns)
        if i % 5 == 0:
            els = [(kd, d, mk, float(rng.normal()) if kd == G.KIND_SPLIT else 0.0)
                   for (kd, d, mk, _) in els]
        lists.append(els)
    lists.append([])                                      # the unchanged grid
    cands = G.Candidates.from_lists(lists)
    mon = np.sort(rng.choice(m, size=77, replace=False)).astype(np.int32)
    out = np.sort(rng.choice(m, size=45, replace=False)).astype(np.int32)
    inj = G.perturbed_injections(g, rng, (len(lists), n_var), 0.2)
    return G.Workload("mixed", g, mon, out, cands, inj, False)


def test_ptdf_build_matches_oracle():
    for w in (G.workload_tiny(0), _mixed_workload(1, n_cand=2)):
        g = w.grid
        say(f"ptdf build n={g.n_bus} m={g.n_branch}")
        from paper_2501_17529_amd import dcflow as D
        plan = D.Plan.from_workload(w)
        h = plan.ptdf().cpu().numpy()
        ho = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
        assert np.abs(h - ho).max() < 1e-11
        fb = plan.f_base().cpu().numpy()
        np.testing.assert_allclose(fb, O.dc_flows(g.n_bus, g.f, g.t, g.b, g.slack, g.p)[0], atol=1e-11)
        np.testing.assert_allclose(plan.rating().cpu().numpy(), oracle_rating(w), rtol=1e-12)
        hdo = plan.hdo().cpu().numpy()
        np.testing.assert_allclose(hdo, ho[:, g.f[w.out]] - ho[:, g.t[w.out]], atol=1e-11)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_tiny_workload_all_candidates(prec):
    w = G.workload_tiny(0)
    r = oracle_rating(w)
    say(f"tiny workload {prec}")
    gpu = run_gpu(w, prec)
    idx = list(range(w.cands.n_cand))
    res = oracle_scores(w, idx, r)
    err = compare(w, gpu, res, r, idx, prec)
    say(f"tiny {prec}: worst |d max_load| = {err:.3e}")
    # islanding contingencies exist in this workload (bridges are in the N-1 set)
    assert sum(int(x["n_island"]) for x in res) > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
@pytest.mark.parametrize("seed", [0, 1])
def test_uneven_rank_mixed_elements(prec, seed):
    w = _mixed_workload(seed)
    r = oracle_rating(w)
    say(f"mixed workload seed={seed} {prec} k={np.diff(w.cands.off).tolist()}")
    gpu = run_gpu(w, prec)
    idx = list(range(w.cands.n_cand))
    res = oracle_scores(w, idx, r)
    compare(w, gpu, res, r, idx, prec)


def test_shared_and_per_candidate_injections_agree():
    w = _mixed_workload(3, n_cand=20, n_var=3)
    say("shared vs per-candidate injections")
    shared_inj = w.inj[0]
    a = run_gpu(w, "fp64", inj=shared_inj, inj_shared=True)
    b = run_gpu(w, "fp64", inj=np.broadcast_to(shared_inj, w.inj.shape).copy(), inj_shared=False)
    np.testing.assert_allclose(a["vmax"], b["vmax"], atol=1e-12)
    np.testing.assert_allclose(a["flows"], b["flows"], atol=1e-12)


def test_edge_cases():
    """Split of the slack bus, injection moved with a split, outage of a moved
    branch, contingency that is a moved branch, contingency already removed,
    a candidate whose new busbar loses every branch (islanded), a bridge outage
    (islanded), the empty candidate."""
    w0 = G.workload_tiny(0)
    g = w0.grid
    inc_s = g.incident(g.slack)
    assert len(inc_s) >= 2
    lists = [[(G.KIND_SPLIT, g.slack, 2, 0.0)],
             [(G.KIND_SPLIT, g.slack, 2, 0.7)]]
    a = int(np.flatnonzero(g.degree() >= 3)[1])
    inc = g.incident(a)
    lists.append([(G.KIND_SPLIT, a, 0b110, 0.3), (G.KIND_OUTAGE, int(inc[1]), 0, 0.0)])
    lists.append([(G.KIND_SPLIT, a, 0b010, 0.0), (G.KIND_OUTAGE, int(inc[1]), 0, 0.0)])  # B isolated
    bridges = np.flatnonzero(O.bridges(g.n_bus, g.f, g.t))
    lists.append([(G.KIND_OUTAGE, int(bridges[0]), 0, 0.0)])
    lists.append([])
    nb = np.flatnonzero(~O.bridges(g.n_bus, g.f, g.t))
    lists.append([(G.KIND_OUTAGE, int(nb[0]), 0, 0.0), (G.KIND_OUTAGE, int(nb[3]), 0, 0.0)])
    cands = G.Candidates.from_lists(lists)
    rng = np.random.default_rng(5)
    inj = G.perturbed_injections(g, rng, (len(lists), 4), 0.3)
    w = G.Workload("edge", g, w0.mon, w0.out, cands, inj, False)
    r = oracle_rating(w)
    for prec in ("fp64", "fp32", "bf16x6"):
        say(f"edge cases {prec}")
        gpu = run_gpu(w, prec)
        res = oracle_scores(w, range(len(lists)), r)
        assert res[3]["status"] & O.ST_DISCONNECTED and res[4]["status"] & O.ST_DISCONNECTED
        compare(w, gpu, res, r, list(range(len(lists))), prec)


def test_nonfinite_injection_flagged():
    w = _mixed_workload(4, n_cand=6, n_var=3)
    inj = w.inj.copy()
    inj[2, 1, 5] = np.nan
    say("nonfinite injection")
    gpu = run_gpu(w, "fp64", inj=inj)
    s = gpu["scores"]
    assert s[2]["status"] & 0x4
    assert s[2]["best_variant"] != 1
    assert np.isinf(gpu["vmax"][2, 1])
    assert all((s[i]["status"] & 0x4) == 0 for i in (0, 1, 3, 4))


def test_repeat_is_bitwise_identical():
    w = _mixed_workload(6, n_cand=30, n_var=4)
    say("determinism")
    a = run_gpu(w, "fp32")
    b = run_gpu(w, "fp32")
    assert np.array_equal(a["scores"].view(np.uint8), b["scores"].view(np.uint8))
    assert np.array_equal(a["vmax"], b["vmax"])


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x6"])
def test_medium_full_batch_sampled(prec):
    """1,000-bus grid, 4,096 candidates x 16 variants, 500 contingencies: the
    full batch runs on the GPU; 12 sampled candidates are checked against the
    oracle one by one, all others by invariants."""
    w = G.workload_medium(0)
    r = oracle_rating(w)
    say(f"medium full batch {prec}")
    gpu = run_gpu(w, prec)
    sc = gpu["scores"]
    assert np.all(np.isfinite(sc["max_load"]))
    assert np.all((sc["status"] & 0x7) == 0)
    assert np.all((sc["best_variant"] >= 0) & (sc["best_variant"] < 16))
    vm = gpu["vmax"]
    np.testing.assert_array_equal(sc["best_variant"], np.argmin(vm, axis=1))
    rng = np.random.default_rng(11)
    idx = sorted(rng.choice(w.cands.n_cand, size=12, replace=False).tolist())
    res = oracle_scores(w, idx, r)
    err = compare(w, gpu, res, r, idx, prec)
    say(f"medium {prec}: worst |d max_load| on the sample = {err:.3e}")


def test_bf16_flows_within_rounding_bound():
    """Plain BF16 mode: every N-0 flow within the bound that BF16 rounding of
    both GEMM operands allows, |dF| <= 2^-7 sum_k |H_lk x_k| (plus the FP32
    accumulation), element by element against the oracle's flows."""
    w = _mixed_workload(7, n_cand=12, n_var=3)
    say("bf16 flows bound")
    g = w.grid
    gpu = run_gpu(w, "bf16")
    from _gpu_common import kept_rows
    er = kept_rows(w.mon, w.out)
    h = O.ptdf(g.n_bus, g.f, g.t, g.b, g.slack)
    worst = 0.0
    for i in range(w.cands.n_cand):
        els = w.cands.elements(i)
        cf = O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, w.inj[i], w.out)
        if not cf["connected"]:
            continue
        p0 = cf["p0"][:, er]                       # [V, n_er]
        got = gpu["flows"][i][:, : len(er)]
        # the GEMM part is H_er x; the rank-k correction is FP64, so bound the GEMM error
        bound = 2.0 ** -7 * (np.abs(h[er]) @ np.abs(w.inj[i]).T).T + 1e-5
        err = np.abs(got - p0)
        worst = max(worst, float((err / bound).max()))
        assert (err <= bound).all(), (i, float((err / bound).max()))
    say(f"bf16: worst error / bound = {worst:.3f}")


@pytest.mark.parametrize("prec", ["bf16x6", "fp32"])
def test_bf16x6_gemm_in_column_blocks(monkeypatch, prec):
    """With the split buffer (BF16 parts, or x - p_base in FP32) capped below the
    batch's columns the GEMM runs in blocks of whole candidates: the flows are the
    same, bit for bit; and in FP32 they equal the FP64 path's within FP32 rounding."""
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = G.workload_medium(3, n_cand=40, n_var=4)
    plan = D.Plan.from_workload(w)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    got = []
    for cap in (None, "24"):   # 24 columns = 6 candidates of 4 variants per block
        if cap:
            monkeypatch.setenv("DCFLOW_SPLIT_COLS", cap)
        bt = D.Batch(plan, w.cands, 4)
        bt.eval_topologies()
        fl = bt.eval_injections(x, 4, False, prec)
        torch.cuda.synchronize()
        got.append(fl.clone())
    assert torch.equal(got[0], got[1])
    if prec == "fp32":
        monkeypatch.delenv("DCFLOW_SPLIT_COLS", raising=False)
        bt = D.Batch(plan, w.cands, 4)
        bt.eval_topologies()
        f64 = bt.eval_injections(x, 4, False, "fp64").double()
        torch.cuda.synchronize()
        f32 = got[0].double()
        scale = f64.abs().max().item()
        assert (f32 - f64).abs().max().item() <= 1e-4 * scale + 1e-9
