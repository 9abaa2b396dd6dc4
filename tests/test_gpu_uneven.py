"""Uneven-rank configuration at its full size on one GPU: the 10,000-bus /
15,500-branch grid, 65,536 candidates of rank uniform in 1..8, every branch
monitored, 2,000 contingencies, one injection per candidate.

* FP64 path: 256 sampled candidates against the oracle's stored results
  (tests/golden/uneven_oracle.json, written by make_uneven_oracle.py, which
  rebuilds and factorises each candidate grid; the stored input fingerprint
  must match the generator's output here) at 1e-6 of rating; invariants over
  the whole batch.
* FP32 and BF16X6 paths: every one of the 65,536 candidates within 1e-4 of
  rating of the FP64 path (and the sample within 1e-4 of the oracle), in the
  persistent launch and in the banded launch the benchmark times (bit for bit
  the same scores); the winners' worst-case lists against the oracle."""
import importlib.util
import json
import os

import numpy as np
import pytest

import gridgen as G

from _gpu_common import gpu_available, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

HERE = os.path.dirname(os.path.abspath(__file__))
N_CAND = 65536
ST_GUARDED = 0x8
NOT_GUARDED = np.uint32(0xFFFFFFFF ^ ST_GUARDED)


def _golden_module():
    spec = importlib.util.spec_from_file_location(
        "make_uneven_oracle", os.path.join(HERE, "golden", "make_uneven_oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def uneven():
    import torch
    from paper_2501_17529_amd import dcflow as D
    say(f"uneven: generating the 10,000-bus grid and {N_CAND} candidates")
    w = G.workload_uneven(0, n_cand=N_CAND)
    gm = _golden_module()
    path = os.path.join(HERE, "golden", "uneven_oracle.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/uneven_oracle.json not written yet (make_uneven_oracle.py)")
    gold = json.load(open(path))
    idx = [c["index"] for c in gold["candidates"]]
    assert idx == gm.sample_indices()
    assert gold["fingerprint"] == gm.fingerprint(w, idx), "generator output changed"
    say("uneven: plan build")
    plan = D.Plan.from_workload(w)
    bt = D.Batch(plan, w.cands, 1)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()
    bt.set_tuning(persistent=1)
    bt.eval_topologies()
    say("uneven: FP64 path")
    fl = bt.eval_injections(x, 1, False, "fp64")
    out = bt.n1_score(fl, 1, "fp64")
    worst = bt.n1_worst(fl, 1, "fp64", out, 16)
    torch.cuda.synchronize()
    ref = D.Batch.scores_to_numpy(out, bt.n_cand).copy()
    ref_worst = D.Batch.cases_to_numpy(worst, bt.n_cand, 16)[idx].copy()
    del fl, out, worst
    torch.cuda.empty_cache()
    return dict(w=w, plan=plan, bt=bt, x=x, gold=gold["candidates"], idx=idx, ref=ref,
                ref_worst=ref_worst)


def _check_sample(sc, gold, tol, ctx):
    """Scores of the sampled candidates against the oracle's stored ones."""
    worst = 0.0
    for c in gold:
        i = c["index"]
        s = sc[i]
        assert (int(s["status"]) & 0x7) == c["status"], (ctx, i)
        assert (int(s["status"]) >> 8) == c["n_island"], (ctx, i, s["status"] >> 8, c["n_island"])
        err = abs(float(s["max_load"]) - c["max_load"][0])
        worst = max(worst, err)
        assert err <= tol, (ctx, i, s["max_load"], c["max_load"][0])
        assert abs(float(s["overload_sum"]) - c["overload_sum"]) <= tol * (
            1 + 10 * abs(c["overload_sum"])), (ctx, i, s["overload_sum"], c["overload_sum"])
        # the worst case: the stored list names every case within the tolerance of the maximum
        near = {(b, o) for v, b, o in c["worst16"] if v >= c["max_load"][0] - 2 * tol}
        if len(near) < 16:
            assert (int(s["worst_branch"]), int(s["worst_outage"])) in near, (ctx, i)
    return worst


def _check_worst(cases, gold, tol, ctx):
    """The winners' top-16 lists against the oracle's: ranked loads within tol."""
    for ci, c in enumerate(gold):
        want = np.array([v for v, _, _ in c["worst16"]])
        got = cases[ci]["load"][:len(want)]
        np.testing.assert_allclose(got, want, atol=tol, rtol=0, err_msg=f"{ctx} cand {c['index']}")


def test_uneven_fp64_against_oracle(uneven):
    u = uneven
    sc, w = u["ref"], u["w"]
    k = np.diff(w.cands.off)
    assert k.min() == 1 and k.max() == 8
    assert np.all((sc["status"] & 0x7) == 0)
    assert np.all(np.isfinite(sc["max_load"])) and np.all(sc["max_load"] > 0)
    assert np.all(np.isin(sc["worst_branch"], w.mon))
    assert np.all((sc["worst_outage"] == -1) | np.isin(sc["worst_outage"], w.out))
    err = _check_sample(sc, u["gold"], 1e-6, "fp64")
    _check_worst(u["ref_worst"], u["gold"], 1e-6, "fp64 worst")
    say(f"uneven fp64: 256 sampled candidates against the oracle, largest |d max_load| {err:.2e}")


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_uneven_mixed_whole_batch(uneven, prec):
    import torch
    from paper_2501_17529_amd import dcflow as D
    u = uneven
    bt, x, ref = u["bt"], u["x"], u["ref"]
    fl = bt.eval_injections(x, 1, False, prec)
    res = {}
    for name, tun in (("persistent", dict(persistent=1)), ("bands", dict(scan_band=512))):
        bt.set_tuning(**tun)
        out = bt.n1_score(fl, 1, prec)
        torch.cuda.synchronize()
        res[name] = (out, D.Batch.scores_to_numpy(out, bt.n_cand).copy())
    a, b = res["persistent"][1], res["bands"][1]
    for key in ("max_load", "worst_branch", "worst_outage", "status"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{prec} launch shapes: {key}")
    sc = a
    d = np.abs(sc["max_load"] - ref["max_load"])
    n_guard = int(((sc["status"] & ST_GUARDED) != 0).sum())
    say(f"uneven {prec}: all {N_CAND} candidates: max |d max_load| vs FP64 {d.max():.3e}, "
        f"median {np.median(d):.2e}, {int((d > 1e-4).sum())} over 1e-4, {n_guard} guarded")
    np.testing.assert_array_equal(sc["status"] & NOT_GUARDED, ref["status"])
    assert d.max() <= 1e-4, (int(np.argmax(d)), float(d.max()))
    err = _check_sample(sc, u["gold"], 1e-4, prec)
    cases = D.Batch.cases_to_numpy(bt.n1_worst(fl, 1, prec, res["persistent"][0], 16),
                                   bt.n_cand, 16)
    assert np.all(cases["load"][:, 0] == sc["max_load"])
    _check_worst(cases[u["idx"]], u["gold"], 1e-4, f"{prec} worst")
    say(f"uneven {prec}: sampled candidates against the oracle, largest |d max_load| {err:.2e}")
    bt.set_tuning(persistent=1)
    del fl
    torch.cuda.empty_cache()
