"""Error guard of the reduced-precision scan: contingency columns whose FP32
error bound exceeds the tolerance are computed in FP64 instead.  With a
tolerance that flags every scored column, the FP32 and BF16X6 paths must agree
with the plain FP64 path to FP32 rounding of the stored flows (every LODF'
entry is then FP64), in the scores, the per-variant maxima and both worst-case
lists; with the guard off no candidate carries the guarded status bit."""
import numpy as np
import pytest

import gridgen as G

from _gpu_common import gpu_available, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ST_GUARDED = 0x8
NOT_GUARDED = np.uint32(0xFFFFFFFF ^ ST_GUARDED)


@pytest.fixture(scope="module")
def medium():
    import torch
    from paper_2501_17529_amd import dcflow as D
    w = G.workload_medium(0, n_cand=384, n_var=4)
    rng = np.random.default_rng(5)
    w.gens = G.generator_outages(w.grid, rng, 12)
    plan = D.Plan.from_workload(w)
    x = torch.from_numpy(np.ascontiguousarray(w.inj)).cuda()

    def run(prec, guard_tol=0.0, top_k=8, per_case=3):
        bt = D.Batch(plan, w.cands, 4)
        bt.set_tuning(guard_tol=guard_tol)
        bt.eval_topologies()
        flows = bt.eval_injections(x, 4, False, prec)
        out = bt.n1_score(flows, 4, prec)
        worst = bt.n1_worst(flows, 4, prec, out, top_k)
        pc = bt.n1_worst_per_case(flows, 4, prec, out, per_case, top_k)
        torch.cuda.synchronize()
        return dict(sc=D.Batch.scores_to_numpy(out, bt.n_cand).copy(),
                    vm=bt.variant_max(4).cpu().numpy().copy(),
                    worst=D.Batch.cases_to_numpy(worst, bt.n_cand, top_k).copy(),
                    pc=D.Batch.cases_to_numpy(pc, bt.n_cand, top_k).copy())
    return w, run, run("fp64")


def _lists_close(a, b, tol, ctx):
    """Two worst-case lists of one candidate: ranked loads within tol; the same
    cases where the loads are apart by more than 2 tol from their neighbours."""
    np.testing.assert_allclose(a["load"], b["load"], atol=tol, rtol=0, err_msg=ctx)
    for j in range(len(a)):
        lo = b["load"][j]
        near = np.abs(b["load"] - lo) <= 2 * tol
        if near.sum() == 1:
            assert (a["branch"][j], a["outage"][j]) == (b["branch"][j], b["outage"][j]), (ctx, j)


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_guard_everywhere_matches_fp64(medium, prec):
    w, run, ref = medium
    got = run(prec, guard_tol=1e-30)
    sc, rs = got["sc"], ref["sc"]
    scored = (rs["status"] & 1) == 0
    # every connected candidate has scored columns, so every one is guarded
    assert np.all((sc["status"][scored] & ST_GUARDED) != 0)
    np.testing.assert_array_equal(sc["status"] & NOT_GUARDED, rs["status"])
    # what remains is the FP32 rounding of the stored flows (a few units of 2^-24
    # relative to the largest load) and of the GEMM's load perturbations
    tol = 1e-7 + 4 * 2.0 ** -24 * float(rs["max_load"][scored].max())
    err = np.abs(got["vm"][scored] - ref["vm"][scored]).max()
    say(f"guard everywhere {prec}: max |d variant max| vs FP64 = {err:.3e} (bound {tol:.2e})")
    assert err <= tol
    np.testing.assert_allclose(sc["max_load"][scored], rs["max_load"][scored], atol=tol, rtol=0)
    np.testing.assert_allclose(sc["overload_sum"][scored], rs["overload_sum"][scored],
                               atol=1e-4, rtol=1e-5)
    for i in np.flatnonzero(scored)[::7]:
        _lists_close(got["worst"][i], ref["worst"][i], tol, f"{prec} worst cand {i}")
        _lists_close(got["pc"][i], ref["pc"][i], tol, f"{prec} per-case cand {i}")
        # the global list starts with the score's maximum and worst case
        assert got["worst"][i]["load"][0] == sc["max_load"][i]
        assert (got["worst"][i]["branch"][0], got["worst"][i]["outage"][0]) == (
            sc["worst_branch"][i], sc["worst_outage"][i])


def test_guard_default_and_off(medium):
    w, run, ref = medium
    on = run("fp32")
    off = run("fp32", guard_tol=-1.0)
    scored = (ref["sc"]["status"] & 1) == 0
    assert not np.any(off["sc"]["status"] & ST_GUARDED)
    for name, r in (("default", on), ("off", off)):
        err = np.abs(r["vm"][scored] - ref["vm"][scored]).max()
        say(f"guard {name}: max |d variant max| vs FP64 = {err:.3e}, "
            f"{int(((r['sc']['status'] & ST_GUARDED) != 0).sum())} guarded candidates")
        assert err <= 1e-4
        np.testing.assert_array_equal(r["sc"]["status"] & NOT_GUARDED, ref["sc"]["status"])
