"""Phase shifters that are contingencies, outaged, or on a branch that a split
moves to the new busbar (the end of Sec. II names the PSDF; the shift's direct
term is part of the flows the corrections and the LODF act on).  The 30-bus grid
with two shifters and two HVDC links, the shifters' branches among the
contingencies, candidates that touch the shifters in every way, four
control/load combinations shared by all candidates: GPU scores and N-0 flows
against the oracle (rebuild + dense LU with the control model on the post-change
network), element by element, in all three precisions."""
import numpy as np
import pytest

import gridgen as G
from oracle import dcflow_oracle as O

from _gpu_common import compare, gpu_available, oracle_rating, oracle_scores, run_gpu, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _workload():
    w0 = G.workload_tiny(0)
    g = w0.grid
    nb = np.flatnonzero(~O.bridges(g.n_bus, g.f, g.t))
    pst = [int(nb[0]), int(nb[4])]
    controls = dict(pst=pst, pst_scale=np.pi / 180.0, hvdc=[(3, 17), (8, 25)], hvdc_scale=0.25)
    rng = np.random.default_rng(11)
    ctrl = np.column_stack([rng.integers(-10, 11, size=(4, 2)),
                            rng.integers(0, 8, size=(4, 2))]).astype(np.float64)
    x = G.perturbed_injections(g, rng, (4,), 0.2)
    inj = np.concatenate([x, ctrl], axis=1)
    out = np.asarray(sorted(int(c) for c in nb[:14]), np.int32)
    assert set(pst) <= set(out.tolist())

    def moving(branch, bus, extra_bit):
        inc = list(O.incident_branches(g.f, g.t, bus))
        return (G.KIND_SPLIT, bus, (1 << inc.index(branch)) | (1 << extra_bit), 0.1)

    a = int(np.flatnonzero(g.degree() >= 3)[2])
    lists = [[], [(G.KIND_OUTAGE, pst[1], 0, 0.0)], [(G.KIND_OUTAGE, pst[0], 0, 0.0)],
             [moving(pst[1], int(g.t[pst[1]]), 0), (G.KIND_OUTAGE, int(out[6]), 0, 0.0)],
             [moving(pst[0], int(g.t[pst[0]]), 0)], [moving(pst[1], int(g.f[pst[1]]), 0)],
             [(G.KIND_SPLIT, a, 2, 0.4), (G.KIND_OUTAGE, pst[0], 0, 0.0)]]
    # keep the candidates whose network stays connected
    keep = [els for els in lists
            if O.candidate_flows(g.n_bus, g.f, g.t, g.b, g.slack, els, x[:1], out)["connected"]]
    assert len(keep) >= 5
    return G.Workload("tiny-pst", g, np.arange(g.n_branch, dtype=np.int32), out,
                      G.Candidates.from_lists(keep), inj, True, controls=controls)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_phase_shifter_cases(prec):
    w = _workload()
    r = oracle_rating(w)
    idx = list(range(w.cands.n_cand))
    say(f"pst {prec}: {len(idx)} candidates, shifters {w.controls['pst']}")
    gpu = run_gpu(w, prec, rating=r)
    res = oracle_scores(w, idx, r)
    err = compare(w, gpu, res, r, idx, prec)
    say(f"pst {prec}: largest |d max_load| {err:.2e}")
