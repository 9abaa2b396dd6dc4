"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects malformed input before touching a GPU."""
import os
import re

import numpy as np
import pytest

import gridgen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def d():
    from paper_2501_17529_amd import dcflow
    return dcflow


def test_header_symbols_exported(d):
    hdr = open(os.path.join(ROOT, "include", "dcflow.h")).read()
    declared = set(re.findall(r"^(?:int|void|size_t|const char \*|const double \*)\s*(dcflow_[a-z0-9_]+)\(",
                              hdr, flags=re.M))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(d._lib, name), name
    assert declared == set(d.EXPORTED)


def _grid_args(d, w):
    g = w.grid
    return d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, g.slack)


def test_fig1_packing_counts(d):
    import json
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "fig1_packing.json")))
    w = G.workload_tiny(0)
    g = w.grid
    buses = [int(x) for x in np.flatnonzero(g.degree() >= 3)[:3]]
    split = {f"S{i + 1}": G.random_split(g, np.random.default_rng(i), b) for i, b in enumerate(buses)}
    lists = [[split[s] for s in c] for c in fx["candidates"]]
    packed, padded = d.validate_candidates(_grid_args(d, w), G.Candidates.from_lists(lists))
    assert packed == fx["naive_applications"]
    assert padded == fx["padded_simd_applications"]


def _bad(d, w, lists, expect_index):
    with pytest.raises(d.DcflowError) as ei:
        d.validate_candidates(_grid_args(d, w), G.Candidates.from_lists(lists))
    assert ei.value.code == -6
    assert ei.value.bad_index == expect_index


def test_candidate_validation_errors(d):
    w = G.workload_tiny(0)
    g = w.grid
    a = int(np.flatnonzero(g.degree() >= 3)[0])
    deg = len(g.incident(a))
    ok = (G.KIND_SPLIT, a, 2, 0.0)
    _bad(d, w, [[ok], [(G.KIND_OUTAGE, g.n_branch, 0, 0.0)]], 1)          # branch out of range
    _bad(d, w, [[(G.KIND_SPLIT, a, 0, 0.0)]], 0)                           # empty mask
    _bad(d, w, [[(G.KIND_SPLIT, a, (1 << deg) - 1, 0.0)]], 0)              # moves every branch
    _bad(d, w, [[(G.KIND_SPLIT, a, 1 << deg, 0.0)]], 0)                    # bit beyond degree
    _bad(d, w, [[ok, ok]], 1)                                              # two splits of one bus
    _bad(d, w, [[(G.KIND_OUTAGE, 3, 0, 0.0), (G.KIND_OUTAGE, 3, 0, 0.0)]], 1)  # duplicate outage
    _bad(d, w, [[(G.KIND_OUTAGE, i, 0, 0.0) for i in range(9)]], -1)       # rank 9 > 8
    _bad(d, w, [[(G.KIND_SPLIT, a, 2, float("nan"))]], 0)                  # non-finite p_new
    deg1 = np.flatnonzero(g.degree() == 1)
    if len(deg1):
        _bad(d, w, [[(G.KIND_SPLIT, int(deg1[0]), 1, 0.0)]], 0)            # degree-1 bus


def test_empty_and_rank_zero_candidates_are_valid(d):
    w = G.workload_tiny(0)
    assert d.validate_candidates(_grid_args(d, w), G.Candidates.from_lists([])) == (0, 0)
    assert d.validate_candidates(_grid_args(d, w), G.Candidates.from_lists([[], []])) == (0, 0)


def test_grid_validation_errors(d):
    w = G.workload_tiny(0)
    g = w.grid
    f = g.f.copy()
    f[0] = g.t[0]                      # self loop
    ga = d._GridArgs(g.n_bus, f, g.t, g.b, w.mon, w.out, g.p)
    with pytest.raises(d.DcflowError) as ei:
        d.validate_candidates(ga, w.cands)
    assert ei.value.code == -2
    b = g.b.copy()
    b[3] = -1.0                        # negative susceptance
    ga = d._GridArgs(g.n_bus, g.f, g.t, b, w.mon, w.out, g.p)
    with pytest.raises(d.DcflowError) as ei:
        d.validate_candidates(ga, w.cands)
    assert ei.value.code == -1
    ga = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, np.array([1, 1]), g.p)   # duplicate contingency
    with pytest.raises(d.DcflowError) as ei:
        d.validate_candidates(ga, w.cands)
    assert ei.value.code == -2
    for gens, code in [(([3, g.n_bus], [0.5, 0.5]), -2),      # generator bus out of range
                       (([3, -1], [0.5, 0.5]), -2),
                       (([3, 4], [0.5, np.inf]), -1),          # non-finite lost output
                       (([3, 4], [0.5, np.nan]), -1)]:
        ga = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, gens=gens)
        with pytest.raises(d.DcflowError) as ei:
            d.validate_candidates(ga, w.cands)
        assert ei.value.code == code, gens
    ga = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, gens=([3, 3, 0], [0.5, 0.1, 2.0]))
    d.validate_candidates(ga, w.cands)   # shared buses and the slack are allowed
    o = [int(c) for c in w.out[:20]]     # a contingency list without branch w.out[25]
    not_out = int(w.out[25])
    for multi, code in [([[o[0], not_out]], -2),                 # branch not a contingency
                        ([[o[0], o[1], o[2], o[3], o[4]]], -2),   # more than four branches
                        ([[o[0], o[0]]], -2),                     # repeated branch
                        ([[o[0]], []], -2)]:                      # empty case
        ga = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, o, g.p, multi=multi)
        with pytest.raises(d.DcflowError) as ei:
            d.validate_candidates(ga, w.cands)
        assert ei.value.code == code, multi
    ga = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, o, g.p, multi=[[o[0]], o[1:5]])
    d.validate_candidates(ga, w.cands)


def test_library_binds_to_torch_hip_runtime():
    """Importing the binding first must still leave one HIP runtime in the
    process, torch's: the library shares torch's device pointers and streams."""
    import subprocess
    import sys
    code = ("import paper_2501_17529_amd.dcflow, torch, os\n"
            "maps = open('/proc/self/maps').read()\n"
            "libs = {l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}\n"
            "tdir = os.path.dirname(torch.__file__)\n"
            "print(len(libs), all(p.startswith(tdir) for p in libs))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["1", "True"], r.stdout


def test_control_validation(d):
    """Phase shifters may be contingencies, outaged or moved by a split (the
    grid and the candidates are accepted); bad control definitions are rejected
    before any device work."""
    import ctypes
    w = G.workload_brute(0, n_topo=2, n_comb=4)
    g = w.grid
    ok = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, g.slack, controls=w.controls)
    nbytes = ctypes.c_size_t(0)
    assert d._lib.dcflow_plan_workspace_bytes(ctypes.byref(ok.desc), ctypes.byref(nbytes)) == 0
    pst = w.controls["pst"]
    extra = [int(l) for l in pst if int(l) not in set(w.out.tolist())]
    with_pst = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, np.sort(np.append(w.out, extra[0])), g.p,
                           g.slack, controls=w.controls)
    assert d._lib.dcflow_plan_workspace_bytes(ctypes.byref(with_pst.desc), ctypes.byref(nbytes)) == 0
    c2 = dict(w.controls, hvdc=[(3, 3)])
    same = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, g.slack, controls=c2)
    assert d._lib.dcflow_plan_workspace_bytes(ctypes.byref(same.desc), ctypes.byref(nbytes)) == -2
    c3 = dict(w.controls, pst=[pst[0], pst[0]] + list(pst[2:]))
    dup = d._GridArgs(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, g.slack, controls=c3)
    assert d._lib.dcflow_plan_workspace_bytes(ctypes.byref(dup.desc), ctypes.byref(nbytes)) == -2
    # candidates: outage of a shifter, split of a shifter's bus (accepted)
    buses = [int(g.f[l]) for l in pst] + [int(g.t[l]) for l in pst]
    a = next(x for x in buses if len(g.incident(x)) >= 3)
    c = G.Candidates.from_lists([[], [(G.KIND_OUTAGE, pst[0], 0, 0.0)],
                                 [(G.KIND_SPLIT, a, 2, 0.0)]])
    d.validate_candidates(ok, c)


def test_status_strings(d):
    """Every status of the header has its own message (the launch-shape status
    of a tuning included); unknown codes are named as such."""
    import ctypes
    f = d._lib.dcflow_strerror
    f.restype = ctypes.c_char_p
    f.argtypes = [ctypes.c_int]
    msgs = [f(c).decode() for c in range(0, -9, -1)]
    assert len(set(msgs)) == len(msgs)
    assert "unknown" not in " ".join(msgs)
    assert "launch shape" in msgs[8]
    assert f(-9).decode() == "unknown status"
