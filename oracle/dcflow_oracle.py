"""Plain FP64 CPU oracle for the batched DC-loadflow screen.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports, links or
calls this module; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

It computes, slowly and directly, what the GPU path computes with low-rank
updates: for every topology candidate the grid is rebuilt (busbar splits
re-terminate branches on a new node, remedial outages drop branches), the
reduced nodal susceptance system is factorised from scratch by dense LU
(LAPACK getrf/getrs, partial pivoting) and solved for every injection variant.
No base PTDF, BSDF or MODF is ever used.

Paper passages followed (Westerbeck et al., "Accelerated DC loadflow solver
for topology optimization"):
  * Sec. II, definition of the weighted connectivity matrix C_w and of the
    nodal susceptance matrix B (a graph Laplacian); slack exclusion (primes).
  * Sec. II, Def. of the PTDF (PTDF' B' = C_w', slack column zero) and the N-0
    flows p = PTDF P (Eq. ptdf_times_nodal_inj).
  * Sec. II, Def. of the LODF and Eq. lodf_delta for N-1 flows, applied with
    the candidate network's own PTDF.
  * Sec. II, Eq. ptdf_delta (flow change = PTDF times the injection change)
    and Sec. III-C step 8d: generator-outage N-1 cases, here by solving the
    candidate network again with the lost output removed.
  * Def. eq_modf and Sec. III-C steps 5 and 8c: multi-outage N-1 cases (several
    branches tripped together), here by solving the candidate network again
    without all of them.
  * Sec. III-A, task definition: N-0 and N-1 flows over monitored branches,
    agg_m = maximum relative branch load, t_i* = argmin over the injection
    variants (Eq. solver_end_to_end).

Readings where the paper is silent:
  * the new busbar of the j-th split of a candidate is node n_bus + j;
  * the slack absorbs any imbalance (its injection is minus the sum of the
    others), which leaves all flows unchanged since its PTDF column is zero;
  * an N-1 contingency that is a bridge of the candidate network islands part
    of the grid: it is excluded from the score and counted;
  * an N-1 contingency already removed by a remedial outage leaves the N-0
    flows unchanged (it is still scored);
  * a generator outage removes the generator's output from its bus (busbar A
    when the candidate splits that bus) and the slack takes it up; generator
    cases come after the branch contingencies and are reported as -2 - g;
  * a multi-outage case that islands the candidate network is excluded and
    counted with the islanding contingencies; branches the candidate removed
    drop out of it; multi cases come after the generator outages and are
    reported as -2 - G - q (G generator outages);
  * agg_m covers N-0 and every valid N-1 case over the monitored branches;
    the overload sum adds max(0, |p|/r - 1) over the same set for the best
    variant; ties pick the lowest variant, then the lowest (outage, branch)
    with the N-0 case first.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

KIND_OUTAGE = 0
KIND_SPLIT = 1

ST_DISCONNECTED = 1
ST_SINGULAR = 2
ST_NONFINITE = 4


# ------------------------------------------------------------- matrices

def weighted_connectivity(n, f, t, b):
    """C_w[l, f_l] = b_l, C_w[l, t_l] = -b_l (Sec. II definition)."""
    m = len(f)
    cw = np.zeros((m, n))
    rows = np.arange(m)
    cw[rows, f] += b
    cw[rows, t] -= b
    return cw


def nodal_susceptance(n, f, t, b):
    """Graph Laplacian B: off-diagonal -b per edge, diagonal = sum of incident b."""
    bm = np.zeros((n, n))
    for fl, tl, bl in zip(f, t, b):
        bm[fl, fl] += bl
        bm[tl, tl] += bl
        bm[fl, tl] -= bl
        bm[tl, fl] -= bl
    return bm


def _keep(n, slack):
    return np.array([i for i in range(n) if i != slack], dtype=np.int64)


def ptdf(n, f, t, b, slack):
    """Solution of PTDF' B' = C_w' with a zero slack column (Def. eq_ptdf)."""
    keep = _keep(n, slack)
    br = nodal_susceptance(n, f, t, b)[np.ix_(keep, keep)]
    cw = weighted_connectivity(n, f, t, b)[:, keep]
    # PTDF' = C_w' B'^-1 ; B' is symmetric, so solve B' Y = C_w'^T, PTDF' = Y^T.
    y = sla.solve(br, cw.T)
    h = np.zeros((len(f), n))
    h[:, keep] = y.T
    return h


def dc_flows(n, f, t, b, slack, p):
    """Branch flows for nodal injections ``p`` ([n] or [V, n]) by a dense LU
    solve of the reduced system B' theta' = P' (theta_slack = 0)."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    keep = _keep(n, slack)
    br = nodal_susceptance(n, f, t, b)[np.ix_(keep, keep)]
    theta = np.zeros((p.shape[0], n))
    theta[:, keep] = sla.lu_solve(sla.lu_factor(br), p[:, keep].T).T
    return b * (theta[:, f] - theta[:, t])


# ------------------------------------------------------------ graph tests

def connected(n, f, t):
    """Union-find connectivity test."""
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    comps = n
    for a, c in zip(f, t):
        ra, rc = find(int(a)), find(int(c))
        if ra != rc:
            parent[ra] = rc
            comps -= 1
    return comps == 1


def bridges(n, f, t):
    """Bridge edges of an undirected multigraph (Tarjan low-link, iterative).
    Parallel edges are distinguished by edge id, so a doubled line is no bridge."""
    m = len(f)
    adj = [[] for _ in range(n)]
    for e in range(m):
        adj[int(f[e])].append((int(t[e]), e))
        adj[int(t[e])].append((int(f[e]), e))
    disc = [-1] * n
    low = [0] * n
    out = np.zeros(m, bool)
    timer = 0
    for root in range(n):
        if disc[root] != -1:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, iter(adj[root]))]
        while stack:
            u, pe, it = stack[-1]
            descended = False
            for (w, e) in it:
                if e == pe:
                    continue
                if disc[w] == -1:
                    disc[w] = low[w] = timer
                    timer += 1
                    stack.append((w, e, iter(adj[w])))
                    descended = True
                    break
                low[u] = min(low[u], disc[w])
            if descended:
                continue
            stack.pop()
            if stack:
                par = stack[-1][0]
                low[par] = min(low[par], low[u])
                if low[u] > disc[par]:
                    out[pe] = True
    return out


# ----------------------------------------------------- candidate rebuild

def incident_branches(f, t, bus):
    return np.flatnonzero((np.asarray(f) == bus) | (np.asarray(t) == bus))


def rebuild(n, f, t, elems):
    """Post-change network of a candidate (step 1 of the oracle).

    Returns (n_nodes, f2, t2, alive, splits) where splits lists
    (A, B, p_new) per split in element order; B = n + j for the j-th split.
    Branch ids are kept; removed branches have alive = False.
    """
    f2 = np.asarray(f, np.int64).copy()
    t2 = np.asarray(t, np.int64).copy()
    alive = np.ones(len(f2), bool)
    splits = []
    for (kind, ident, mask, p_new) in elems:
        if kind == KIND_SPLIT:
            a = int(ident)
            newbus = n + len(splits)
            for bit, br in enumerate(incident_branches(f, t, a)):
                if (int(mask) >> bit) & 1:
                    if f[br] == a:
                        f2[br] = newbus
                    else:
                        t2[br] = newbus
            # p_new: one value, or one per injection variant (injection topologies T_i
            # of Sec. III-A regroup a substation's injections between its busbars)
            pn = np.asarray(p_new, np.float64)
            splits.append((a, newbus, float(pn) if pn.ndim == 0 else pn))
        elif kind == KIND_OUTAGE:
            alive[int(ident)] = False
        else:
            raise ValueError(f"unknown element kind {kind}")
    return n + len(splits), f2, t2, alive, splits


def candidate_injections(n_nodes, x, splits, slack):
    """Injections of the rebuilt network for base-numbered variants ``x``
    ([V, n]): busbar B_j receives p_new_j (a number, or one per variant), taken
    from its parent bus A_j; the slack absorbs the imbalance."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    v, n = x.shape
    p = np.zeros((v, n_nodes))
    p[:, :n] = x
    for (a, bnew, pn) in splits:
        p[:, bnew] += pn
        p[:, a] -= pn
    p[:, slack] = 0.0
    p[:, slack] = -p.sum(axis=1)
    return p


def ratings(n, f, t, b, slack, p_base, mon, scale=1.2, offset=0.1):
    """Workload rating rule: r = scale |base flow| + offset on monitored rows."""
    fb = dc_flows(n, f, t, b, slack, p_base)[0]
    return scale * np.abs(fb[np.asarray(mon)]) + offset


# ---------------------------------------------------- per-candidate solve

def control_terms(n2, f2, t2, alive, b, controls, ctrl):
    """Nodal injections and direct branch-flow terms of the controls (the end of
    Sec. II names phase shifters and HVDC links, modelled through PSDF/DCDF,
    without formulas; the DC models used here):

      * a phase-shifting transformer of angle alpha (rad) in series with branch l:
        p_l = b_l (theta_f - theta_t - alpha), i.e. Kirchhoff's law sees an extra
        injection b_l alpha at f and -b_l alpha at t, and the flow on l itself
        carries -b_l alpha on top of b_l (theta_f - theta_t); a phase shifter on
        a removed branch does nothing;
      * an HVDC link from bus i to bus j with setpoint P withdraws P at i and
        injects it at j.

    controls = dict(pst=[branch ids], hvdc=[(i, j)], pst_scale (rad per unit of
    ctrl), hvdc_scale (p.u. per unit of ctrl)); ctrl [V, n_pst + n_hvdc].
    Terminals are those of the (possibly rebuilt) network f2, t2.
    Returns (dp [V, n2], dflow [V, m])."""
    ctrl = np.atleast_2d(np.asarray(ctrl, np.float64))
    v = ctrl.shape[0]
    pst = list(controls.get("pst", []))
    hvdc = list(controls.get("hvdc", []))
    dp = np.zeros((v, n2))
    dflow = np.zeros((v, len(f2)))
    for q, l in enumerate(pst):
        if not alive[l]:
            continue
        a = ctrl[:, q] * controls.get("pst_scale", np.pi / 180.0)
        dp[:, f2[l]] += b[l] * a
        dp[:, t2[l]] -= b[l] * a
        dflow[:, l] -= b[l] * a
    for q, (i, j) in enumerate(hvdc):
        pv = ctrl[:, len(pst) + q] * controls.get("hvdc_scale", 1.0)
        dp[:, i] -= pv
        dp[:, j] += pv
    return dp, dflow


def candidate_flows(n, f, t, b, slack, elems, x, out, controls=None, ctrl=None, gens=None):
    """N-0 flows and N-1 flows of a candidate, by rebuild + dense LU.

    Returns dict with
      p0 [V, m]          N-0 flows (0 on removed branches);
      state [|O|]        0 = valid LODF case, 1 = already removed (p1 = p0),
                         2 = islanding (bridge of the candidate network);
      lodf [m, |O|]      LODF columns of the candidate network (Def. eq_lodf,
                         with LODF[c, c] = -1), zero for states 1 and 2;
      den [|O|]          LODF denominators 1 - (PTDF'[c, f_c] - PTDF'[c, t_c]);
      gcol [m, G]        PTDF' column of each generator's bus (gens = (bus ids,
                         outputs); G = 0 without gens): losing generator g
                         changes the flows by -P_g gcol[:, g] (Eq. ptdf_delta);
      connected          False if the candidate network itself is islanded.
    """
    n2, f2, t2, alive, splits = rebuild(n, f, t, elems)
    m = len(f2)
    fa, ta, ba = f2[alive], t2[alive], np.asarray(b)[alive]
    res = dict(n_nodes=n2, f=f2, t=t2, alive=alive, splits=splits)
    if not connected(n2, fa, ta):
        res["connected"] = False
        return res
    res["connected"] = True
    keep = _keep(n2, slack)
    br = nodal_susceptance(n2, fa, ta, ba)[np.ix_(keep, keep)]
    lu = sla.lu_factor(br)
    p = candidate_injections(n2, x, splits, slack)
    dflow = None
    if controls is not None:
        dp, dflow = control_terms(n2, f2, t2, alive, np.asarray(b), controls, ctrl)
        p = p + dp
        p[:, slack] = 0.0
    theta = np.zeros((p.shape[0], n2))
    theta[:, keep] = sla.lu_solve(lu, p[:, keep].T).T
    p0 = np.zeros((p.shape[0], m))
    p0[:, alive] = ba * (theta[:, fa] - theta[:, ta])
    if dflow is not None:
        p0 = p0 + dflow
    res["p0"] = p0

    out = np.asarray(out, np.int64)
    isb = np.zeros(m, bool)
    isb[np.flatnonzero(alive)] = bridges(n2, fa, ta)
    state = np.zeros(len(out), np.int8)
    state[~alive[out]] = 1
    state[alive[out] & isb[out]] = 2
    lodf = np.zeros((m, len(out)))
    den = np.zeros(len(out))
    valid = np.flatnonzero(state == 0)
    if len(valid):
        cs = out[valid]
        # PTDF' of the candidate network applied to the transfer d_c = e_f' - e_t'
        d = np.zeros((n2, len(cs)))
        d[f2[cs], np.arange(len(cs))] += 1.0
        d[t2[cs], np.arange(len(cs))] -= 1.0
        xs = np.zeros((n2, len(cs)))
        xs[keep] = sla.lu_solve(lu, d[keep])
        col = np.zeros((m, len(cs)))
        col[alive] = ba[:, None] * (xs[fa] - xs[ta])
        dd = 1.0 - col[cs, np.arange(len(cs))]
        lodf[:, valid] = col / dd
        lodf[cs, valid] = -1.0
        den[valid] = dd
    gb = np.asarray([] if gens is None else gens[0], np.int64)
    gcol = np.zeros((m, len(gb)))
    if len(gb):
        # unit injection at the generator's bus, taken up by the slack
        e = np.zeros((n2, len(gb)))
        e[gb, np.arange(len(gb))] = 1.0
        th = np.zeros((n2, len(gb)))
        th[keep] = sla.lu_solve(lu, e[keep])
        gcol[alive] = ba[:, None] * (th[fa] - th[ta])
    res.update(state=state, lodf=lodf, den=den, gcol=gcol)
    return res


def n1_flows_bruteforce(n, f, t, b, slack, elems, x, out, controls=None, ctrl=None, gens=None):
    """N-1 flows by rebuilding the candidate network without each contingency
    and solving again (one factorisation per case), controls included with the
    model of control_terms on each post-contingency network; then, for each
    generator outage of gens = (bus ids, outputs), the candidate network solved
    with that output removed from its bus (the slack re-balances).  Returns
    (p1 [V, |O| + G, m], islanded [|O| + G])."""
    n2, f2, t2, alive, splits = rebuild(n, f, t, elems)
    p = candidate_injections(n2, x, splits, slack)
    m = len(f2)
    out = np.asarray(out, np.int64)
    gb = np.asarray([] if gens is None else gens[0], np.int64)
    gp = np.asarray([] if gens is None else gens[1], np.float64)
    p1 = np.zeros((p.shape[0], len(out) + len(gb), m))
    isl = np.zeros(len(out) + len(gb), bool)
    keep = _keep(n2, slack)
    for ci, c in enumerate(out):
        al = alive.copy()
        al[c] = False
        fa, ta, ba = f2[al], t2[al], np.asarray(b)[al]
        if not connected(n2, fa, ta):
            isl[ci] = True
            continue
        br = nodal_susceptance(n2, fa, ta, ba)[np.ix_(keep, keep)]
        pc, dflow = p, None
        if controls is not None:
            dp, dflow = control_terms(n2, f2, t2, al, np.asarray(b), controls, ctrl)
            pc = p + dp
        theta = np.zeros((p.shape[0], n2))
        theta[:, keep] = sla.solve(br, pc[:, keep].T).T
        p1[:, ci, al] = ba * (theta[:, fa] - theta[:, ta])
        if dflow is not None:
            p1[:, ci, :] += dflow
    if len(gb):
        fa, ta, ba = f2[alive], t2[alive], np.asarray(b)[alive]
        if not connected(n2, fa, ta):
            isl[len(out):] = True
            return p1, isl
        br = nodal_susceptance(n2, fa, ta, ba)[np.ix_(keep, keep)]
        pc, dflow = p, None
        if controls is not None:
            dp, dflow = control_terms(n2, f2, t2, alive, np.asarray(b), controls, ctrl)
            pc = p + dp
        for gi in range(len(gb)):
            pg = pc.copy()
            pg[:, gb[gi]] -= gp[gi]
            pg[:, slack] = 0.0
            pg[:, slack] = -pg.sum(axis=1)
            theta = np.zeros((p.shape[0], n2))
            theta[:, keep] = sla.solve(br, pg[:, keep].T).T
            p1[:, len(out) + gi, alive] = ba * (theta[:, fa] - theta[:, ta])
            if dflow is not None:
                p1[:, len(out) + gi, :] += dflow
    return p1, isl


def multi_outage_flows(n, f, t, b, slack, elems, x, cases, controls=None, ctrl=None):
    """Flows of the candidate network with every branch of a case tripped
    together (cases: lists of branch ids), by solving that network again; the
    controls follow control_terms on it.  Returns (p [V, Q, m], islanded [Q])."""
    n2, f2, t2, alive, splits = rebuild(n, f, t, elems)
    p = candidate_injections(n2, x, splits, slack)
    m = len(f2)
    keep = _keep(n2, slack)
    pm = np.zeros((p.shape[0], len(cases), m))
    isl = np.zeros(len(cases), bool)
    for qi, case in enumerate(cases):
        al = alive.copy()
        al[np.asarray(case, np.int64)] = False
        fa, ta, ba = f2[al], t2[al], np.asarray(b)[al]
        if not connected(n2, fa, ta):
            isl[qi] = True
            continue
        br = nodal_susceptance(n2, fa, ta, ba)[np.ix_(keep, keep)]
        pc, dflow = p, None
        if controls is not None:
            dp, dflow = control_terms(n2, f2, t2, al, np.asarray(b), controls, ctrl)
            pc = p + dp
        theta = np.zeros((p.shape[0], n2))
        theta[:, keep] = sla.solve(br, pc[:, keep].T).T
        pm[:, qi, al] = ba * (theta[:, fa] - theta[:, ta])
        if dflow is not None:
            pm[:, qi, :] += dflow
    return pm, isl


def score_candidate(n, f, t, b, slack, elems, x, mon, out, rating, controls=None, ctrl=None,
                    gens=None, multi=None):
    """Score one candidate over its injection variants (Sec. III-A); gens =
    (bus ids, outputs) adds the generator-outage N-1 cases (Sec. III-C step 8d),
    multi = [branch id lists] the multi-outage cases (steps 5 and 8c).

    Returns dict(max_load [V], best_variant, best_max_load, overload_sum,
    worst_branch, worst_outage, n_island, status)."""
    mon = np.asarray(mon, np.int64)
    out = np.asarray(out, np.int64)
    r = np.asarray(rating, np.float64)
    # (with controls the N-0 flows carry the phase shifts' direct terms; tripping a
    # branch, phase shifter or not, leaves the other shifts fixed and moves its N-0
    # flow through the rest of the network: the LODF superposition below holds)
    cf = candidate_flows(n, f, t, b, slack, elems, x, out, controls, ctrl, gens)
    nv = np.atleast_2d(x).shape[0]
    if not cf["connected"]:
        return dict(max_load=np.full(nv, np.inf), best_variant=-1, best_max_load=np.inf,
                    overload_sum=0.0, worst_branch=-1, worst_outage=-1, n_island=0,
                    status=ST_DISCONNECTED, flows=cf)
    p0 = cf["p0"]
    state = cf["state"]
    lodf = cf["lodf"]
    scored = np.flatnonzero(state != 2)
    # N-1 flows on the monitored rows: p1[v, c, l] = p0[v, l] + LODF[l, c] p0[v, c]
    p1 = p0[:, None, mon] + lodf[mon][:, scored].T[None, :, :] * p0[:, out[scored]][:, :, None]
    case_ids = out[scored]
    if gens is not None and len(gens[0]):
        # generator g lost: p0 - P_g PTDF'[:, bus_g] (Eq. ptdf_delta)
        gp = np.asarray(gens[1], np.float64)
        pg = p0[:, None, mon] - gp[None, :, None] * cf["gcol"][mon].T[None, :, :]
        p1 = np.concatenate([p1, pg], axis=1)
        case_ids = np.concatenate([case_ids, -2 - np.arange(len(gp))])
    n_isl_multi = 0
    if multi is not None and len(multi):
        pm, isl_m = multi_outage_flows(n, f, t, b, slack, elems, x, multi, controls, ctrl)
        okq = np.flatnonzero(~isl_m)
        p1 = np.concatenate([p1, pm[:, okq][:, :, mon]], axis=1)
        n_gen = 0 if gens is None else len(gens[0])
        case_ids = np.concatenate([case_ids, -2 - n_gen - okq])
        n_isl_multi = int(isl_m.sum())
    load0 = np.abs(p0[:, mon]) / r
    load1 = np.abs(p1) / r
    maxl = load0.max(axis=1)
    if p1.shape[1]:
        maxl = np.maximum(maxl, load1.reshape(nv, -1).max(axis=1))
    best = int(np.argmin(maxl))
    allload = np.concatenate([load0[best][None, :], load1[best]], axis=0)
    ov = float(np.maximum(allload - 1.0, 0.0).sum())
    flat = int(np.argmax(allload))
    ci, li = divmod(flat, len(mon))
    worst_out = -1 if ci == 0 else int(case_ids[ci - 1])
    status = 0
    if not np.all(np.isfinite(maxl)):
        status |= ST_NONFINITE
    return dict(max_load=maxl, best_variant=best, best_max_load=float(maxl[best]),
                overload_sum=ov, worst_branch=int(mon[li]), worst_outage=worst_out,
                n_island=int((state == 2).sum()) + n_isl_multi, status=status, flows=cf,
                loads_best=allload, scored_out=case_ids)


def worst_cases(sc, mon, out, k):
    """agg_i of Sec. III-A for the winning variant (metric-first mode, Sec. IV-B:
    the details are produced for t_i* only): the k largest relative loads over
    the monitored branches in N-0 and in every scored N-1 case, as a list of
    (load, branch, outage) with outage -1 for N-0.  Order: load descending, ties
    by case (N-0 first, then contingencies in the order of `out`, then generator
    outages, then multi-outage cases), then by the branch's position in `mon`.  `sc` is a result of score_candidate; a
    disconnected candidate has no entries."""
    if sc["best_variant"] < 0:
        return []
    mon = np.asarray(mon, np.int64)
    out = np.asarray(out, np.int64)
    loads = sc["loads_best"]               # [1 + n_scored, n_mon]
    pos = {int(o): i for i, o in enumerate(out)}
    # generator g (id -2 - g) ranks after every branch contingency, multi case q
    # (id -2 - G - q) after every generator
    pos.update({int(o): len(out) - 2 - int(o) for o in sc["scored_out"] if o <= -2})
    cases = np.asarray([-1] + [int(o) for o in sc["scored_out"]], np.int64)
    # ordering key of every entry: the branch's position for N-0, else
    # (position of the contingency in `out` + 1) * n_mon + position
    first = np.asarray([0] + [(pos[int(o)] + 1) * len(mon) for o in cases[1:]], np.int64)
    keys = first[:, None] + np.arange(len(mon))[None, :]
    flat = loads.ravel()
    k = min(k, flat.size)
    if k == 0:
        return []
    # every entry at or above the k-th largest load, then an exact sort of those
    kth = np.partition(flat, flat.size - k)[flat.size - k]
    sel = np.flatnonzero(flat >= kth)
    order = sel[np.lexsort((keys.ravel()[sel], -flat[sel]))][:k]
    ci, li = np.divmod(order, len(mon))
    return [(float(flat[j]), int(mon[b]), int(cases[c])) for j, c, b in zip(order, ci, li)]


def worst_cases_per_case(sc, mon, out, per_case, k):
    """agg_i in the two levels of Sec. IV-B: within every case of the winning
    variant (N-0, each scored contingency, generator and multi-outage case) the
    per_case largest loads (ties: branch position in `mon`), then the k largest of
    their collection, ordered as in worst_cases (load descending, then case, then
    branch position).  A case thus holds at most per_case places."""
    if sc["best_variant"] < 0:
        return []
    mon = np.asarray(mon, np.int64)
    out = np.asarray(out, np.int64)
    loads = sc["loads_best"]               # [cases, n_mon]
    cases = np.asarray([-1] + [int(o) for o in sc["scored_out"]], np.int64)
    pos = {int(o): i for i, o in enumerate(out)}
    pos.update({int(o): len(out) - 2 - int(o) for o in sc["scored_out"] if o <= -2})
    first = [0] + [(pos[int(o)] + 1) * len(mon) for o in cases[1:]]
    picked = []                            # (load, key, case row, branch position)
    for ci in range(loads.shape[0]):
        order = np.lexsort((np.arange(len(mon)), -loads[ci]))[:per_case]
        picked += [(float(loads[ci, b]), first[ci] + int(b), ci, int(b)) for b in order]
    picked.sort(key=lambda e: (-e[0], e[1]))
    return [(v, int(mon[b]), int(cases[ci])) for v, _, ci, b in picked[:k]]


def score_workload(w, idx=None, rating=None):
    """Score the candidates ``idx`` (default all) of a gridgen Workload."""
    g = w.grid
    if rating is None:
        rating = ratings(g.n_bus, g.f, g.t, g.b, g.slack, g.p, w.mon,
                         w.rating_scale, w.rating_offset)
    if idx is None:
        idx = range(w.cands.n_cand)
    res = []
    for i in idx:
        x = w.inj if w.inj_shared else w.inj[i]
        res.append(score_candidate(g.n_bus, g.f, g.t, g.b, g.slack, w.cands.elements(int(i)),
                                   x, w.mon, w.out, rating, gens=getattr(w, "gens", None),
                                   multi=getattr(w, "multi", None)))
    return res, rating
