"""The paper's distribution-factor formulas, written out on dense PTDFs.

TEST INFRASTRUCTURE ONLY (small grids).  These functions restate Sec. II of
the paper (Def. eq_lodf, Eq. lodf_ptdf, Def. eq_modf, Def. eq_bsdf and
Eq. bsdf_application) so that the tests can pin each reading of the paper
against the rebuild-and-factorise oracle in ``dcflow_oracle``.  The solver
library does not use them.

Readings (the paper leaves these open):
  * MODF: the outaged from/to node "sets" are ordered lists, one column per
    outaged branch;
  * BSDF: the new busbar B gets an extended PTDF column equal to column A
    (both are one electrical node before the coupler opens); S is the set of
    branches that stay on busbar A; the correction vector uses the sign of the
    branch orientation at A; the coupler row PTDF_bbc follows from Kirchhoff's
    current law at A: injection at A minus the flow leaving A over S, where a
    PTDF column means a unit injection withdrawn at the slack; so when A is
    itself the slack every non-slack entry drops by one, and the slack entry
    is zero like in every PTDF row.
"""
from __future__ import annotations

import numpy as np


def lodf_matrix(h, f, t):
    """Def. eq_lodf: column k = (PTDF[:, f_k] - PTDF[:, t_k]) / (1 - (PTDF[k, f_k] - PTDF[k, t_k])),
    with -1 on the diagonal."""
    d = h[:, f] - h[:, t]
    den = 1.0 - np.diag(d)
    with np.errstate(divide="ignore", invalid="ignore"):   # bridges: zero denominator
        out = d / den[None, :]
    np.fill_diagonal(out, -1.0)
    return out


def ptdf_after_outage(h, f, t, k):
    """Eq. lodf_ptdf: PTDF' = PTDF + LODF[:, k] PTDF[k, :]."""
    d = h[:, f[k]] - h[:, t[k]]
    col = d / (1.0 - d[k])
    col[k] = -1.0
    return h + np.outer(col, h[k])


def modf(h, f, t, outs):
    """Def. eq_modf: MODF (I - (PTDF[O, fO] - PTDF[O, tO])) = PTDF[:, fO] - PTDF[:, tO],
    then the rows of the outaged branches are set to -identity."""
    outs = np.asarray(outs)
    d = h[:, f[outs]] - h[:, t[outs]]
    mm = d[outs, :]
    k = len(outs)
    res = np.linalg.solve((np.eye(k) - mm).T, d.T).T
    res[outs, :] = -np.eye(k)
    return res


def ptdf_after_modf(h, f, t, outs):
    """PTDF' = PTDF + MODF PTDF[O, :] (the MODF analogue of Eq. lodf_ptdf)."""
    return h + modf(h, f, t, outs) @ h[np.asarray(outs)]


def bsdf_split(h, f, t, b, bus_a, moved, slack=0):
    """One two-way split of ``bus_a``: branches ``moved`` go to a new node
    B = h.shape[1] (appended column), the rest (S) stay on A.

    Returns the post-split PTDF (|E| x (n+1)) by Def. eq_bsdf and
    Eq. bsdf_application."""
    m, n = h.shape
    inc = np.flatnonzero((f == bus_a) | (t == bus_a))
    moved = set(int(x) for x in moved)
    stay = [int(l) for l in inc if int(l) not in moved]
    hx = np.concatenate([h, h[:, [bus_a]]], axis=1)   # column B := column A
    bnode = n
    beta = sum(b[l] for l in stay)
    p_shift = np.zeros(n + 1)
    p_shift[bnode] = -1.0
    p_corr = np.zeros(m)
    bbc = np.zeros(n + 1)
    bbc[bus_a] = 1.0
    for l in stay:
        far = t[l] if f[l] == bus_a else f[l]
        s = 1.0 if f[l] == bus_a else -1.0
        p_shift[far] += b[l] / beta
        p_corr[l] = s * b[l] / beta
        bbc -= s * hx[l]
    if bus_a == slack:
        bbc -= 1.0        # the unit injection at any node is withdrawn at A itself
    bbc[slack] = 0.0      # like every PTDF row, the coupler row has a zero slack column
    vec = (hx @ p_shift + p_corr) / (1.0 - bbc @ p_shift)
    return hx + np.outer(vec, bbc)
