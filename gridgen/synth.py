"""Seeded synthetic inputs for the batched DC-loadflow screen.

Input data only: grid topology, susceptances, balanced nodal injections,
monitored / contingency branch sets, topology candidates and injection
variants.  Nothing here solves a loadflow; branch ratings, which depend on the
base-case flows, are derived by each consumer (the solver library computes
them on the device, the CPU oracle computes its own).

Grid recipe (random geometric meshed grid):
  * bus positions uniform in [0, 1)^2;
  * spanning tree: buses in random order, each attached to the nearest bus
    already placed;
  * chords: a random bus joined to one of its 2nd..5th nearest buses, no
    duplicates, no self loops, until the branch count is reached;
  * random orientation per branch, reactance x ~ lognormal(-2.5, 0.5) p.u.,
    susceptance b = 1/x;
  * injections P ~ N(0, 1) shifted to sum to zero; bus 0 is the slack.

Candidate encoding (one record per topology candidate, CSR over elements):
  kind 0 = remedial outage of branch ``id`` (the paper's t_d);
  kind 1 = two-way split of bus ``id`` (the paper's t_b): bit i of ``mask``
  moves the i-th incident branch of the bus (incident branches taken in
  ascending branch id) onto the new busbar B; ``p_new`` is the injection that
  moves with them (0: the bus injection stays on busbar A).
"""
from __future__ import annotations

from dataclasses import dataclass, field

from typing import Optional

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

KIND_OUTAGE = 0
KIND_SPLIT = 1
MAX_RANK = 8          # elements per candidate
MAX_SPLIT_DEGREE = 32  # incident branches addressable by a 32-bit mask


@dataclass
class Grid:
    n_bus: int
    f: np.ndarray      # int32 [m] from bus
    t: np.ndarray      # int32 [m] to bus
    x: np.ndarray      # float64 [m] reactance
    b: np.ndarray      # float64 [m] susceptance 1/x
    p: np.ndarray      # float64 [n] balanced base injections
    pos: np.ndarray    # float64 [n, 2]
    slack: int = 0

    @property
    def n_branch(self) -> int:
        return int(self.f.shape[0])

    def incident(self, bus: int) -> np.ndarray:
        """Branch ids touching ``bus`` in ascending order (mask bit order)."""
        adj = self.__dict__.get("_adj")
        if adj is None:
            m = len(self.f)
            ends = np.concatenate([self.f, self.t]).astype(np.int64)
            br = np.concatenate([np.arange(m), np.arange(m)])
            order = np.lexsort((br, ends))
            off = np.zeros(self.n_bus + 1, np.int64)
            np.add.at(off, ends + 1, 1)
            adj = (np.cumsum(off), br[order].astype(np.int32))
            self.__dict__["_adj"] = adj
        off, lst = adj
        return lst[off[bus]:off[bus + 1]]

    def degree(self) -> np.ndarray:
        return np.bincount(np.concatenate([self.f, self.t]), minlength=self.n_bus)


@dataclass
class Candidates:
    off: np.ndarray     # int32 [n_cand + 1]
    kind: np.ndarray    # int8  [n_elem]
    id: np.ndarray      # int32 [n_elem]
    mask: np.ndarray    # uint32 [n_elem]
    p_new: np.ndarray   # float64 [n_elem]

    @property
    def n_cand(self) -> int:
        return int(self.off.shape[0] - 1)

    @property
    def n_elem(self) -> int:
        return int(self.kind.shape[0])

    def elements(self, i: int):
        """List of (kind, id, mask, p_new) tuples of candidate ``i``."""
        a, e = int(self.off[i]), int(self.off[i + 1])
        return [(int(self.kind[j]), int(self.id[j]), int(self.mask[j]), float(self.p_new[j]))
                for j in range(a, e)]

    def subset(self, idx) -> "Candidates":
        return Candidates.from_lists([self.elements(int(i)) for i in idx])

    @staticmethod
    def from_lists(cands) -> "Candidates":
        off = np.zeros(len(cands) + 1, np.int32)
        kind, ids, masks, pn = [], [], [], []
        for i, els in enumerate(cands):
            off[i + 1] = off[i] + len(els)
            for (k, d, m, p) in els:
                kind.append(k)
                ids.append(d)
                masks.append(m)
                pn.append(p)
        return Candidates(off, np.asarray(kind, np.int8), np.asarray(ids, np.int32),
                          np.asarray(masks, np.uint32), np.asarray(pn, np.float64))


@dataclass
class Workload:
    name: str
    grid: Grid
    mon: np.ndarray          # int32 monitored branch ids (E_m)
    out: np.ndarray          # int32 N-1 contingency branch ids (O)
    cands: Candidates
    inj: np.ndarray          # float64 [V, n] (shared) or [n_cand, V, n]
    inj_shared: bool
    rating_scale: float = 1.2
    rating_offset: float = 0.1
    meta: dict = field(default_factory=dict)
    # controls: None or dict(pst=[branch ids], pst_scale, hvdc=[(i, j)], hvdc_scale);
    # their values follow the n nodal entries of every injection vector
    controls: Optional[dict] = None
    # generator-outage N-1 cases: None or (bus ids int32 [G], lost outputs float64 [G])
    gens: Optional[tuple] = None
    # multi-outage N-1 cases: None or a list of branch-id lists (each within `out`)
    multi: Optional[list] = None

    @property
    def n_var(self) -> int:
        return int(self.inj.shape[-2])


# ---------------------------------------------------------------- grid

def make_grid(n_bus: int, n_branch: int, seed: int) -> Grid:
    if n_branch < n_bus - 1:
        raise ValueError("need at least n_bus - 1 branches for a connected grid")
    rng = np.random.default_rng(seed)
    pos = rng.random((n_bus, 2))
    order = rng.permutation(n_bus)
    edges = []
    placed = np.empty((n_bus, 2))
    placed_ids = np.empty(n_bus, np.int64)
    placed[0] = pos[order[0]]
    placed_ids[0] = order[0]
    for i in range(1, n_bus):
        u = order[i]
        d = np.sum((placed[:i] - pos[u]) ** 2, axis=1)
        v = placed_ids[int(np.argmin(d))]
        edges.append((int(v), int(u)))
        placed[i] = pos[u]
        placed_ids[i] = u
    have = {(min(a, c), max(a, c)) for a, c in edges}
    kq = min(6, n_bus)
    _, nbr = cKDTree(pos).query(pos, k=kq)
    tries = 0
    while len(edges) < n_branch:
        tries += 1
        if tries > 200 * n_branch:
            raise RuntimeError("could not place the requested number of chords")
        u = int(rng.integers(n_bus))
        lo = min(2, kq - 1)
        v = int(nbr[u, int(rng.integers(lo, kq))])
        if u == v:
            continue
        key = (min(u, v), max(u, v))
        if key in have:
            continue
        have.add(key)
        edges.append((u, v))
    e = np.asarray(edges, np.int64)
    flip = rng.random(len(e)) < 0.5
    f = np.where(flip, e[:, 1], e[:, 0]).astype(np.int32)
    t = np.where(flip, e[:, 0], e[:, 1]).astype(np.int32)
    x = rng.lognormal(mean=-2.5, sigma=0.5, size=len(e))
    p = rng.normal(0.0, 1.0, n_bus)
    p -= p.mean()
    return Grid(n_bus=n_bus, f=f, t=t, x=x, b=1.0 / x, p=p, pos=pos, slack=0)


# ------------------------------------------------------- topology helpers

def candidate_topology(grid: Grid, elems):
    """Post-change edge list of a candidate: (n_nodes, f, t, alive).

    New busbar of the j-th split (in element order) gets node id n_bus + j.
    """
    f = grid.f.astype(np.int64).copy()
    t = grid.t.astype(np.int64).copy()
    alive = np.ones(grid.n_branch, bool)
    n_new = 0
    for (k, d, m, _p) in elems:
        if k == KIND_SPLIT:
            inc = grid.incident(d)
            newbus = grid.n_bus + n_new
            n_new += 1
            for bit, br in enumerate(inc):
                if (m >> bit) & 1:
                    if grid.f[br] == d:
                        f[br] = newbus
                    else:
                        t[br] = newbus
        else:
            alive[d] = False
    return grid.n_bus + n_new, f, t, alive


_UF = None


def _uf_lib():
    """Optional C union-find (gridgen/libgguf.so, built by build_uf()); None if absent."""
    global _UF
    if _UF is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgguf.so")
        _UF = False
        if os.path.exists(path):
            lib = ctypes.CDLL(path)
            lib.gg_connected.restype = ctypes.c_int
            lib.gg_connected.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
            _UF = lib
    return _UF or None


def build_uf() -> str:
    """Compile the optional C union-find helper in place (gcc)."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    out = os.path.join(here, "libgguf.so")
    subprocess.run(["gcc", "-O2", "-shared", "-fPIC", os.path.join(here, "uf.c"), "-o", out],
                   check=True)
    return out


def is_connected(n_nodes: int, f, t, alive=None) -> bool:
    lib = _uf_lib()
    if lib is not None:
        f64 = np.ascontiguousarray(f, np.int64)
        t64 = np.ascontiguousarray(t, np.int64)
        al = None if alive is None else np.ascontiguousarray(alive, np.uint8)
        r = lib.gg_connected(int(n_nodes), len(f64), f64.ctypes.data, t64.ctypes.data,
                             None if al is None else al.ctypes.data)
        if r >= 0:
            return bool(r)
    if alive is not None:
        f = f[alive]
        t = t[alive]
    if n_nodes <= 1:
        return True
    g = coo_matrix((np.ones(len(f)), (f, t)), shape=(n_nodes, n_nodes))
    nc, _ = connected_components(g, directed=False)
    return nc == 1


def non_bridges(grid: Grid, rng, count: int) -> np.ndarray:
    """``count`` distinct branch ids, uniform among non-bridges of the grid."""
    chosen = []
    for br in rng.permutation(grid.n_branch):
        alive = np.ones(grid.n_branch, bool)
        alive[br] = False
        if is_connected(grid.n_bus, grid.f, grid.t, alive):
            chosen.append(int(br))
            if len(chosen) == count:
                break
    if len(chosen) < count:
        raise ValueError("grid has fewer non-bridge branches than requested")
    return np.sort(np.asarray(chosen, np.int32))


def _split_buses(grid: Grid) -> np.ndarray:
    deg = grid.degree()
    return np.flatnonzero((deg >= 3) & (deg <= MAX_SPLIT_DEGREE))


def random_split(grid: Grid, rng, bus: int):
    """Canonical non-trivial mask: bit 0 clear (first branch stays on A)."""
    d = len(grid.incident(bus))
    m = int(rng.integers(1, 1 << (d - 1))) << 1
    return (KIND_SPLIT, int(bus), m, 0.0)


def sample_candidate(grid: Grid, rng, n_split: int, n_out: int, split_buses=None,
                     max_tries: int = 200, forbid_out=()):
    """One connected candidate with ``n_split`` bus splits then ``n_out``
    remedial outages: a uniform set of distinct branches that keeps the
    candidate grid connected."""
    if split_buses is None:
        split_buses = _split_buses(grid)
    for _ in range(max_tries):
        buses = []
        while len(buses) < n_split:
            bus = int(split_buses[int(rng.integers(len(split_buses)))])
            if bus not in buses:
                buses.append(bus)
        elems = [random_split(grid, rng, bus) for bus in buses]
        n_nodes, f, t, alive = candidate_topology(grid, elems)
        if not is_connected(n_nodes, f, t, alive):
            continue
        if n_out == 0:
            return elems
        # remedial outages: a uniform set of distinct branches that keeps the
        # candidate grid connected (rejection sampling of the whole set)
        for _r in range(max_tries):
            outs = []
            while len(outs) < n_out:
                br = int(rng.integers(grid.n_branch))
                if br not in outs and br not in forbid_out:
                    outs.append(br)
            al = alive.copy()
            al[outs] = False
            if is_connected(n_nodes, f, t, al):
                return elems + [(KIND_OUTAGE, br, 0, 0.0) for br in outs]
    raise RuntimeError("could not sample a connected candidate")


def balanced(p: np.ndarray, slack: int) -> np.ndarray:
    """Return ``p`` with the slack entry set so every row sums to zero."""
    q = np.array(p, dtype=np.float64, copy=True)
    q[..., slack] = 0.0
    q[..., slack] = -q.sum(axis=-1)
    return q


def perturbed_injections(grid: Grid, rng, shape, rel_sigma: float) -> np.ndarray:
    """Load perturbations P_v = P_base (1 + rel_sigma g), g ~ N(0, 1) per bus."""
    g = rng.normal(0.0, 1.0, tuple(shape) + (grid.n_bus,))
    return balanced(grid.p * (1.0 + rel_sigma * g), grid.slack)


def attach_stubs(grid: Grid, rng, n_stubs: int, max_len: int = 3) -> Grid:
    """The grid with n_stubs radial chains of 1..max_len new buses attached to
    random buses (power-plant connections and their step-up transformers), each
    new bus injecting a positive output; the slack balances the total."""
    f, t, x = list(grid.f), list(grid.t), list(grid.x)
    p = list(grid.p)
    pos = [tuple(r) for r in grid.pos]
    n = grid.n_bus
    for _ in range(n_stubs):
        at = int(rng.integers(grid.n_bus))
        for _ in range(int(rng.integers(1, max_len + 1))):
            f.append(at)
            t.append(n)
            x.append(float(rng.lognormal(-2.5, 0.5)))
            p.append(float(rng.uniform(0.2, 1.5)))
            pos.append(tuple(grid.pos[at % grid.n_bus]))
            at = n
            n += 1
    p = balanced(np.asarray(p), grid.slack)
    x = np.asarray(x)
    return Grid(n_bus=n, f=np.asarray(f, np.int32), t=np.asarray(t, np.int32), x=x, b=1.0 / x,
                p=p, pos=np.asarray(pos), slack=grid.slack)


def generator_outages(grid: Grid, rng, n_gen: int):
    """Generator-outage N-1 cases: n_gen generators at distinct buses drawn among
    those with a positive base injection (the slack left out), each losing
    between half and all of its bus's base injection.  Returns (bus ids, outputs)."""
    gen_buses = np.flatnonzero(grid.p > 0.0)
    gen_buses = gen_buses[gen_buses != grid.slack]
    n_gen = min(n_gen, len(gen_buses))
    bus = np.sort(rng.choice(gen_buses, size=n_gen, replace=False)).astype(np.int32)
    pg = grid.p[bus] * rng.uniform(0.5, 1.0, size=n_gen)
    return bus, pg.astype(np.float64)


def multi_outage_cases(grid: Grid, out, rng, n_cases: int, max_size: int = 4):
    """Multi-outage N-1 cases drawn from the contingency list: half of them trip
    2..max_size contingency branches at one bus (a busbar fault; when they are all
    of the bus's branches the bus islands), the rest 2..max_size contingency
    branches anywhere (common-mode outages).  Returns a list of branch-id lists."""
    out = np.asarray(out, np.int64)
    in_out = np.zeros(grid.n_branch, bool)
    in_out[out] = True
    buses = [a for a in range(grid.n_bus) if in_out[grid.incident(a)].sum() >= 2]
    cases = []
    while len(cases) < n_cases:
        if len(cases) % 2 == 0 and buses:
            a = int(rng.choice(buses))
            inc = [int(l) for l in grid.incident(a) if in_out[l]]
            k = int(rng.integers(2, min(max_size, len(inc)) + 1))
            cases.append(sorted(int(x) for x in rng.choice(inc, size=k, replace=False)))
        else:
            k = int(rng.integers(2, max_size + 1))
            cases.append(sorted(int(x) for x in rng.choice(out, size=k, replace=False)))
    return cases


# ------------------------------------------------------------- workloads

def workload_tiny(seed: int = 0, n_cand: int = 100) -> Workload:
    """30 buses / 41 branches, single-split candidates, one injection, N-1 over
    every branch (bridges included), FP64."""
    rng = np.random.default_rng(seed + 1000)
    grid = make_grid(30, 41, seed)
    allbr = np.arange(grid.n_branch, dtype=np.int32)
    cands = Candidates.from_lists(
        [sample_candidate(grid, rng, 1, 0) for _ in range(n_cand)])
    inj = balanced(grid.p, grid.slack)[None, :]
    return Workload("tiny-30bus", grid, allbr, allbr, cands, inj, True,
                    meta=dict(n_bus=30, n_branch=41, n_cand=n_cand, n_var=1))


def busbar_injection_topologies(grid: Grid, cands: Candidates, rng, n_var: int,
                                n_parts: int = 4) -> np.ndarray:
    """Injection topologies T_i (Sec. III-A) for the split elements of a candidate
    set: the base injection of each split bus is cut into n_parts random shares
    (standing in for the loads and generators of the substation), and variant v
    puts a random subset of them on the new busbar.  Returns [n_elem][n_var] (0 for
    outage elements): the injection moved to busbar B per element and variant."""
    out = np.zeros((cands.n_elem, n_var))
    for e in range(cands.n_elem):
        if int(cands.kind[e]) != KIND_SPLIT:
            continue
        share = rng.dirichlet(np.ones(n_parts)) * float(grid.p[int(cands.id[e])])
        pick = rng.integers(0, 2, size=(n_var, n_parts))
        out[e] = pick @ share
    return out


def workload_medium(seed: int = 0, n_cand: int = 4096, n_var: int = 16,
                    n_out: int = 500) -> Workload:
    """1,000 buses / 1,600 branches, 1-3 splits plus 0-2 outages per candidate,
    16 load-perturbed injection variants per candidate, the 500 contingency
    branches are also the monitored set."""
    rng = np.random.default_rng(seed + 2000)
    grid = make_grid(1000, 1600, seed)
    out = non_bridges(grid, rng, n_out)
    sb = _split_buses(grid)
    lists = []
    for _ in range(n_cand):
        ns = int(rng.integers(1, 4))
        no = int(rng.integers(0, 3))
        lists.append(sample_candidate(grid, rng, ns, no, sb))
    cands = Candidates.from_lists(lists)
    inj = perturbed_injections(grid, rng, (n_cand, n_var), 0.05)
    return Workload("medium-1000bus", grid, out.copy(), out, cands, inj, False,
                    meta=dict(n_bus=1000, n_branch=1600, n_cand=n_cand, n_var=n_var,
                              n_out=n_out))


def workload_uneven(seed: int = 0, n_cand: int = 65536, n_out: int = 2000,
                    n_bus: int = 10000, n_branch: int = 15500) -> Workload:
    """10,000 buses / 15,500 branches, rank uniform in 1..8 (each element a
    split with probability 1/2, else an outage), one perturbed injection per
    candidate, every branch monitored, 2,000 contingencies."""
    rng = np.random.default_rng(seed + 3000)
    grid = make_grid(n_bus, n_branch, seed)
    out = non_bridges(grid, rng, n_out)
    sb = _split_buses(grid)
    lists = []
    for _ in range(n_cand):
        k = int(rng.integers(1, MAX_RANK + 1))
        ns = int(rng.binomial(k, 0.5))
        lists.append(sample_candidate(grid, rng, ns, k - ns, sb))
    cands = Candidates.from_lists(lists)
    inj = perturbed_injections(grid, rng, (n_cand, 1), 0.05)
    mon = np.arange(grid.n_branch, dtype=np.int32)
    return Workload("uneven-10000bus", grid, mon, out, cands, inj, False,
                    meta=dict(n_bus=n_bus, n_branch=n_branch, n_cand=n_cand, n_var=1,
                              n_out=n_out))



def _hops(grid: Grid, src: int) -> np.ndarray:
    """Breadth-first hop counts from bus ``src``."""
    adj = [[] for _ in range(grid.n_bus)]
    for a, c in zip(grid.f, grid.t):
        adj[int(a)].append(int(c))
        adj[int(c)].append(int(a))
    d = np.full(grid.n_bus, -1)
    d[src] = 0
    q = [src]
    for u in q:
        for v in adj[u]:
            if d[v] < 0:
                d[v] = d[u] + 1
                q.append(v)
    return d


def workload_brute(seed: int = 0, n_topo: int = 1024, n_comb: int = 4096, n_out: int = 1000,
                   n_bus: int = 2000, n_branch: int = 3100, n_pst: int = 20,
                   n_hvdc: int = 4) -> Workload:
    """Injection brute force: 2,000 buses / 3,100 branches with 20 phase shifters
    (random non-bridges) and 4 HVDC links (random bus pairs at least 5 hops
    apart); topologies as in the medium workload (1-3 splits + 0-2 outages; a
    split may move a shifter's branch and an outage may remove one); the same
    n_comb control and load combinations for every topology (integer shifter
    degrees in -10..10, HVDC levels 0..7 of 0.25 p.u., loads perturbed by
    N(0, 0.05)); every branch monitored, n_out contingencies among the
    non-bridges (shifters included)."""
    rng = np.random.default_rng(seed + 4000)
    grid = make_grid(n_bus, n_branch, seed)
    pst = [int(x) for x in non_bridges(grid, rng, n_pst)]
    hvdc = []
    while len(hvdc) < n_hvdc:
        i = int(rng.integers(n_bus))
        far = np.flatnonzero(_hops(grid, i) >= 5)
        if len(far):
            hvdc.append((i, int(rng.choice(far))))
    out = np.sort(np.asarray([int(x) for x in non_bridges(grid, rng, n_out)], np.int32))
    sb = _split_buses(grid)
    lists = []
    for _ in range(n_topo):
        lists.append(sample_candidate(grid, rng, int(rng.integers(1, 4)), int(rng.integers(0, 3)),
                                      sb))
    cands = Candidates.from_lists(lists)
    loads = perturbed_injections(grid, rng, (n_comb,), 0.05)
    deg = rng.integers(-10, 11, size=(n_comb, n_pst)).astype(np.float64)
    lev = rng.integers(0, 8, size=(n_comb, n_hvdc)).astype(np.float64)
    inj = np.concatenate([loads, deg, lev], axis=1)
    mon = np.arange(grid.n_branch, dtype=np.int32)
    controls = dict(pst=pst, pst_scale=np.pi / 180.0, hvdc=hvdc, hvdc_scale=0.25)
    return Workload("brute-2000bus", grid, mon, out, cands, inj, True,
                    meta=dict(n_bus=n_bus, n_branch=n_branch, n_topo=n_topo, n_comb=n_comb,
                              n_out=n_out, n_pst=n_pst, n_hvdc=n_hvdc),
                    controls=controls)
