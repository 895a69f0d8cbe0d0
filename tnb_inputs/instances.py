"""Seeded Ising instances H(s) = sum_ij J_ij s_i s_j + sum_i h_i s_i on a
clustered graph.  Spin s = +1 is stored as bit 1 of the cluster variable."""
from dataclasses import dataclass, field
import numpy as np

from .rng import uniform01, integers
from . import geometry as G


@dataclass
class Instance:
    n_spins: int
    edges: np.ndarray          # (E, 2) int64, i < j, lexicographic
    J: np.ndarray              # (E,) float64
    h: np.ndarray              # (N,) float64
    R: int
    C: int
    cell_of: np.ndarray        # (N,) int64, r*C + c
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return self.R * self.C


# The eight symmetries of the R x C cluster lattice (Sec. V.A): the search and
# the boundary MPSs always run rows top to bottom and columns left to right,
# so relabelling the cluster positions changes the order in which the method
# meets the clusters, and with it the approximation, but not the instance.
# Transformation t = 4 f + q: q quarter turns clockwise, then a left-right
# mirror when f = 1.
N_TRANSFORMS = 8


def transform_cells(R, C, t):
    """(R', C', map) with map(r, c) -> (r', c') for transformation t (0..7)."""
    if not 0 <= t < N_TRANSFORMS:
        raise ValueError("t must be in 0..7")
    q, f = t % 4, t // 4

    def turn(r, c, R, C):            # one quarter turn clockwise
        return c, R - 1 - r, C, R
    def f_map(r, c):
        RR, CC = R, C
        for _ in range(q):
            r, c, RR, CC = turn(r, c, RR, CC)
        if f:
            c = CC - 1 - c
        return r, c
    RR, CC = (R, C) if q % 2 == 0 else (C, R)
    return RR, CC, f_map


def transform(inst, t):
    """The same instance (spins, couplings, fields) with its clusters placed by
    lattice symmetry t; t = 0 is the identity."""
    R2, C2, f = transform_cells(inst.R, inst.C, t)
    r, c = np.divmod(np.asarray(inst.cell_of, dtype=np.int64), inst.C)
    r2, c2 = f(r, c)
    cell = np.asarray(r2, dtype=np.int64) * C2 + np.asarray(c2, dtype=np.int64)
    meta = dict(inst.meta, transform=t)
    return Instance(inst.n_spins, inst.edges, inst.J, inst.h, R2, C2, cell, meta)


def random_couplings(n_edges, n_spins, seed, jdist="uniform", hdist="zero"):
    """Class I / II draws: J ~ U[-1,1] (or {+-1..+-4}/4), h ~ U[-0.1,0.1] or 0."""
    if jdist == "uniform":
        J = 2.0 * uniform01(seed, n_edges, stream=1) - 1.0
    elif jdist == "quarter":
        k = integers(seed, n_edges, 1, 8)
        mag = (k % 4 + 1).astype(np.float64) / 4.0
        J = np.where(k >= 4, mag, -mag)
    elif jdist == "zero":
        J = np.zeros(n_edges)
    else:
        raise ValueError(jdist)
    if hdist == "uniform0.1":
        h = 0.1 * (2.0 * uniform01(seed, n_spins, stream=2) - 1.0)
    elif hdist == "uniform1":
        h = 2.0 * uniform01(seed, n_spins, stream=2) - 1.0
    elif hdist == "zero":
        h = np.zeros(n_spins)
    else:
        raise ValueError(hdist)
    return J, h


def make_instance(kind, seed, jdist="uniform", hdist="zero", **kw):
    """kind: 'zephyr' (m, t), 'king' (R, C, a, diag), 'chain' (n)."""
    if kind == "zephyr":
        m, t = kw["m"], kw.get("t", 4)
        n, e = G.zephyr_graph(m, t)
        R, C, cell_of = G.zephyr_cross_cells(m, t)
    elif kind == "king":
        (n, e), (R, C, cell_of) = G.king_lattice(kw["R"], kw["C"], kw.get("a", 1),
                                                 kw.get("diag", True))
    elif kind == "chain":
        (n, e), (R, C, cell_of) = G.chain_lattice(kw["n"])
    else:
        raise ValueError(kind)
    J, h = random_couplings(len(e), n, seed, jdist, hdist)
    return Instance(n, e, J, h, R, C, cell_of, dict(kind=kind, seed=seed, **kw))


def _find_cycle(adj, start, L, rnd):
    """Randomised DFS for a simple cycle of exactly L vertices through start."""
    path, seen = [start], {start}
    def dfs(v, budget):
        if budget[0] <= 0:
            return False
        budget[0] -= 1
        nb = list(adj[v])
        order = rnd(len(nb))
        for idx in order:
            u = nb[idx]
            if len(path) == L:
                return False
            if u == start and len(path) == L:
                return True
            if u in seen:
                continue
            path.append(u); seen.add(u)
            if len(path) == L and start in adj[u]:
                return True
            if dfs(u, budget):
                return True
            path.pop(); seen.discard(u)
        return False
    return list(path) if dfs(start, [20000]) else None


def planted_loops(m, t, seed, loops_per_cell=3):
    """Tile-planted Zephyr instance: hidden s*, frustrated loops per cell.

    Each loop of L in [4, 8] spins (anchored at a spin of the cell, free to
    use edges into neighbouring cells) adds -s*_i s*_j on L-1 of its edges and
    +0.5 s*_i s*_j on one edge.  s* violates only the weak edge of each loop,
    so every loop sits at its minimum 1.5 - L and E0 = sum_l (1.5 - L_l).
    Returns (instance, s_star, E0).
    """
    n, e = G.zephyr_graph(m, t)
    R, C, cell_of = G.zephyr_cross_cells(m, t)
    return planted_on_graph(n, e, R, C, cell_of, seed, loops_per_cell,
                            dict(kind="zephyr_planted", m=m, t=t, seed=seed))


def planted_king(R, C, a, seed, loops_per_cell=2):
    """The same tile planting on a king's lattice of a x a spin blocks (the
    square / king's-lattice workload of App. B has one spin per site, a = 1).
    Returns (instance, s_star, E0)."""
    (n, e), (R2, C2, cell_of) = G.king_lattice(R, C, a, True)
    return planted_on_graph(n, e, R2, C2, cell_of, seed, loops_per_cell,
                            dict(kind="king_planted", R=R, C=C, a=a, seed=seed))


def planted_on_graph(n, e, R, C, cell_of, seed, loops_per_cell, meta):
    """Frustrated loops planted around a hidden s* (see planted_loops) on any
    clustered graph; E0 = sum over loops of (1.5 - L)."""
    s_star = np.where(integers(seed, n, 7, 2) == 1, 1, -1).astype(np.int64)
    adj = [set() for _ in range(n)]
    for a, b in e:
        adj[a].add(int(b)); adj[b].add(int(a))
    eidx = {(int(a), int(b)): k for k, (a, b) in enumerate(e)}
    J = np.zeros(len(e))
    state = [np.uint64(seed * 7919 + 13)]
    def draws(count):
        from .rng import splitmix64
        state[0] = state[0] + np.uint64(1)
        v = splitmix64(state[0] * np.uint64(1 << 20) + np.arange(count, dtype=np.uint64))
        return np.argsort(v, kind="stable")
    E0 = 0.0
    members = [[] for _ in range(R * C)]
    for i in range(n):
        members[cell_of[i]].append(i)
    for cell in range(R * C):
        if not members[cell]:
            continue
        for l in range(loops_per_cell):
            pick = integers(seed * 1009 + cell, 3, 11 + l, 1 << 30)
            start = members[cell][int(pick[0]) % len(members[cell])]
            L = 4 + int(pick[1]) % 5
            cyc = None
            for attempt in range(6):
                cyc = _find_cycle(adj, start, L, draws)
                if cyc is not None:
                    break
                L = 4 if L > 4 else L
            if cyc is None:
                continue
            weak = int(pick[2]) % L
            for q in range(L):
                a, b = cyc[q], cyc[(q + 1) % L]
                k = eidx[(min(a, b), max(a, b))]
                sgn = s_star[a] * s_star[b]
                J[k] += (0.5 * sgn) if q == weak else (-1.0 * sgn)
            E0 += 1.5 - L
    h = np.zeros(n)
    inst = Instance(n, e, J, h, R, C, cell_of, meta)
    return inst, s_star, E0
