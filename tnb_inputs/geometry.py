"""Interaction graphs and cluster maps (king's-lattice Potts clusters).

Every graph is returned as ``(n_spins, edges)`` with ``edges`` an (E, 2) int64
array, i < j, sorted lexicographically.  A cluster map is ``(R, C, cell_of)``:
spin i belongs to lattice cell ``cell_of[i] = r * C + c``.  Couplings may only
join cells that are king's-lattice neighbours (|dr|, |dc| <= 1); that is
checked by ``validate_king``.
"""
import numpy as np


def _finish(n, pairs):
    e = np.array(sorted({(min(a, b), max(a, b)) for a, b in pairs if a != b}),
                 dtype=np.int64).reshape(-1, 2)
    return n, e


# --------------------------------------------------------------------------
# Zephyr Z(m, t): coordinates (u, w, k, j, z), u orientation, w in [0, 2m],
# k in [0, t), j in {0, 1}, z in [0, m).  Linear index as in the published
# coordinate convention: ((((u*(2m+1) + w)*t + k)*2 + j)*m + z).
# Edges: "external" (same line, z -> z+1), "odd" (j=0 at z with j=1 at z and
# z-1) and "internal" (orthogonal qubits that cross).  4tm(2m+1) spins.
# --------------------------------------------------------------------------
def zephyr_index(m, t, u, w, k, j, z):
    return (((u * (2 * m + 1) + w) * t + k) * 2 + j) * m + z


def zephyr_graph(m, t=4):
    M = 2 * m + 1
    ix = lambda u, w, k, j, z: zephyr_index(m, t, u, w, k, j, z)
    pairs = []
    for u in range(2):
        for w in range(M):
            for k in range(t):
                for j in range(2):
                    for z in range(m - 1):
                        pairs.append((ix(u, w, k, j, z), ix(u, w, k, j, z + 1)))
                for a in range(2):
                    for z in range(a, m):
                        pairs.append((ix(u, w, k, 0, z), ix(u, w, k, 1, z - a)))
    for w in range(m):
        for z in range(m):
            for h in range(t):
                for k in range(t):
                    for i in range(2):
                        for j in range(2):
                            for a in range(2):
                                for b in range(2):
                                    pairs.append((ix(0, 2 * w + 1 + a * (2 * i - 1), k, j, z),
                                                  ix(1, 2 * z + 1 + b * (2 * j - 1), h, i, w)))
    return _finish(4 * t * m * (2 * m + 1), pairs)


def zephyr_cross_cells(m, t=4):
    """Cluster map of Z(m, t) into "cross" cells on a 2m x 2m king's lattice.

    A qubit (u, w, k, j, z) lies on line w at position p = 2z + j and spans
    grid points [p, p+1] along that line.  Draw the vertical lines at x = w and
    the horizontal ones at y = w.  Cell (X, Y), for grid points with X + Y odd,
    collects the vertical qubits on x = X at positions Y-1, Y and the
    horizontal qubits on y = Y at positions X-1, X: a cross of 4t qubits.
    Crosses sit at (s, t') = ((X+Y-1)/2, (X-Y-1)/2 + m); two crosses couple
    only when they are king's-lattice neighbours there, and every pair of
    neighbouring cells shares 2t qubits per side (2^8 projections for t = 4).
    Boundary crosses are partial (2t or 3t qubits).
    """
    n = 4 * t * m * (2 * m + 1)
    cell_of = np.empty(n, dtype=np.int64)
    R = C = 2 * m
    for u in range(2):
        for w in range(2 * m + 1):
            for k in range(t):
                for j in range(2):
                    for z in range(m):
                        p = 2 * z + j
                        other = p if (w + p) % 2 == 1 else p + 1
                        X, Y = (w, other) if u == 0 else (other, w)
                        s, tt = (X + Y - 1) // 2, (X - Y - 1) // 2 + m
                        cell_of[zephyr_index(m, t, u, w, k, j, z)] = s * C + tt
    return R, C, cell_of


# --------------------------------------------------------------------------
# King's lattice of spins clustered into a x a blocks (and the plain square
# lattice with diag=False).  Spin (y, x) on an (R*a) x (C*a) grid has index
# y*(C*a) + x; cell (y // a, x // a).
# --------------------------------------------------------------------------
def king_lattice(R, C, a=1, diag=True):
    H, W = R * a, C * a
    idx = lambda y, x: y * W + x
    pairs = []
    for y in range(H):
        for x in range(W):
            if x + 1 < W:
                pairs.append((idx(y, x), idx(y, x + 1)))
            if y + 1 < H:
                pairs.append((idx(y, x), idx(y + 1, x)))
                if diag and x + 1 < W:
                    pairs.append((idx(y, x), idx(y + 1, x + 1)))
                if diag and x - 1 >= 0:
                    pairs.append((idx(y, x), idx(y + 1, x - 1)))
    n, e = _finish(H * W, pairs)
    cell_of = np.array([(y // a) * C + (x // a) for y in range(H) for x in range(W)],
                       dtype=np.int64)
    return (n, e), (R, C, cell_of)


def chain_lattice(n_spins):
    """Open chain: one spin per cell on a 1 x n lattice (a tree)."""
    pairs = [(i, i + 1) for i in range(n_spins - 1)]
    n, e = _finish(n_spins, pairs)
    return (n, e), (1, n_spins, np.arange(n_spins, dtype=np.int64))


def validate_king(edges, R, C, cell_of):
    """Return the number of edges that join cells which are not king neighbours."""
    a, b = cell_of[edges[:, 0]], cell_of[edges[:, 1]]
    ra, ca = np.divmod(a, C)
    rb, cb = np.divmod(b, C)
    return int(np.sum((np.abs(ra - rb) > 1) | (np.abs(ca - cb) > 1)))
