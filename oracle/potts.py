"""Clustered (generalised Potts) form of the Ising problem, Eq. (3)-(5).

Cluster n holds the spins with cell_of == n in ascending global index; bit b
of the cluster variable x_n is spin b of the cluster, bit 1 meaning s = +1.
For neighbouring clusters m, n the projector P^{mn} keeps the spins of m that
have a coupling into n (bit mask B[m, n]); the compressed bond energy
Ebar^{mn}[P^{mn} x_m, P^{nm} x_n] equals the sum of J_ij s_i s_j over the
edges between the two clusters (Eq. 4-5).
"""
import numpy as np


def pext(x, mask):
    """Gather the bits of x selected by mask into the low bits (ascending)."""
    x = np.asarray(x, dtype=np.int64)
    out = np.zeros_like(x)
    j = 0
    b = 0
    m = int(mask)
    while m:
        if m & 1:
            out |= ((x >> b) & 1) << j
            j += 1
        m >>= 1
        b += 1
    return out


def pdep(y, mask):
    """Scatter the low bits of y to the positions set in mask (inverse of pext)."""
    y = np.asarray(y, dtype=np.int64)
    out = np.zeros_like(y)
    j = 0
    b = 0
    m = int(mask)
    while m:
        if m & 1:
            out |= ((y >> j) & 1) << b
            j += 1
        m >>= 1
        b += 1
    return out


def popcount(mask):
    return bin(int(mask)).count("1")


def king_neighbours(R, C, n):
    r, c = divmod(n, C)
    out = []
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if (dr or dc) and 0 <= r + dr < R and 0 <= c + dc < C:
                out.append((r + dr) * C + (c + dc))
    return out


class Potts:
    """Cluster tables of one instance (no inverse temperature involved)."""

    def __init__(self, inst):
        self.inst = inst
        R, C = inst.R, inst.C
        self.R, self.C = R, C
        co = np.asarray(inst.cell_of)
        self.spins = [np.flatnonzero(co == n) for n in range(R * C)]
        self.k = np.array([len(s) for s in self.spins], dtype=np.int64)
        self.bit = np.empty(inst.n_spins, dtype=np.int64)
        for s in self.spins:
            self.bit[s] = np.arange(len(s))
        a, b = co[inst.edges[:, 0]], co[inst.edges[:, 1]]
        ra, ca = np.divmod(a, C)
        rb, cb = np.divmod(b, C)
        if np.any((np.abs(ra - rb) > 1) | (np.abs(ca - cb) > 1)):
            raise ValueError("an edge joins clusters that are not king's-lattice neighbours")
        self.intra = [[] for _ in range(R * C)]     # per cluster: edge ids
        self.inter = {}                              # (m, n), m < n: edge ids
        for e, (p, q) in enumerate(zip(a, b)):
            if p == q:
                self.intra[p].append(e)
            else:
                key = (min(p, q), max(p, q))
                self.inter.setdefault(key, []).append(e)
        self.mask = {}
        for (m, n), es in self.inter.items():
            bm, bn = 0, 0
            for e in es:
                i, j = inst.edges[e]
                if co[i] == m:
                    bm |= 1 << int(self.bit[i]); bn |= 1 << int(self.bit[j])
                else:
                    bm |= 1 << int(self.bit[j]); bn |= 1 << int(self.bit[i])
            self.mask[(m, n)] = bm
            self.mask[(n, m)] = bn

    def B(self, m, n):
        """Bit mask of the spins of cluster m coupled to cluster n (0 if none)."""
        if m < 0 or n < 0:
            return 0
        return self.mask.get((m, n), 0)

    def local_energy(self, n):
        """E_n[x] for all x in [0, 2^k_n): intra-cluster couplings, then fields."""
        k = int(self.k[n])
        x = np.arange(1 << k, dtype=np.int64)
        E = np.zeros(1 << k)
        inst = self.inst
        for e in self.intra[n]:
            i, j = inst.edges[e]
            si = ((x >> self.bit[i]) & 1) * 2 - 1
            sj = ((x >> self.bit[j]) & 1) * 2 - 1
            E = E + inst.J[e] * (si * sj)
        for i in self.spins[n]:
            E = E + inst.h[i] * (((x >> self.bit[i]) & 1) * 2 - 1)
        return E

    def bond_energy(self, m, n):
        """Ebar^{mn}[p, q], p = P^{mn} x_m, q = P^{nm} x_n (Eq. 4-5)."""
        bm, bn = self.B(m, n), self.B(n, m)
        dm, dn = 1 << popcount(bm), 1 << popcount(bn)
        p = np.arange(dm)[:, None]
        q = np.arange(dn)[None, :]
        xm, xn = pdep(p, bm), pdep(q, bn)
        E = np.zeros((dm, dn))
        key = (min(m, n), max(m, n))
        inst = self.inst
        for e in self.inter.get(key, []):
            i, j = inst.edges[e]
            if inst.cell_of[i] != m:
                i, j = j, i
            si = ((xm >> self.bit[i]) & 1) * 2 - 1
            sj = ((xn >> self.bit[j]) & 1) * 2 - 1
            E = E + inst.J[e] * (si * sj)
        return E

    def cluster_of_states(self, states):
        """Spin states (K x N, +-1) -> cluster variables (K x n_cells)."""
        s = np.asarray(states)
        X = np.zeros((s.shape[0], self.R * self.C), dtype=np.int64)
        for n, sp in enumerate(self.spins):
            for b, i in enumerate(sp):
                X[:, n] |= (s[:, i] > 0).astype(np.int64) << b
        return X

    def states_of_clusters(self, X):
        X = np.asarray(X, dtype=np.int64)
        s = np.empty((X.shape[0], self.inst.n_spins), dtype=np.int8)
        for n, sp in enumerate(self.spins):
            for b, i in enumerate(sp):
                s[:, i] = ((X[:, n] >> b) & 1) * 2 - 1
        return s
