"""Excitations (spin-glass droplets) from the boundary merge (Sec. III.A, Fig. 4).

When the branch step groups candidate partial configurations by their
boundary, the most probable one of a group becomes the main branch and every
other member differs from it only away from the boundary: that difference is
a low-energy excitation above the main branch.  The main branch keeps its
own excitations, gains the differences of the group's other members, and
takes over their excitations too (expressed relative to itself).

A droplet is stored as a flip set F, a sorted tuple of (cluster, XOR mask of
the cluster's spins) with non-zero masks, together with its energy
dE = E(main branch with F flipped) - E(main branch) of Eq. (1).  Because the
flipped spins never couple to an unfixed cluster, dE does not change as the
branch grows, and for an excitation F_d of a merged member m (itself
m = w + F_m) the flip set relative to w is F_m xor F_d with energy
dE_m + dE_d exactly (the two differences telescope).

Which excitations are kept (the paper leaves the bookkeeping open; these are
the readings the GPU path implements too):
  * the group's members are ranked by score (then parent, then cluster value)
    and the first ``max_losers`` contribute;
  * a flip set is kept when it is non-empty, touches at most ``max_cells``
    clusters, has dE <= ``max_dE`` and (``connected_only``) its clusters form
    one connected set of the cluster bond graph (clusters joined by at least
    one coupling);
  * candidates are visited by increasing dE, ties by the flip set compared as
    a sequence of (cluster, mask) pairs, and accepted while their Hamming
    distance (spins flipped in one and not the other) to every accepted one
    is at least ``min_hamming``, up to ``max_droplets``.

Parity pinned by: dE against Eq. (1) on the completed states (exact with
quarter-integer couplings); with every limit lifted and an exact search that
keeps all groups, the final states and their droplet states partition the
configuration space (each configuration appears exactly once), checked by
enumeration; connectivity, Hamming distances and the bound on the count; and
a hand-worked chain.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class DropletOptions:
    max_droplets: int = 16
    max_losers: int = 8
    min_hamming: int = 1
    max_cells: int = 64
    max_dE: float = np.inf
    connected_only: bool = True


def fixed_energy(inst, cell_of, state, n_fixed):
    """Eq. (1) restricted to the spins of clusters 0 .. n_fixed-1: every
    coupling with both ends fixed, then every fixed spin's field, summed in
    edge order and spin order."""
    fixed = np.asarray(cell_of) < n_fixed
    e = 0.0
    for k, (i, j) in enumerate(inst.edges):
        if fixed[i] and fixed[j]:
            e += inst.J[k] * float(state[i]) * float(state[j])
    for i in range(inst.n_spins):
        if fixed[i]:
            e += inst.h[i] * float(state[i])
    return e


def flip_between(xa, xb, n_fixed):
    """Flip set taking cluster configuration xb to xa over clusters < n_fixed."""
    return tuple((k, int(xa[k]) ^ int(xb[k])) for k in range(n_fixed) if int(xa[k]) != int(xb[k]))


def compose(fa, fb):
    """F_a xor F_b (cluster-wise), zero masks dropped."""
    d = dict(fa)
    for k, m in fb:
        d[k] = d.get(k, 0) ^ m
    return tuple(sorted((k, m) for k, m in d.items() if m))


def hamming(fa, fb):
    return sum(bin(m).count("1") for _, m in compose(fa, fb))


def connected(flip, bonds):
    """One connected set of clusters in the bond graph (bonds: set of (m, n))."""
    cells = [k for k, _ in flip]
    if not cells:
        return False
    seen, todo = {cells[0]}, [cells[0]]
    rest = set(cells)
    while todo:
        a = todo.pop()
        for b in rest:
            if b not in seen and ((min(a, b), max(a, b)) in bonds):
                seen.add(b)
                todo.append(b)
    return len(seen) == len(cells)


def cluster_bonds(P):
    """Pairs (m, n), m < n, of clusters joined by at least one coupling."""
    return set(P.inter.keys())


def select(cands, opts, bonds):
    """Filter and greedy selection of (flip, dE) candidates (module docstring)."""
    ok = [(f, e) for f, e in cands
          if f and len(f) <= opts.max_cells and e <= opts.max_dE
          and (not opts.connected_only or connected(f, bonds))]
    ok.sort(key=lambda c: (c[1], c[0]))
    kept = []
    for f, e in ok:
        if len(kept) == opts.max_droplets:
            break
        if all(hamming(f, g) >= opts.min_hamming for g, _ in kept):
            kept.append((f, e))
    return kept


def merge_step(inst, P, bonds, opts, X, drop, n, bb, xx, sc, keys, keep):
    """Droplets of the kept main branches after the merge at step n.

    X: parent cluster configurations; drop: parent droplet lists; (bb, xx, sc):
    every candidate's parent, value of cluster n and score; keys: their
    boundary keys (rows); keep: indices (into the candidates) of the kept
    group winners.  Returns one droplet list per kept winner."""
    out = []
    nf = n + 1
    kb = [k.tobytes() for k in keys]
    for w in keep:
        xw = X[bb[w]].copy()
        xw[n] = xx[w]
        members = [i for i in range(len(bb)) if kb[i] == kb[w] and i != w]
        members.sort(key=lambda i: (-sc[i], bb[i], xx[i]))
        members = members[:opts.max_losers]
        sw = P.states_of_clusters(xw[None, :])[0]
        ew = fixed_energy(inst, inst.cell_of, sw, nf)
        cands = list(drop[bb[w]])
        for i in members:
            xl = X[bb[i]].copy()
            xl[n] = xx[i]
            fl = flip_between(xl, xw, nf)
            sl = P.states_of_clusters(xl[None, :])[0]
            el = fixed_energy(inst, inst.cell_of, sl, nf) - ew
            cands.append((fl, el))
            for fd, ed in drop[bb[i]]:
                cands.append((compose(fl, fd), el + ed))
        out.append(select(cands, opts, bonds))
    return out


def apply_flip(x, flip):
    y = np.array(x, copy=True)
    for k, m in flip:
        y[k] ^= m
    return y
