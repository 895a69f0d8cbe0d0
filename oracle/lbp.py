"""Local dimensional reduction by loopy belief propagation (Sec. IV, Fig. 9).

Messages live on projected cluster states (Eq. 4): nu[m -> n] is a function
of xbar_n = P^{nm} x_n, the spins of n coupled to m.  One iteration updates
every directed bond from the messages of the previous one (synchronous):

  mu[m -> n](xbar_m) = sum_{x_m : P^{mn} x_m = xbar_m} w_m(x_m)
                       prod_{m' in N(m), m' != n} nu[m' -> m](P^{mm'} x_m)
  nu[m -> n](xbar_n) = sum_{xbar_m} W_mn(xbar_m, xbar_n) mu[m -> n](xbar_m)

with w_m and W_mn the Boltzmann tables of Eq. (6) (shifted by their minima,
which the normalisation removes) and every new message normalised to sum 1.
Messages start uniform.  The cluster beliefs are

  p_n(x) ~ w_n(x) prod_{m in N(n)} nu[m -> n](P^{nm} x)

normalised over x, and the reduction keeps the `keep` most probable states
of each cluster (ties: the smaller x).  N(m): king neighbours coupled to m.

Parity pinned by: exact marginals (brute force) on cluster trees, uniform
beliefs at beta = 0, the local Boltzmann distribution of an uncoupled cluster,
and the fixed point of a converged tree (tests/test_oracle_lbp.py).
"""
import numpy as np

from .bmps import Network
from .potts import pext, popcount, king_neighbours


def _neighbours(net, n):
    R, C = net.R, net.C
    return [m for m in king_neighbours(R, C, n) if net.B(n, m)]


def lbp(inst, beta, iters, net=None):
    """(beliefs per cluster, messages, largest change in the last iteration)."""
    net = net if net is not None else Network(inst, beta)
    ncell = net.R * net.C
    nbrs = [_neighbours(net, n) for n in range(ncell)]
    k = net.P.k
    nu = {}
    for m in range(ncell):
        for n in nbrs[m]:
            d = 1 << popcount(net.B(n, m))
            nu[(m, n)] = np.full(d, 1.0 / d)
    change = 0.0
    for _ in range(iters):
        new = {}
        for (m, n), old in nu.items():
            x = np.arange(1 << int(k[m]), dtype=np.int64)
            g = net.w[m].copy()
            for mp in nbrs[m]:
                if mp != n:
                    g = g * nu[(mp, m)][pext(x, net.B(m, mp))]
            dm = 1 << popcount(net.B(m, n))
            mu = np.zeros(dm)
            np.add.at(mu, pext(x, net.B(m, n)), g)
            v = net.Wt(m, n).T @ mu                 # W(xbar_m, xbar_n) summed over xbar_m
            s = v.sum()
            new[(m, n)] = v / s if s > 0 else np.full(len(v), 1.0 / len(v))
        change = max([np.abs(new[e] - nu[e]).max() for e in nu], default=0.0)
        nu = new
    beliefs = []
    for n in range(ncell):
        x = np.arange(1 << int(k[n]), dtype=np.int64)
        p = net.w[n].copy()
        for m in nbrs[n]:
            p = p * nu[(m, n)][pext(x, net.B(n, m))]
        beliefs.append(p / p.sum())
    return beliefs, nu, change


def select(beliefs, keep):
    """Boolean mask per cluster: its `keep` most probable states (ties by x)."""
    out = []
    for p in beliefs:
        order = np.lexsort((np.arange(len(p)), -p))
        m = np.zeros(len(p), dtype=bool)
        m[order[:keep]] = True
        out.append(m)
    return out


def exact_marginals(inst, beta, P):
    """Brute-force cluster marginals p_n(x) from Eq. (6) (small instances)."""
    from .ising import all_states, energies
    s = all_states(inst.n_spins)
    E = energies(inst, s)
    w = np.exp(-beta * (E - E.min()))
    X = P.cluster_of_states(s)
    out = []
    for n in range(P.R * P.C):
        p = np.zeros(1 << int(P.k[n]))
        np.add.at(p, X[:, n], w)
        out.append(p / p.sum())
    return out
