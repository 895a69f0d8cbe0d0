"""Exact definitions on the spin level (Eq. 1, 6, 10).  Plain and slow."""
import numpy as np


def energies(inst, states):
    """Eq. (1) for each row of ``states`` (K x N, entries +-1).

    Couplings are summed one after another in the (i, j)-sorted edge order,
    then the fields in index order, each term rounded in FP64 and no fused
    multiply-add: numpy's cumsum is a plain sequential loop, so the last
    partial sum is the sequential sum.
    """
    s = np.asarray(states, dtype=np.float64)
    if s.ndim == 1:
        s = s[None, :]
    i, j = inst.edges[:, 0], inst.edges[:, 1]
    terms = np.concatenate([inst.J[None, :] * s[:, i] * s[:, j], inst.h[None, :] * s], axis=1)
    acc = np.zeros((s.shape[0], 1))
    return np.cumsum(np.concatenate([acc, terms], axis=1), axis=1)[:, -1]


def all_states(n):
    """All 2^n configurations, bit b of the row index -> spin b (bit 1 = +1)."""
    x = np.arange(1 << n, dtype=np.int64)
    return (((x[:, None] >> np.arange(n)) & 1) * 2 - 1).astype(np.int8)


def brute_force(inst, beta):
    """log Z, <s_i>, <s_i s_j> (per edge) and the minimum energy, by summing
    over all 2^N configurations (Eq. 6, 10).

    The spins are split into a low half a and a high half b, so that
    H(s) = H_a(s_a) + H_b(s_b) + s_a^T J_ab s_b and the 2^N energies form a
    2^|a| x 2^|b| matrix built with one matrix product.
    """
    n = inst.n_spins
    assert n <= 28, "brute force is for small subgraphs only"
    na = n // 2
    nb = n - na
    Sa = (((np.arange(1 << na)[:, None] >> np.arange(na)) & 1) * 2 - 1).astype(np.float64)
    Sb = (((np.arange(1 << nb)[:, None] >> np.arange(nb)) & 1) * 2 - 1).astype(np.float64)
    i, j = inst.edges[:, 0], inst.edges[:, 1]
    Ea = Sa @ inst.h[:na]
    Eb = Sb @ inst.h[na:]
    Jab = np.zeros((na, nb))
    for e, (p, q) in enumerate(zip(i, j)):
        if q < na:
            Ea = Ea + inst.J[e] * Sa[:, p] * Sa[:, q]
        elif p >= na:
            Eb = Eb + inst.J[e] * Sb[:, p - na] * Sb[:, q - na]
        else:
            Jab[p, q - na] += inst.J[e]
    E = Ea[:, None] + Eb[None, :] + (Sa @ Jab) @ Sb.T
    E_min = E.min()
    W = np.exp(-beta * (E - E_min))
    Z = W.sum()
    wa, wb = W.sum(axis=1), W.sum(axis=0)
    m1 = np.concatenate([wa @ Sa, wb @ Sb]) / Z
    cross = Sa.T @ W @ Sb                       # sum_s w(s) s_p s_q, p in a, q in b
    m2 = np.empty(len(inst.J))
    for e, (p, q) in enumerate(zip(i, j)):
        if q < na:
            m2[e] = wa @ (Sa[:, p] * Sa[:, q])
        elif p >= na:
            m2[e] = wb @ (Sb[:, p - na] * Sb[:, q - na])
        else:
            m2[e] = cross[p, q - na]
    m2 /= Z
    ia, ib = np.nonzero(np.abs(E - E_min) <= 1e-9 * max(1.0, abs(E_min)))
    ground = np.sort(ia.astype(np.int64) + (ib.astype(np.int64) << na))
    return dict(logZ=np.log(Z) - beta * E_min, m1=m1, m2=m2, E_min=E_min, ground=ground)


def logz_field_only(h, beta):
    """J = 0: log Z = sum_i log(2 cosh(beta h_i))."""
    return float(np.sum(np.log(2.0 * np.cosh(beta * np.asarray(h)))))


def logz_tree(J, n, beta):
    """Tree with h = 0: Z = 2^N prod_e cosh(beta J_e)."""
    return float(n * np.log(2.0) + np.sum(np.log(np.cosh(beta * np.asarray(J)))))
