"""Branch and bound over cluster variables with boundary merging (Sec. III.A).

Clusters are visited row after row, left to right (R2).  For a partial
configuration (parent) b at step n+1 = (r, c) the conditional marginal
p(x_{r,c} | boundary of b) comes from the exact contraction of the network of
Fig. 6(b): rows above r and row-r columns < c fixed to b, cluster (r,c) open,
row-r columns > c summed, and the boundary MPS Psi_{r+1} below.  Because
row r-1 is fixed for the whole of row r, the couplings to it are local
weights phi_b on row r, and the contraction of columns > c is a right
environment R_b^{(c)} computed once per parent at the start of the row.
"""
import numpy as np

from .potts import pext, popcount
from .bmps import sub, _segment_sum
from .ising import energies


class RowEnv:
    """Right environments R^{(c)}[beta, pi_c] of row r for one parent."""


def _row_data(net, env, r):
    C = net.C
    psi = env.psi[r + 1]
    cols = []
    for c in range(C):
        n = net.cell(r, c)
        k = int(net.P.k[n])
        x = np.arange(1 << k, dtype=np.int64)
        PRR = net.B(n, net.cell(r, c + 1)) | net.B(n, net.cell(r + 1, c + 1))
        d = dict(n=n, x=x, w=net.w[n], PRR=PRR, pi=pext(x, PRR),
                 vd=pext(x, net.B(n, net.cell(r + 1, c))))
        if c > 0:
            nl = net.cell(r, c - 1)
            d["xh"] = pext(x, net.B(n, nl))                       # spins facing (r, c-1)
            d["bd"] = pext(x, net.B(n, net.cell(r + 1, c - 1)))   # Psi site 2c-1, b'
            d["dxh"] = 1 << popcount(net.B(n, nl))
            d["dbd"] = 1 << popcount(net.B(n, net.cell(r + 1, c - 1)))
            d["da2"] = 1 << popcount(net.B(nl, net.cell(r + 1, c)))
        cols.append(d)
    return psi, cols


def _phi(net, r, c, X):
    """phi_b(c, x) for every parent row of X (n_par x n_cells) and every x."""
    n = net.cell(r, c)
    k = int(net.P.k[n])
    x = np.arange(1 << k, dtype=np.int64)
    out = np.ones((X.shape[0], 1 << k))
    for dc in (-1, 0, 1):
        up = net.cell(r - 1, c + dc)
        if up < 0 or net.B(n, up) == 0:
            continue
        W = net.Wt(up, n)
        out = out * W[pext(X[:, up], net.B(up, n))[:, None], pext(x, net.B(n, up))[None, :]]
    return out


def right_envs(net, env, r, Xpar):
    """R_b^{(c)} for c = 0..C-1 and every parent (rows of Xpar)."""
    C = net.C
    psi, cols = _row_data(net, env, r)
    npar = Xpar.shape[0]
    R = [None] * C
    R[C - 1] = np.ones((npar, 1, 1))
    for c in range(C - 1, 0, -1):
        d, dl = cols[c], cols[c - 1]
        A2c, A2cm1 = psi[2 * c], psi[2 * c - 1]
        g = d["w"][None, :] * _phi(net, r, c, Xpar)                   # (npar, x)
        Rc = R[c]
        out = np.zeros((npar, A2cm1.shape[0], 1 << popcount(dl["PRR"])))
        pi_prev = np.arange(1 << popcount(dl["PRR"]))
        nl, n = dl["n"], d["n"]
        hpart = sub(pi_prev, dl["PRR"], net.B(nl, n))
        apart = sub(pi_prev, dl["PRR"], net.B(nl, net.cell(r + 1, c)))
        Wh = net.Wt(nl, n)[hpart]                                     # (pi, xh)
        grp = d["xh"] * d["dbd"] + d["bd"]
        for b in range(npar):
            u = np.einsum("gxe,xe->xg", A2c[:, d["vd"], :], Rc[b][:, d["pi"]].T)
            U = _segment_sum(g[b][:, None] * u, grp, d["dxh"] * d["dbd"])
            U = U.reshape(d["dxh"], d["dbd"], -1)                      # (xh, b', gamma)
            A4 = A2cm1.reshape(A2cm1.shape[0], d["dbd"], d["da2"], A2cm1.shape[2])  # (beta, b', a', gamma)
            V = np.einsum("pbag,hbg->ahp", A4, U)                       # (a', xh, beta)
            val = np.einsum("ih,ihp->pi", Wh, V[apart])
            mx = np.abs(val).max()
            out[b] = val / mx if mx > 0 else val
        R[c - 1] = out
    return R


def marginals(net, env, r, c, Xpar, L, Rrow):
    """q_b[x] (unnormalised) and the new left vectors for every (b, x).

    Xpar: parents' cluster values; L: left vectors (over the bond left of
    Psi site 2c-1, or of site 0 when c = 0); Rrow: R^{(c)} per parent.
    Returns q (npar, d) and vec (npar, d, D) = left vector after fixing x.
    """
    psi, cols = _row_data(net, env, r)
    d = cols[c]
    A2c = psi[2 * c]
    npar = Xpar.shape[0]
    g = d["w"][None, :] * _phi(net, r, c, Xpar)
    if c == 0:
        vec = np.broadcast_to(A2c[0][d["vd"], :], (npar,) + A2c[0][d["vd"], :].shape).copy()
    else:
        nl = net.cell(r, c - 1)
        A2cm1 = psi[2 * c - 1]
        a_fix = pext(Xpar[:, nl], net.B(nl, net.cell(r + 1, c)))
        sig = a_fix[:, None] + d["da2"] * d["bd"][None, :]              # (npar, x)
        T = np.einsum("pa,pxag->pxg", L, np.transpose(A2cm1[:, sig, :], (1, 2, 0, 3)))
        vec = np.einsum("pxg,gxe->pxe", T, A2c[:, d["vd"], :])
        Whf = net.Wt(nl, d["n"])[pext(Xpar[:, nl], net.B(nl, d["n"]))[:, None], d["xh"][None, :]]
        g = g * Whf
    q = g * np.einsum("pxe,pex->px", vec, Rrow[:, :, d["pi"]])
    return q, vec


def boundary_key_masks(net, n_fixed):
    """(cell, union mask) for fixed cells with an unfixed king neighbour.
    Cells are fixed in row-major order; the first n_fixed are fixed."""
    from .potts import king_neighbours
    out = []
    for k in range(n_fixed):
        U = 0
        for l in king_neighbours(net.R, net.C, k):
            if l >= n_fixed:
                U |= net.B(k, l)
        if U:
            out.append((k, U))
    return out


def solve(inst, beta, env, M, K=8, merge=True, trace=False):
    """Full search; returns dict with the K lowest states and diagnostics."""
    net = env.net
    R, C = net.R, net.C
    ncell = R * C
    X = np.zeros((1, ncell), dtype=np.int64)
    logp = np.zeros(1)
    L = np.ones((1, 1))
    pd_log = -np.inf
    steps = []
    Rrow = None
    for r in range(R):
        Rrow = right_envs(net, env, r, X)
        rid = np.arange(X.shape[0])
        for c in range(C):
            n = r * C + c
            last = (n == ncell - 1)
            q, vec = marginals(net, env, r, c, X, L, Rrow[c][rid])
            # Eq. (9) is a ratio of two contractions of the same network, so a
            # common sign of the approximate environment cancels: entries are
            # taken with the sign of their sum, and those left non-positive get
            # probability 0 (R9).
            sgn = np.where(q.sum(axis=1, keepdims=True) < 0, -1.0, 1.0)
            qpos = np.where(q * sgn > 0, q * sgn, 0.0)
            Zb = qpos.sum(axis=1)
            alive = Zb > 0
            with np.errstate(divide="ignore"):
                lp = np.where(qpos > 0, np.log(qpos) - np.log(np.where(alive, Zb, 1.0))[:, None], -np.inf)
            score = logp[:, None] + lp
            score[~alive] = -np.inf
            npar, d = score.shape
            bb, xx = np.meshgrid(np.arange(npar), np.arange(d), indexing="ij")
            bb, xx, sc = bb.ravel(), xx.ravel(), score.ravel()
            ok = np.isfinite(sc)
            bb, xx, sc = bb[ok], xx[ok], sc[ok]
            if merge and not last:
                masks = boundary_key_masks(net, n + 1)
                keycols = []
                for (k, U) in masks:
                    vals = xx if k == n else X[bb, k]
                    keycols.append(pext(vals, U))
                keys = np.stack(keycols, axis=1) if keycols else np.zeros((len(bb), 0), dtype=np.int64)
                # group winners: best score, ties -> smaller (b, x)
                order = np.lexsort((xx, bb, -sc))
                _, first = np.unique(keys[order], axis=0, return_index=True)
                win = order[np.sort(first)]
                # np.unique sorts by key; re-rank winners by score then (b, x)
                win = win[np.lexsort((xx[win], bb[win], -sc[win]))]
            else:
                win = np.lexsort((xx, bb, -sc))
            keep = win[:M]
            if len(win) > M:
                pd_log = max(pd_log, sc[win[M]])
            rec = dict(n=n, candidates=len(bb), groups=len(win), kept=len(keep))
            if trace:
                rec["p"] = np.where(alive[:, None], qpos / np.where(alive, Zb, 1.0)[:, None], 0.0)
                rec["X"] = X[bb[keep]].copy()
                rec["X"][:, n] = xx[keep]
                rec["logp"] = sc[keep].copy()
                rec["p_d_log"] = pd_log
            steps.append(rec)
            Xn = X[bb[keep]].copy()
            Xn[:, n] = xx[keep]
            Ln = vec[bb[keep], xx[keep]]
            nrm = np.abs(Ln).max(axis=1, keepdims=True)
            Ln = Ln / np.where(nrm > 0, nrm, 1.0)
            rid = rid[bb[keep]]
            X, logp, L = Xn, sc[keep], Ln
    states = net.P.states_of_clusters(X)
    E = energies(inst, states)
    order = np.lexsort(tuple(states[:, ::-1].T) + (E,))
    seen, out = set(), []
    for i in order:
        key = states[i].tobytes()
        if key in seen:
            continue
        seen.add(key)
        out.append(i)
        if len(out) == K:
            break
    out = np.array(out, dtype=np.int64)
    return dict(states=states[out], energies=E[out], logp=logp[out], X=X[out],
                p_d_log=pd_log, steps=steps, all_states=states, all_logp=logp)


def root_marginal_check(net, env):
    """Sum over x of q at the first step; equals Z / exp(shift + lam_1) up to the
    normalisation of R (used by tests as a consistency identity)."""
    X = np.zeros((1, net.R * net.C), dtype=np.int64)
    Rrow = right_envs(net, env, 0, X)
    q, _ = marginals(net, env, 0, 0, X, np.ones((1, 1)), Rrow[0])
    return q
