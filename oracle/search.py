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


def solve(inst, beta, env, M, K=8, merge=True, trace=False, droplets=None):
    """Full search; returns dict with the K lowest states and diagnostics.
    droplets: a droplets.DropletOptions to keep the excitations found by the
    merge (Fig. 4) with every branch; they are returned per output state."""
    from . import droplets as dl
    net = env.net
    R, C = net.R, net.C
    ncell = R * C
    bonds = dl.cluster_bonds(net.P) if droplets is not None else None
    drop = [[]]
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
            # merge by boundary (Eq. 8) while some fixed cluster still couples
            # to an unfixed one; with an empty boundary (the last step, or only
            # uncoupled clusters left) every candidate is kept (R12)
            masks = boundary_key_masks(net, n + 1)
            if merge and masks:
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
            if droplets is not None:
                if merge and masks:
                    drop = dl.merge_step(inst, net.P, bonds, droplets, X, drop, n, bb, xx, sc, keys, keep)
                else:
                    drop = [list(drop[bb[i]]) for i in keep]
            rec = dict(n=n, candidates=len(bb), groups=len(win), kept=len(keep))
            if trace:
                # selection margins (R7, R10): the score gap between the last
                # kept group and the first dropped one, and the smallest gap
                # between a group's winner and its runner-up
                rec["boundary_gap"] = sc[win[M - 1]] - sc[win[M]] if len(win) > M else np.inf
                if merge and masks and len(bb) > len(win):
                    ordk = np.lexsort((-sc,) + tuple(keys[:, i] for i in range(keys.shape[1] - 1, -1, -1)))
                    ks, ss = keys[ordk], sc[ordk]
                    same = np.all(ks[1:] == ks[:-1], axis=1)
                    head = same & np.r_[True, ~same[:-1]]      # winner and runner-up of a group
                    rec["group_gap"] = float(np.min((ss[:-1] - ss[1:])[head])) if head.any() else np.inf
                else:
                    rec["group_gap"] = np.inf
                rec["p"] = np.where(alive[:, None], qpos / np.where(alive, Zb, 1.0)[:, None], 0.0)
                rec["X"] = X[bb[keep]].copy()
                rec["X"][:, n] = xx[keep]
                rec["logp"] = sc[keep].copy()
                rec["p_d_log"] = pd_log
                if droplets is not None:
                    rec["droplets"] = [list(d) for d in drop]
            steps.append(rec)
            Xn = X[bb[keep]].copy()
            Xn[:, n] = xx[keep]
            Ln = vec[bb[keep], xx[keep]]
            nrm = np.abs(Ln).max(axis=1, keepdims=True)
            Ln = Ln / np.where(nrm > 0, nrm, 1.0)
            if trace:
                rec["L"] = Ln.copy()
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
    res = dict(states=states[out], energies=E[out], logp=logp[out], X=X[out],
               p_d_log=pd_log, steps=steps, all_states=states, all_logp=logp)
    if droplets is not None:
        res["droplets"] = [drop[i] for i in out]
        res["all_droplets"] = drop
    return res


def root_marginal_check(net, env):
    """Sum over x of q at the first step; equals Z / exp(shift + lam_1) up to the
    normalisation of R (used by tests as a consistency identity)."""
    X = np.zeros((1, net.R * net.C), dtype=np.int64)
    Rrow = right_envs(net, env, 0, X)
    q, _ = marginals(net, env, 0, 0, X, np.ones((1, 1)), Rrow[0])
    return q


def _row_contract(net, env, r, c, xb, lvec, clamp):
    """Contract the free clusters c..C-1 of row r with Psi_{r+1} for one parent.

    xb: the parent's cluster values (row r-1 and row-r columns < c fixed);
    lvec: its left vector (over the bond left of Psi site 2c-1); clamp:
    {cell: allowed boolean mask over x} restricting free clusters.  Returns
    (sign, log|Z|).  Plain left-to-right transfer over the full configuration
    of the previous cluster.
    """
    psi, cols = _row_data(net, env, r)
    C = net.C
    logs = 0.0
    # state: S[beta, x_prev] with x_prev the previous cluster's full value
    if c == 0:
        S = np.ones((1, 1))
        prev_vals = np.zeros(1, dtype=np.int64)
    else:
        S = lvec.reshape(-1, 1)
        prev_vals = np.array([xb[net.cell(r, c - 1)]], dtype=np.int64)
    for cc in range(c, C):
        d = cols[cc]
        n = d["n"]
        x = d["x"]
        g = d["w"] * _phi(net, r, cc, xb[None, :])[0]
        if n in clamp:
            g = g * clamp[n]
        A2c = psi[2 * cc]
        newS = np.zeros((A2c.shape[2], len(x)))
        if cc == 0:
            vec = A2c[0][d["vd"], :]                                      # (x, D)
            newS = (g[:, None] * vec).T
        else:
            nl = net.cell(r, cc - 1)
            A2m = psi[2 * cc - 1]
            Wh = net.Wt(nl, n)
            for ip, xp in enumerate(prev_vals):
                if not np.any(S[:, ip]):
                    continue
                ap = pext(np.array([xp]), net.B(nl, net.cell(r + 1, cc)))[0]
                hp = pext(np.array([xp]), net.B(nl, n))[0]
                sig = ap + d["da2"] * d["bd"]                                # (x,)
                T = np.einsum("a,xag->xg", S[:, ip], np.transpose(A2m[:, sig, :], (1, 0, 2)))
                vec = np.einsum("xg,gxe->xe", T, A2c[:, d["vd"], :])
                newS += (g * Wh[hp, d["xh"]])[None, :] * vec.T
        mx = np.abs(newS).max()
        if mx == 0:
            return 0.0, -np.inf
        S = newS / mx
        logs += np.log(mx)
        prev_vals = x
    tot = S.sum()
    return (1.0 if tot > 0 else -1.0), logs + np.log(abs(tot))


def row_spins_edges(net, r, c):
    """Spins of the unfixed clusters c..C-1 of row r (cluster by cluster,
    ascending) and the couplings with both ends in one of those clusters."""
    P = net.P
    spins, edges = [], []
    for cc in range(c, net.C):
        n = net.cell(r, cc)
        spins.extend(P.spins[n].tolist())
        edges.extend(P.intra[n])
    return np.array(spins, dtype=np.int64), np.array(edges, dtype=np.int64)


def row_moments(net, env, r, c, Xpar, L):
    """<s_i>_b and <s_i s_j>_b over the unfixed clusters c..C-1 of row r, for
    every parent b (rows of Xpar, left vectors L), with Psi_{r+1} fixed.

    Definition by clamping: <s_i>_b = (Z_b(s_i=+1) - Z_b(s_i=-1)) / Z_b and
    <s_i s_j>_b = (Z_b(s_i s_j=+1) - Z_b(s_i s_j=-1)) / Z_b, every Z_b a full
    contraction of the conditioned network of Fig. 6(b) (Eq. 10).  These are
    -1/beta d log Z_b / d h_i and -1/beta d log Z_b / d J_ij.  The values are
    signed ratios of the approximate contraction: no clipping is applied, so
    they are exact derivatives of log|Z_b| even where the approximate
    environment produces negative terms.  Returns (m1 [npar, spins],
    m2 [npar, edges], spins, edges).
    """
    P = net.P
    inst = P.inst
    spins, edges = row_spins_edges(net, r, c)
    m1 = np.zeros((Xpar.shape[0], len(spins)))
    m2 = np.zeros((Xpar.shape[0], len(edges)))

    def ratio(b, clamps):
        vals = []
        for cl in clamps:
            sg, lz = _row_contract(net, env, r, c, Xpar[b], L[b], cl)
            vals.append((sg, lz))
        return vals

    for b in range(Xpar.shape[0]):
        for col, i in enumerate(spins):
            n = int(net.P.inst.cell_of[i])
            x = np.arange(1 << int(P.k[n]))
            up = ((x >> P.bit[i]) & 1).astype(float)
            (sp, lp), (sm, lm) = ratio(b, [{n: up}, {n: 1.0 - up}])
            top = max(lp, lm)
            zp = sp * np.exp(lp - top) if np.isfinite(lp) else 0.0
            zm = sm * np.exp(lm - top) if np.isfinite(lm) else 0.0
            m1[b, col] = (zp - zm) / (zp + zm)
        for col, e in enumerate(edges):
            i, j = inst.edges[e]
            n = int(inst.cell_of[i])
            x = np.arange(1 << int(P.k[n]))
            par = (((x >> P.bit[i]) ^ (x >> P.bit[j])) & 1) == 0
            (sp, lp), (sm, lm) = ratio(b, [{n: par.astype(float)}, {n: (~par).astype(float)}])
            top = max(lp, lm)
            zp = sp * np.exp(lp - top) if np.isfinite(lp) else 0.0
            zm = sm * np.exp(lm - top) if np.isfinite(lm) else 0.0
            m2[b, col] = (zp - zm) / (zp + zm)
    return m1, m2, spins, edges


def row_logz(net, env, r, c, xb, lvec):
    """log|Z_b| of the conditioned row network including the local log-scales
    of the unfixed clusters (the -beta * min E_n of Eq. 6), so that finite
    differences in h or J of a row-r spin are taken on the true log Z_b up
    to terms that do not depend on them."""
    sg, lz = _row_contract(net, env, r, c, xb, lvec, {})
    for cc in range(c, net.C):
        lz += -net.beta * net.P.local_energy(net.cell(r, cc)).min()
    return lz
