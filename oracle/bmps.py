"""Boundary-MPS approximation of the lower half of the PEPS (Sec. III.B).

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke run
and the CPU-baseline leg of the benchmark use this module.

Tensor network (one fixed decomposition; the paper's Fig. 5 and A6 are not
recoverable).  The boundary MPS Psi_r stands for all rows >= r as a function
of the configuration of row r-1 and has 2C-1 sites:
  site 2c   : v_c = P^{(r-1,c),(r,c)} x_{r-1,c}                (vertical bond)
  site 2c+1 : (a_c, b_c) = (P^{(r-1,c),(r,c+1)} x_{r-1,c},
                            P^{(r-1,c+1),(r,c)} x_{r-1,c+1})   (two diagonals)
              stored as the index a_c + d_a * b_c.
Row r is an MPO of site tensors S_c (which trace x_{r,c} out) and mediating
tensors M_c (which carry the horizontal and both diagonal couplings between
columns c and c+1).  The MPO bond between S_c and M_c is rho = P^R x_{r,c},
the spins of (r,c) coupled to any cluster of column c+1; between M_c and
S_{c+1} it is l = P^L x_{r,c+1}.  Site and mediating tensors are never built:
every use goes through the diagrams below, which enumerate x (site) or
(rho, l) (mediating), as in Fig. 7.

Psi_R = 1 and Psi_r = compress_chi(T_r Psi_{r+1}) for r = R-1 .. 1, where
compress is the variational zipper of Fig. 8 (Sec. III.B, "Variational
zipper algorithm for boundary MPS"):
  1. MPO tensors are attached right to left to the left-canonical
     Psi_{r+1}; at each site the dashed-box operator is truncated to 2 chi
     singular triplets by a matrix-free randomized SVD (Halko et al.);
  2. each zipper step is followed by a variational sweep over the two sites
     next to the zipper centre (the new site and the one built before it);
  3. the finished 2 chi MPS is refined by full one-site variational sweeps
     that maximise its overlap with T_r Psi_{r+1};
  4. a left-to-right SVD sweep truncates it to chi.
All Boltzmann tables are shifted by their minimum energy (per-table
log-scale).

Pins.  The untruncated contraction is pinned to brute force and closed forms.
The three diagram forms (apply, transpose, left transfer) are tied to each
other by adjoint identities on random tensors.  Every variational update is
checked never to move the state away from its target.  The chi truncation is
pinned to the TT-SVD upper bound and the Eckart-Young lower bound of the
exact state.  The value of log Z under truncation has no worked values to
compare with, so it is parity unpinned beyond those bounds and
chi-convergence.
"""
import numpy as np

from .potts import Potts, pext, pdep, popcount

SPLITMIX_GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


def splitmix64_finalize(z):
    """The SplitMix64 output function applied to a generator state z."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64(c):
    """Output c of the SplitMix64 stream started from state 0, i.e. the
    finaliser of the state (c + 1) * golden (vectorised over uint64)."""
    z = np.asarray(c, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z + np.uint64(1)) * np.uint64(SPLITMIX_GOLDEN)
    return splitmix64_finalize(z)


def rademacher(n_rows, n_cols, seed, r, k):
    """+-1 test matrix: entry (i, j) is + iff the top bit of
    splitmix64(key + i*n_cols + j) is set, key = splitmix64((seed<<24)+(r<<12)+k)."""
    key = splitmix64(np.uint64(((int(seed) << 24) + (r << 12) + k) & MASK64))
    idx = np.arange(n_rows * n_cols, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = splitmix64(key + idx)
    return np.where((z >> np.uint64(63)) == 1, 1.0, -1.0).reshape(n_rows, n_cols)


def orth(Y, cut):
    """Orthonormal basis of the numerical range of Y (singular values above
    cut * the largest), zero-padded to Y's column count."""
    out = np.zeros_like(Y)
    if Y.size == 0:
        return out
    U, s, _ = np.linalg.svd(Y, full_matrices=False)
    if s[0] <= 0:
        return out
    keep = s > cut * s[0]
    out[:, :int(keep.sum())] = U[:, keep]
    return out


def keep_triplets(U, S, Vt, t, cut):
    """The leading t singular triplets of an SVD, zero-padded to t, with
    those of sigma <= cut * sigma_max set to zero together with their
    vectors (R7)."""
    S = S[:t].copy()
    U = U[:, :t].copy()
    Vt = Vt[:t].copy()
    if S.size and S[0] > 0:
        drop = S <= cut * S[0]
    else:
        drop = np.ones(S.shape, dtype=bool)
    S[drop] = 0.0
    U[:, drop] = 0.0
    Vt[drop, :] = 0.0
    if S.size < t:                      # fewer singular values than the target
        pad = t - S.size
        S = np.concatenate([S, np.zeros(pad)])
        U = np.concatenate([U, np.zeros((U.shape[0], pad))], axis=1)
        Vt = np.concatenate([Vt, np.zeros((pad, Vt.shape[1]))], axis=0)
    return U, S, Vt


def svd_keep(M, t, cut):
    """Thin SVD of M with keep_triplets applied."""
    U, S, Vt = np.linalg.svd(M, full_matrices=False)
    return keep_triplets(U, S, Vt, t, cut)


def rsvd(apply, applyT, n_rows, n_cols, t, width, power, cut, seed, r, k):
    """Randomized truncated SVD of the implicit n_rows x n_cols operator D.

    Range finder Y = D Omega (Omega Rademacher, or the identity when D has no
    more columns than the sketch), `power` subspace iterations, Q = orth(Y),
    B = Q^T D, B = U S V^T; returns Q U[:, :t], S[:t], V^T[:t] with singular
    triplets below cut * S[0] set to zero.
    """
    if n_cols <= width:
        Y = apply(np.eye(n_cols))
        iters = 0
    else:
        Y = apply(rademacher(n_cols, width, seed, r, k))
        iters = power
    for _ in range(iters):
        Z = applyT(orth(Y, cut))
        Y = apply(orth(Z, cut))
    Q = orth(Y, cut)
    B = applyT(Q).T                     # (s, n_cols) = Q^T D
    Ub, S, Vt = svd_keep(B, t, cut)
    return Q @ Ub, S, Vt


def _segment_sum(vals, idx, n):
    """out[g] = sum of vals[i] with idx[i] == g (first axis)."""
    out = np.zeros((n,) + vals.shape[1:])
    if len(idx) == 0:
        return out
    order = np.argsort(idx, kind="stable")
    si = idx[order]
    starts = np.flatnonzero(np.r_[True, si[1:] != si[:-1]])
    out[si[starts]] = np.add.reduceat(vals[order], starts, axis=0)
    return out


class Network:
    """Boltzmann tables of one instance at inverse temperature beta (Eq. 6),
    each shifted by its minimum energy; `shift` is the total log-scale."""

    def __init__(self, inst, beta, keep=None):
        """keep: optional boolean mask per cluster (the states a local
        dimensional reduction retains, Sec. IV); the others get weight 0."""
        self.P = P = Potts(inst)
        self.beta = beta
        self.R, self.C = P.R, P.C
        self.w = []
        shift = 0.0
        for n in range(P.R * P.C):
            E = P.local_energy(n)
            Emin = E.min()
            shift += -beta * Emin
            w = np.exp(-beta * (E - Emin))
            self.w.append(w if keep is None else np.where(keep[n], w, 0.0))
        self.W = {}
        for (m, n) in P.inter:
            Eb = P.bond_energy(m, n)
            Emin = Eb.min()
            shift += -beta * Emin
            self.W[(m, n)] = np.exp(-beta * (Eb - Emin))
            self.W[(n, m)] = self.W[(m, n)].T
        self.shift = shift

    def cell(self, r, c):
        if 0 <= r < self.R and 0 <= c < self.C:
            return r * self.C + c
        return -1

    def B(self, m, n):
        return self.P.B(m, n) if (m >= 0 and n >= 0) else 0

    def Wt(self, m, n):
        """Bond weight table W[P^{mn} x_m, P^{nm} x_n] (ones(1,1) if none)."""
        if m < 0 or n < 0 or (m, n) not in self.W:
            return np.ones((1 << popcount(self.B(m, n)), 1 << popcount(self.B(n, m))))
        return self.W[(m, n)]

    # ---- boundary-MPS physical dimensions for the cut above row r ----------
    def phys_dims(self, r):
        """Physical dims of Psi_r (2C-1 sites) and the (d_a, d_b) split."""
        C = self.C
        dims, split = [], []
        for c in range(C):
            up, lo = self.cell(r - 1, c), self.cell(r, c)
            dims.append(1 << popcount(self.B(up, lo)))
            split.append(None)
            if c + 1 < C:
                da = 1 << popcount(self.B(self.cell(r - 1, c), self.cell(r, c + 1)))
                db = 1 << popcount(self.B(self.cell(r - 1, c + 1), self.cell(r, c)))
                dims.append(da * db)
                split.append((da, db))
        return dims, split

    def PL(self, r, c):
        n = self.cell(r, c)
        return (self.B(n, self.cell(r - 1, c - 1)) | self.B(n, self.cell(r, c - 1))
                | self.B(n, self.cell(r + 1, c - 1)))

    def PR(self, r, c):
        n = self.cell(r, c)
        return (self.B(n, self.cell(r - 1, c + 1)) | self.B(n, self.cell(r, c + 1))
                | self.B(n, self.cell(r + 1, c + 1)))


def sub(y, outer, inner):
    """Bits `inner` (subset of `outer`) of a value y = pext(x, outer)."""
    return pext(pdep(y, outer), inner)


class RowOps:
    """Diagram data for the row-r MPO (site tensors S_c, mediating M_c)."""

    def __init__(self, net, r):
        self.net, self.r = net, r
        C = net.C
        self.site = []
        for c in range(C):
            n = net.cell(r, c)
            up = net.cell(r - 1, c)
            k = int(net.P.k[n])
            x = np.arange(1 << k, dtype=np.int64)
            PL, PR = net.PL(r, c), net.PR(r, c)
            self.site.append(dict(
                w=net.w[n], x=x,
                u=pext(x, net.B(n, up)),                       # spins facing the upper cell
                Wv=net.Wt(up, n),                              # [v, u]
                vd=pext(x, net.B(n, net.cell(r + 1, c))),      # Psi_{r+1} site 2c index
                l=pext(x, PL), rho=pext(x, PR),
                dL=1 << popcount(PL), dR=1 << popcount(PR), PL=PL, PR=PR))
        self.med = []
        for c in range(C - 1):
            n0, n1 = net.cell(r, c), net.cell(r, c + 1)
            PR0, PL1 = net.PR(r, c), net.PL(r, c + 1)
            rho = np.arange(1 << popcount(PR0))
            ell = np.arange(1 << popcount(PL1))
            up0, up1 = net.cell(r - 1, c), net.cell(r - 1, c + 1)
            ld = sub(ell, PL1, net.B(n1, up0))          # spins of (r,c+1) facing (r-1,c)
            rd = sub(rho, PR0, net.B(n0, up1))          # spins of (r,c) facing (r-1,c+1)
            self.med.append(dict(
                Wh_tab=net.Wt(n0, n1), hr=sub(rho, PR0, net.B(n0, n1)), hl=sub(ell, PL1, net.B(n1, n0)),
                Wdr=net.Wt(up0, n1), Wdl=net.Wt(up1, n0), ld=ld, rd=rd,   # W(a, l_d), W(b, rho_d)
                a2=sub(rho, PR0, net.B(n0, net.cell(r + 1, c + 1))),       # Psi_{r+1} a'
                b2=sub(ell, PL1, net.B(n1, net.cell(r + 1, c))),           # Psi_{r+1} b'
                da2=1 << popcount(net.B(n0, net.cell(r + 1, c + 1))),
                dR=len(rho), dL=len(ell)))

    @staticmethod
    def _Wh_row(M, rho):
        """Horizontal weight W_h(rho, l) for every l (one row, built on demand)."""
        return M["Wh_tab"][M["hr"][rho], M["hl"]]

    # ---- site diagram (Fig. 7a,b) ------------------------------------------
    def site_apply(self, c, A, K, X):
        """(D X)[alpha, l, j] for the dashed box A_{2c} . S_c . K.
        A: (Da, d_v', Db); K: (Db, dR, Dg); X: (d_v, Dg, s)."""
        S = self.site[c]
        Xt = np.einsum("vu,vgj->ugj", S["Wv"], X)                  # W_v folded into X
        T = np.einsum("bxg,xgj->xbj", K[:, S["rho"], :], Xt[S["u"]])
        Y = np.einsum("axb,xbj->xaj", A[:, S["vd"], :], T) * S["w"][:, None, None]
        out = _segment_sum(Y, S["l"], S["dL"])                     # (dL, Da, s)
        return np.transpose(out, (1, 0, 2))

    def site_applyT(self, c, A, K, Y):
        """(D^T Y)[v, gamma, j];  Y: (Da, dL, s)."""
        S = self.site[c]
        Yx = Y[:, S["l"], :]                                       # (Da, x, s)
        T = np.einsum("axb,axj->xbj", A[:, S["vd"], :], Yx)
        G = np.einsum("bxg,xbj->xgj", K[:, S["rho"], :], T) * S["w"][:, None, None]
        Gu = _segment_sum(G, S["u"], S["Wv"].shape[1])              # (d_u, Dg, s)
        return np.einsum("vu,ugj->vgj", S["Wv"], Gu)

    # ---- mediating diagram (Fig. 7c,d) --------------------------------------
    CHUNK = 4096

    def med_apply(self, c, A, K, X, rhos=None):
        """(D X)[alpha, rho, j] for the dashed box A_{2c+1} . M_c . K.
        A: (Da, da'*db', Db); K: (Db, dL, Dg); X: (da, db, Dg, s).
        W_dr depends on l only through l_d and W_dl on rho only through
        rho_d, so both are applied to X first: X2[l_d, rho_d].  With `rhos`
        only those output rows rho are computed (in that order)."""
        M = self.med[c]
        Da = A.shape[0]
        Xa = np.einsum("al,abgj->lbgj", M["Wdr"], X)                 # (l_d, b, Dg, s)
        X2 = np.einsum("br,lbgj->lrgj", M["Wdl"], Xa)                # (l_d, rho_d, Dg, s)
        rhos = np.arange(M["dR"]) if rhos is None else np.asarray(rhos)
        out = np.zeros((Da, len(rhos), X.shape[-1]))
        for i, rho in enumerate(rhos):
            wh = self._Wh_row(M, rho)
            for l0 in range(0, M["dL"], self.CHUNK):
                l1 = min(M["dL"], l0 + self.CHUNK)
                X2r = X2[M["ld"][l0:l1], M["rd"][rho]]                 # (l, Dg, s)
                T = np.einsum("blg,lgj->lbj", K[:, l0:l1, :], X2r)
                Ar = A[:, M["a2"][rho] + M["da2"] * M["b2"][l0:l1], :]   # (Da, l, Db)
                out[:, i, :] += np.einsum("alb,lbj,l->aj", Ar, T, wh[l0:l1])
        return out

    def med_applyT(self, c, A, K, Y):
        """(D^T Y)[a, b, gamma, j];  Y: (Da, dR, s)."""
        M = self.med[c]
        Dg, s = K.shape[2], Y.shape[-1]
        nld, nrd = M["Wdr"].shape[1], M["Wdl"].shape[1]
        G2 = np.zeros((nld, nrd, Dg, s))                               # sum over l in l_d, rho in rho_d
        for rho in range(M["dR"]):
            wh = self._Wh_row(M, rho)
            for l0 in range(0, M["dL"], self.CHUNK):
                l1 = min(M["dL"], l0 + self.CHUNK)
                Ar = A[:, M["a2"][rho] + M["da2"] * M["b2"][l0:l1], :]   # (Da, l, Db)
                T = np.einsum("alb,aj->lbj", Ar, Y[:, rho, :])
                G = np.einsum("blg,lbj,l->lgj", K[:, l0:l1, :], T, wh[l0:l1])
                np.add.at(G2, (M["ld"][l0:l1], M["rd"][rho]), G)
        H = np.einsum("br,lrgj->lbgj", M["Wdl"], G2)                   # (l_d, b, Dg, s)
        return np.einsum("al,lbgj->abgj", M["Wdr"], H)

    # ---- left transfers (Fig. 8d: environments of the overlap) -------------
    def site_left(self, c, A, L, phi):
        """Left environment one site further right, through the site diagram:
        out[b, rho, g] = sum_{a, l, t, v} L[a, l, t] phi[t, v, g]
                         * (A_{2c} . S_c)[(a, l), v, (b, rho)],
        i.e. sum over x with P^R x = rho of w(x) A[:, v'(x), b]^T L[:, l(x), :]
        (sum_v W_v(v, u(x)) phi[:, v, :]).  L: (Da, dL, t); phi: (t, d_v, g)."""
        S = self.site[c]
        Pt = np.einsum("vu,tvg->utg", S["Wv"], phi)                   # (d_u, t, g)
        T = np.einsum("axt,xtg->xag", L[:, S["l"], :], Pt[S["u"]])   # (x, a, g)
        Y = np.einsum("axb,xag->xbg", A[:, S["vd"], :], T) * S["w"][:, None, None]
        out = _segment_sum(Y, S["rho"], S["dR"])                     # (dR, Db, g)
        return np.transpose(out, (1, 0, 2))

    def med_left(self, c, A, L, phi, ells=None):
        """Left environment through the mediating diagram:
        out[b, l, g] = sum_{a, rho, t, alpha, beta} L[a, rho, t] phi[t, alpha + da beta, g]
                       * W_h(rho, l) W_dr(alpha, l_d(l)) W_dl(beta, rho_d(rho))
                       * A[a, a'(rho) + da' b'(l), b].
        L: (Da, dR, t); phi: (t, da*db, g).  With `ells` only those l."""
        M = self.med[c]
        da, db = M["Wdr"].shape[0], M["Wdl"].shape[0]
        t, _, g = phi.shape
        P4 = phi.reshape(t, db, da, g)                                  # [t, beta, alpha, g]
        P2 = np.einsum("al,br,tbag->lrtg", M["Wdr"], M["Wdl"], P4)     # (l_d, rho_d, t, g)
        ells = np.arange(M["dL"]) if ells is None else np.asarray(ells)
        Db = A.shape[2]
        out = np.zeros((Db, len(ells), g))
        for i, l in enumerate(ells):
            for r0 in range(0, M["dR"], self.CHUNK):
                r1 = min(M["dR"], r0 + self.CHUNK)
                rho = np.arange(r0, r1)
                wh = M["Wh_tab"][M["hr"][rho], M["hl"][l]]                 # W_h(rho, l)
                Ar = A[:, M["a2"][rho] + M["da2"] * M["b2"][l], :]         # (Da, rho, Db)
                T = np.einsum("art,rtg->rag", L[:, r0:r1, :], P2[M["ld"][l], M["rd"][rho]])
                out[:, i, :] += np.einsum("arb,rag,r->bg", Ar, T, wh)
        return out


def trivial_mps(dims):
    return [np.ones((1, d, 1)) for d in dims]


class Options:
    """Compression options.  var_window: sites in the variational sweep after
    each zipper step (2: the new site and its right neighbour; 0: none).
    var_sweeps: full one-site sweeps at 2 chi before the chi truncation."""

    def __init__(self, chi, width_extra=8, power=1, cut=1e-6, seed=12345, var_window=2, var_sweeps=1):
        self.chi, self.width_extra, self.power, self.cut, self.seed = chi, width_extra, power, cut, seed
        self.var_window, self.var_sweeps = var_window, var_sweeps


class Box:
    """The dashed box of Fig. 8(c) at site k of the row-r zipper: site k of
    Psi_{r+1} (A, shape (Da, ds', Db)), MPO tensor k of row r and a right
    environment `conn` (Db, dm', Dg).  As a matrix it maps columns
    (sigma, g) (ds * Dg) to rows (a, m) (Da * dm); sigma is the physical
    index of Psi_r at site k."""

    def __init__(self, ops, dims, split, k, A, conn):
        self.ops, self.k, self.A, self.conn = ops, k, A, conn
        self.Da, self.Db = A.shape[0], A.shape[2]
        if k % 2 == 0:
            self.c = k // 2
            self.dm = ops.site[self.c]["dL"]
            self.dm_out = ops.site[self.c]["dR"]
        else:
            self.c = (k - 1) // 2
            self.dm = ops.med[self.c]["dR"]
            self.dm_out = ops.med[self.c]["dL"]
            self.da, self.db = split[k]
        self.ds = dims[k]
        self.Dg = conn.shape[2] if conn is not None else None

    @property
    def n_rows(self):
        return self.Da * self.dm

    def apply(self, Xf):
        """(D X) for X (ds*Dg, s) -> (Da*dm, s)."""
        s = Xf.shape[1]
        if self.k % 2 == 0:
            out = self.ops.site_apply(self.c, self.A, self.conn, Xf.reshape(self.ds, self.Dg, s))
        else:
            # column index sigma = a + da*b: reshape (db, da) then swap to (a, b)
            X = Xf.reshape(self.db, self.da, self.Dg, s).transpose(1, 0, 2, 3)
            out = self.ops.med_apply(self.c, self.A, self.conn, X)
        return out.reshape(-1, s)

    def applyT(self, Yf):
        """(D^T Y) for Y (Da*dm, s) -> (ds*Dg, s)."""
        s = Yf.shape[1]
        Y = Yf.reshape(self.Da, self.dm, s)
        if self.k % 2 == 0:
            out = self.ops.site_applyT(self.c, self.A, self.conn, Y)
        else:
            out = self.ops.med_applyT(self.c, self.A, self.conn, Y).transpose(1, 0, 2, 3)
        return out.reshape(-1, s)

    def left(self, Lf, phi):
        """Left environment after this site: Lf (Da*dm, t) over the rows of
        the box, phi (t, ds, g) the new site -> (Db*dm', g), the rows of the
        next site's box."""
        t = Lf.shape[1]
        L = Lf.reshape(self.Da, self.dm, t)
        if self.k % 2 == 0:
            out = self.ops.site_left(self.c, self.A, L, phi)
        else:
            out = self.ops.med_left(self.c, self.A, L, phi)
        return out.reshape(-1, phi.shape[2])


def site_cols(phi):
    """A site (t, ds, g) as the column block X (ds*g, t) of a box."""
    return phi.reshape(phi.shape[0], -1).T


def window_sweep(mk_box, k, QU, S, Vt, ds, conn_right, cut, trace=None):
    """Variational sweep over sites k and k+1 after zipper step k (R6).

    The rows (a, m) of the box at k stand for the part of T_r Psi_{r+1} left
    of the zipper centre; as in the zipper's own SVD they are taken as an
    orthonormal basis.  In that metric the state after step k is
    QU . (S Vt) . out[k+1] ..., with QU (rows x t) orthonormal columns.  The
    sweep (Fig. 8d) is two one-site overlap-maximisation updates:
      1. move the centre to k+1: S Vt = U_l R (left-canonical U_l), left
         environment L_{k+1} = left transfer of (QU, U_l) through site k;
         update site k+1 to L_{k+1} . (T Psi)_{k+1} . R_{k+2}, i.e. the
         transposed box at k+1 applied to L_{k+1}; make it right-canonical and
         recompute its right environment;
      2. update the centre at k within the span of QU: QU^T . (T Psi)_k .
         R_{k+1}, the transposed box at k applied to QU; split it into a
         right-canonical site and the new connector QU . (V S).
    Each update maximises the overlap with the target over one site with the
    rest fixed, so the distance to the target never grows.  Returns
    (site k, site k+1, connector at k (rows x t), connector at k+1)."""
    t = S.size
    Dg = Vt.shape[1] // ds
    Ul, _, _ = svd_keep((S[:, None] * Vt).reshape(t * ds, Dg), Dg, cut)
    phiL = Ul.reshape(t, ds, Dg)
    L1 = mk_box(k, None).left(QU, phiL)                        # (rows at k+1, Dg)
    b1 = mk_box(k + 1, conn_right)
    c1 = b1.applyT(L1)                                         # (cols at k+1, Dg)
    if trace:
        trace(dict(k=k, stage="window k+1", chain=[QU, phiL, c1.T.reshape(Dg, b1.ds, -1)]))
    U2, _, _ = svd_keep(c1, Dg, cut)
    site1 = U2.T.reshape(Dg, b1.ds, -1)                       # right-canonical
    conn1 = b1.apply(U2).reshape(b1.Da, b1.dm, Dg)
    c0 = mk_box(k, conn1).applyT(QU)                           # (ds*Dg, t)
    U3, S3, V3t = svd_keep(c0, t, cut)
    site0 = U3.T.reshape(t, ds, Dg)
    conn0 = QU @ (V3t.T * S3[None, :])
    if trace:
        trace(dict(k=k, stage="window k", chain=[conn0, site0, site1]))
    return site0, site1, conn0, conn1


def variational_sweeps(mk_box, phi, n_sweeps, cut, trace=None):
    """One-site variational sweeps of the MPS phi (list of (Dl, d, Dr); the
    first site carries the norm, the others are right-canonical) towards the
    target T_r Psi_{r+1} (Fig. 8d, Verstraete et al.).  The centre visits
    0, 1, .., K-1, K-2, .., 0 in the first sweep and 1, .., K-1, .., 0 in every
    further one.  At each visit the centre becomes L_k . (T Psi)_k . R_{k+1}
    (the transposed box applied to the left environment), which maximises the
    overlap over that site with the others fixed; moving on, it is split by
    an SVD into a canonical site and a factor carried to the next site, and
    the environment on the side it leaves is extended.  Returns phi with the
    norm in site 0 and the other sites right-canonical."""
    K = len(phi)
    phi = [p.copy() for p in phi]
    R = [None] * (K + 1)
    R[K] = np.ones((1, 1, 1))
    for k in range(K - 1, 0, -1):
        b = mk_box(k, R[k + 1])
        R[k] = b.apply(site_cols(phi[k])).reshape(b.Da, b.dm, phi[k].shape[0])
    L = [None] * K
    L[0] = np.ones((1, 1))
    seq = list(range(K)) + list(range(K - 2, -1, -1))
    for _ in range(n_sweeps - 1):
        seq += list(range(1, K)) + list(range(K - 2, -1, -1))
    for i, k in enumerate(seq):
        b = mk_box(k, R[k + 1])
        t = L[k].shape[1]
        phi[k] = b.applyT(L[k]).T.reshape(t, b.ds, -1)
        if trace:
            trace(dict(k=k, stage="sweep", phi=[p.copy() for p in phi]))
        nxt = seq[i + 1] if i + 1 < len(seq) else None
        if nxt == k + 1:
            Dg = phi[k].shape[2]
            U, S, Vt = svd_keep(phi[k].reshape(t * b.ds, Dg), Dg, cut)
            phi[k] = U.reshape(t, b.ds, Dg)
            phi[k + 1] = np.einsum("ij,jdx->idx", S[:, None] * Vt, phi[k + 1])
            L[k + 1] = mk_box(k, None).left(L[k], phi[k])
        elif nxt == k - 1:
            U, S, Vt = svd_keep(site_cols(phi[k]), t, cut)
            phi[k] = U.T.reshape(t, b.ds, -1)
            phi[k - 1] = np.einsum("adj,jt->adt", phi[k - 1], Vt.T * S[None, :])
            R[k] = b.apply(U).reshape(b.Da, b.dm, t)
    return phi


def zipper(net, r, psi, opts, truncate=True, trace=None):
    """compress(T_r Psi_{r+1}); psi is the left-canonical Psi_{r+1} (list of
    (Dl, d, Dr) tensors).  Returns (sites of Psi_r, log of the norm factored
    out).  With truncate=False (the top row, whose contraction is exact)
    only the zipper runs.  `trace`, if given, is called with the state after
    every zipper step and every variational update (tests)."""
    ops = RowOps(net, r)
    C = net.C
    K = 2 * C - 1
    dims, split = net.phys_dims(r)
    chi = opts.chi
    width = 2 * chi + opts.width_extra
    mk_box = lambda k, conn: Box(ops, dims, split, k, psi[k], conn)
    conns = [None] * (K + 1)
    conns[K] = np.ones((1, 1, 1))
    out = [None] * K
    for k in reversed(range(K)):
        box = mk_box(k, conns[k + 1])
        n_rows, n_cols = box.n_rows, box.ds * box.Dg
        t = min(2 * chi, n_rows, n_cols)
        QU, S, Vt = rsvd(box.apply, box.applyT, n_rows, n_cols, t, width, opts.power, opts.cut,
                         opts.seed, r, k)
        out[k] = Vt.reshape(t, box.ds, box.Dg)
        conns[k] = (QU * S).reshape(box.Da, box.dm, t)
        if trace:
            trace(dict(k=k, stage="zipper", chain=[QU * S, out[k]] + out[k + 1:]))
        if truncate and opts.var_window >= 2 and k + 1 < K:
            tail = out[k + 2:]
            wtrace = (lambda d: trace(dict(d, chain=d["chain"] + tail))) if trace else None
            out[k], out[k + 1], conn0, conn1 = window_sweep(mk_box, k, QU, S, Vt, box.ds, conns[k + 2],
                                                             opts.cut, wtrace)
            conns[k + 1] = conn1
            conns[k] = conn0.reshape(box.Da, box.dm, t)
    scalar = conns[0].reshape(-1)[0]
    if not truncate:
        out[0] = out[0] * np.sign(scalar) if scalar != 0 else out[0]
        logn = np.log(abs(scalar)) if scalar != 0 else -np.inf
        return out, logn
    out[0] = out[0] * scalar
    if opts.var_sweeps > 0:
        out = variational_sweeps(mk_box, out, opts.var_sweeps, opts.cut, trace)
    return truncate_sweep(out, chi, opts.cut)


def truncate_sweep(sites, chi, cut):
    """Left-to-right SVD sweep keeping chi singular values per bond; the last
    site is normalised and its norm returned as a log."""
    sites = [s.copy() for s in sites]
    for k in range(len(sites) - 1):
        Dl, d, Dr = sites[k].shape
        U, S, Vt = np.linalg.svd(sites[k].reshape(Dl * d, Dr), full_matrices=False)
        t = min(chi, Dl * d, Dr)
        S, U, Vt = S[:t].copy(), U[:, :t].copy(), Vt[:t].copy()
        drop = S <= cut * S[0] if S[0] > 0 else np.ones(t, dtype=bool)
        S[drop] = 0.0
        U[:, drop] = 0.0
        Vt[drop] = 0.0
        sites[k] = U.reshape(Dl, d, t)
        sites[k + 1] = np.einsum("tr,rdx->tdx", S[:, None] * Vt, sites[k + 1])
    nrm = np.linalg.norm(sites[-1])
    if nrm > 0:
        sites[-1] = sites[-1] / nrm
    return sites, (np.log(nrm) if nrm > 0 else -np.inf)


class Env:
    """Boundary MPSs Psi_1 .. Psi_R (Psi_r[k] tensors) and log Z."""

    def __init__(self, psi, lam, logZ, net):
        self.psi, self.lam, self.logZ, self.net = psi, lam, logZ, net


def contract_env(inst, beta, opts, keep=None):
    """All boundary MPSs, bottom-up, and log Z (Eq. 10) from the top row
    (keep: the retained states of a local dimensional reduction, Sec. IV)."""
    net = Network(inst, beta, keep)
    R = net.R
    psi = {R: trivial_mps(net.phys_dims(R)[0])}
    lam = {R: 0.0}
    for r in range(R - 1, 0, -1):
        sites, ln = zipper(net, r, psi[r + 1], opts)
        psi[r] = sites
        lam[r] = lam[r + 1] + ln
    top, ln0 = zipper(net, 0, psi[1], opts, truncate=False)
    val = 1.0
    for s in top:
        val = val * s.reshape(-1)[0] if s.size == 1 else val * s.sum()
    logZ = net.shift + lam[1] + ln0 + np.log(abs(val))
    env = Env(psi, lam, logZ, net)
    env.sign = 1 if val > 0 else -1     # a truncated environment can be sign-indefinite
    return env
