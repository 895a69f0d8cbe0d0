"""Marginals and branch and bound: brute force, exact DP, closed forms."""
import numpy as np
import pytest

from tnb_inputs import make_instance, planted_loops
from oracle import ising
from oracle.bmps import contract_env, Options, Network
from oracle.search import solve, right_envs, marginals
from oracle.potts import Potts


def _brute_cluster_marginal(inst, beta, n_cell):
    # clamp the cluster's spins one configuration at a time via fields:
    # p(x) = Z(x) / Z with Z(x) from brute force on the clamped instance
    import copy
    P = Potts(inst)
    sp = P.spins[n_cell]
    k = len(sp)
    logs = np.empty(1 << k)
    for x in range(1 << k):
        c = copy.deepcopy(inst)
        big = 60.0 / beta
        for b, i in enumerate(sp):
            c.h = c.h.copy()
            c.h[i] += -big if (x >> b) & 1 else big
        logs[x] = ising.brute_force(c, beta)["logZ"] + beta * big * k
    p = np.exp(logs - logs.max())
    return p / p.sum()


@pytest.mark.parametrize("kind,kw", [("king", dict(R=2, C=3, a=2)), ("zephyr", dict(m=1, t=2))])
def test_first_marginal_matches_brute_force(kind, kw):
    inst = make_instance(kind, 51, jdist="uniform", hdist="uniform0.1", **kw)
    env = contract_env(inst, 1.0, Options(chi=128, cut=1e-13))
    net = env.net
    X = np.zeros((1, net.R * net.C), dtype=np.int64)
    R = right_envs(net, env, 0, X)
    q, _ = marginals(net, env, 0, 0, X, np.ones((1, 1)), R[0])
    p = q[0] / q[0].sum()
    assert np.allclose(p, _brute_cluster_marginal(inst, 1.0, 0), atol=1e-12)


def test_conditional_marginal_mid_row_matches_brute_force():
    # parent with row 0 fixed and (1,0) fixed; open (1,1) on a 3x3 king lattice
    inst = make_instance("king", 52, jdist="uniform", hdist="uniform0.1", R=3, C=3, a=1)
    beta = 1.2
    env = contract_env(inst, beta, Options(chi=64, cut=1e-13))
    net = env.net
    fixed = {0: 1, 1: 0, 2: 1, 3: 0}
    X = np.zeros((1, 9), dtype=np.int64)
    for k, v in fixed.items():
        X[0, k] = v
    R = right_envs(net, env, 1, X)
    _, vec = marginals(net, env, 1, 0, X, np.ones((1, 1)), R[0][[0]])
    L = vec[:, X[0, 3]]
    q, _ = marginals(net, env, 1, 1, X, L, R[1])
    p = q[0] / q[0].sum()
    N = 9
    x = np.arange(1 << N)
    s = (((x[:, None] >> np.arange(N)) & 1) * 2 - 1)
    ok = np.all([((x >> k) & 1) == v for k, v in fixed.items()], axis=0)
    E = s[:, inst.edges[:, 0]] * s[:, inst.edges[:, 1]] @ inst.J + s @ inst.h
    w = np.where(ok, np.exp(-beta * (E - E.min())), 0.0)
    pb = np.bincount((x >> 4) & 1, weights=w, minlength=2)
    assert np.allclose(p, pb / pb.sum(), atol=1e-12)


def test_marginals_sum_to_one_and_are_probabilities():
    # every parent's conditional distribution at every step of a truncated
    # run (chi = 4): entries in [0, 1], summing to one
    inst = make_instance("zephyr", 53, jdist="uniform", hdist="uniform0.1", m=1, t=2)
    env = contract_env(inst, 1.0, Options(chi=4))
    res = solve(inst, 1.0, env, M=16, K=4, trace=True)
    for rec in res["steps"]:
        p = rec["p"]
        assert np.all(p >= 0) and np.all(p <= 1)
        assert np.allclose(p.sum(axis=1), 1.0, atol=1e-12)


def test_returned_energies_sorted_and_recomputed():
    inst = make_instance("zephyr", 53, jdist="uniform", hdist="uniform0.1", m=1, t=2)
    env = contract_env(inst, 1.0, Options(chi=4))
    res = solve(inst, 1.0, env, M=16, K=4)
    assert np.all(np.diff(res["energies"]) >= 0)
    assert np.array_equal(res["energies"], ising.energies(inst, res["states"]))


def _brute_beam(inst, beta, M):
    """Branch and bound with probabilities from brute-force enumeration
    (Sec. III.A): the chain-rule score of a partial configuration is then the
    log of its exact marginal probability.  The boundary of a partial
    configuration is the set of fixed spins with a coupling to an unfixed spin
    (Eq. 8), compared by value.  Group winners and the top M go to the larger
    score, ties to the smaller (parent, x); no merge once the boundary is
    empty; p_d is the best top-M loser over all steps."""
    P = Potts(inst)
    N, ncell = inst.n_spins, P.R * P.C
    x = np.arange(1 << N)
    s = ((x[:, None] >> np.arange(N)) & 1) * 2 - 1
    E = (s[:, inst.edges[:, 0]] * s[:, inst.edges[:, 1]]) @ inst.J + s @ inst.h
    w = np.exp(-beta * (E - E.min()))
    w /= w.sum()
    X = P.cluster_of_states(s)                        # (2^N, cells)
    parents = [()]
    pd_log = -np.inf
    steps = []
    for n in range(ncell):
        fixed_cells = set(range(n + 1))
        bnd = sorted({int(i) for (i, j) in inst.edges if (inst.cell_of[i] in fixed_cells) != (inst.cell_of[j] in fixed_cells)
                      for i in ((i,) if inst.cell_of[i] in fixed_cells else (j,))})
        cands = []
        for b, par in enumerate(parents):
            match = np.all(X[:, :n] == np.array(par, dtype=np.int64)[None, :], axis=1) if n else np.ones(len(x), bool)
            for xv in range(1 << int(P.k[n])):
                m = match & (X[:, n] == xv)
                pm = w[m].sum()
                if pm <= 0:
                    continue
                conf = par + (xv,)
                spins_b = s[np.flatnonzero(m)[0]]
                key = tuple(int(spins_b[i]) for i in bnd)
                cands.append((np.log(pm), b, xv, key, conf))
        cands.sort(key=lambda c: (-c[0], c[1], c[2]))
        if bnd:
            seen, win = set(), []
            for c in cands:
                if c[3] not in seen:
                    seen.add(c[3])
                    win.append(c)
        else:
            win = cands
        if len(win) > M:
            pd_log = max(pd_log, win[M][0])
        keep = win[:M]
        steps.append(([(c[4], c[0]) for c in keep], pd_log))
        parents = [c[4] for c in keep]
    return steps, pd_log


@pytest.mark.parametrize("kind,kw,M", [("king", dict(R=3, C=3, a=1), 3), ("king", dict(R=4, C=4, a=1), 4),
                                       ("king", dict(R=2, C=2, a=2), 5), ("king", dict(R=3, C=4, a=1), 2)])
def test_largest_discarded_probability_matches_brute_force_beam(kind, kw, M):
    inst = make_instance(kind, 63, jdist="uniform", hdist="uniform0.1", **kw)
    beta = 1.5
    env = contract_env(inst, beta, Options(chi=128, cut=1e-13))
    res = solve(inst, beta, env, M=M, K=1, trace=True)
    bsteps, bpd = _brute_beam(inst, beta, M)
    assert np.isfinite(bpd)
    assert abs(res["p_d_log"] - bpd) < 1e-9
    assert len(res["steps"]) == len(bsteps)
    for rec, (bs, bpd_n) in zip(res["steps"], bsteps):
        got = sorted((tuple(int(v) for v in row[: rec["n"] + 1]), lp) for row, lp in zip(rec["X"], rec["logp"]))
        ref = sorted(bs)
        assert [g[0] for g in got] == [r[0] for r in ref]
        assert np.allclose([g[1] for g in got], [r[1] for r in ref], atol=1e-9)
        assert rec["p_d_log"] == bpd_n == -np.inf or abs(rec["p_d_log"] - bpd_n) < 1e-9


@pytest.mark.parametrize("kind,kw", [("king", dict(R=3, C=3, a=1)), ("king", dict(R=4, C=5, a=1)),
                                     ("king", dict(R=2, C=2, a=2))])
def test_exact_marginals_large_beam_is_exact_dp(kind, kw):
    inst = make_instance(kind, 61, jdist="uniform", hdist="uniform0.1", **kw)
    env = contract_env(inst, 2.0, Options(chi=64, cut=1e-13))
    res = solve(inst, 2.0, env, M=1 << 12, K=2)
    bf = ising.brute_force(inst, 2.0)
    assert abs(res["energies"][0] - bf["E_min"]) < 1e-12


def test_field_only_ground_state():
    inst = make_instance("king", 62, jdist="zero", hdist="uniform1", R=3, C=4, a=2)
    env = contract_env(inst, 1.0, Options(chi=2))
    res = solve(inst, 1.0, env, M=4, K=1)
    assert np.array_equal(res["states"][0], -np.sign(inst.h).astype(np.int8))
    assert abs(res["energies"][0] + np.abs(inst.h).sum()) < 1e-12


def test_planted_small_instance_reaches_planted_energy():
    inst, s, E0 = planted_loops(1, 2, 77, loops_per_cell=2)
    env = contract_env(inst, 1.0, Options(chi=32))
    res = solve(inst, 1.0, env, M=256, K=2)
    bf = ising.brute_force(inst, 1.0)
    assert abs(bf["E_min"] - E0) < 1e-12        # the planted energy is the ground energy
    assert abs(res["energies"][0] - E0) < 1e-12


# ---- row moments (adjoint of the row contraction) -------------------------

from oracle.search import row_moments, row_logz, row_spins_edges  # noqa: E402
from oracle.bmps import Network as _Net  # noqa: E402


def _cond_brute(inst, beta, fixed, spins, edges):
    """<s_i>, <s_i s_j> given fixed spins {i: +-1}, by enumerating the rest."""
    N = inst.n_spins
    free = np.array([i for i in range(N) if i not in fixed], dtype=np.int64)
    x = np.arange(1 << len(free))
    s = np.zeros((len(x), N))
    for i, v in fixed.items():
        s[:, i] = v
    s[:, free] = ((x[:, None] >> np.arange(len(free))) & 1) * 2 - 1
    E = (s[:, inst.edges[:, 0]] * s[:, inst.edges[:, 1]]) @ inst.J + s @ inst.h
    w = np.exp(-beta * (E - E.min()))
    w /= w.sum()
    m1 = w @ s[:, spins]
    ee = inst.edges[edges]
    m2 = w @ (s[:, ee[:, 0]] * s[:, ee[:, 1]])
    return m1, m2


def _spins_of_cells(inst, X, cells):
    from oracle.potts import Potts
    P = Potts(inst)
    out = {}
    for n in cells:
        for b, i in enumerate(P.spins[n]):
            out[int(i)] = 1 if (X[n] >> b) & 1 else -1
    return out


def test_row_moments_first_row_match_brute_force():
    # exact environment: the row moments of the empty configuration are the
    # unconditioned <s_i>, <s_i s_j> of row 0
    inst = make_instance("king", 81, jdist="uniform", hdist="uniform0.1", R=2, C=2, a=2)
    beta = 0.9
    env = contract_env(inst, beta, Options(chi=64, cut=1e-13))
    net = env.net
    X = np.zeros((1, 4), dtype=np.int64)
    m1, m2, sp, ed = row_moments(net, env, 0, 0, X, np.ones((1, 1)))
    assert len(ed) > 0
    b1, b2 = _cond_brute(inst, beta, {}, sp, ed)
    assert np.allclose(m1[0], b1, atol=1e-12)
    assert np.allclose(m2[0], b2, atol=1e-12)


@pytest.mark.parametrize("kind,kw,r,c", [("king", dict(R=2, C=3, a=2), 1, 1),
                                         ("king", dict(R=3, C=3, a=1), 1, 2),
                                         ("zephyr", dict(m=1, t=2), 1, 0)])
def test_row_moments_mid_row_match_conditional_brute_force(kind, kw, r, c):
    inst = make_instance(kind, 82, jdist="uniform", hdist="uniform0.1", **kw)
    beta = 1.1
    env = contract_env(inst, beta, Options(chi=64, cut=1e-13))
    net = env.net
    ncell = net.R * net.C
    rng = np.random.default_rng(5)
    X = np.zeros((2, ncell), dtype=np.int64)
    n0 = r * net.C + c
    for k in range(n0):
        X[:, k] = rng.integers(0, 1 << int(net.P.k[k]), size=2)
    # left vectors from the oracle's own marginals
    Rr = right_envs(net, env, r, X)
    L = np.ones((2, 1))
    for cc in range(c):
        _, vec = marginals(net, env, r, cc, X, L, Rr[cc])
        L = vec[np.arange(2), X[:, r * net.C + cc]]
    m1, m2, sp, ed = row_moments(net, env, r, c, X, L)
    for b in range(2):
        fixed = _spins_of_cells(inst, X[b], range(n0))
        b1, b2 = _cond_brute(inst, beta, fixed, sp, ed)
        assert np.allclose(m1[b], b1, atol=1e-11)
        assert np.allclose(m2[b], b2, atol=1e-11)


def test_row_moments_are_log_z_derivatives_of_the_approximate_network():
    # for any fixed Psi_{r+1} (here a truncated one) the moments are
    # -1/beta d log Z_b / d h_i and -1/beta d log Z_b / d J_ij
    inst = make_instance("king", 83, jdist="uniform", hdist="uniform0.1", R=3, C=3, a=2)
    beta, r, c, eps = 1.3, 1, 1, 1e-6
    env = contract_env(inst, beta, Options(chi=3))
    net = env.net
    X = np.zeros((1, 9), dtype=np.int64)
    X[0, :4] = [5, 9, 12, 3]
    Rr = right_envs(net, env, r, X)
    _, vec = marginals(net, env, r, 0, X, np.ones((1, 1)), Rr[0])
    L = vec[:, X[0, 3]]
    m1, m2, sp, ed = row_moments(net, env, r, c, X, L)
    import copy

    def lz(dh=None, dJ=None):
        k = copy.deepcopy(inst)
        if dh is not None:
            k.h = k.h + dh
        if dJ is not None:
            k.J = k.J + dJ
        return row_logz(_Net(k, beta), env, r, c, X[0], L[0])

    for col in (0, 3, len(sp) - 1):
        dh = np.zeros(inst.n_spins)
        dh[sp[col]] = eps
        fd = (lz(dh=dh) - lz(dh=-dh)) / (2 * eps)
        assert abs(fd + beta * m1[0, col]) < 1e-7
    for col in (0, len(ed) - 1):
        dJ = np.zeros(len(inst.J))
        dJ[ed[col]] = eps
        fd = (lz(dJ=dJ) - lz(dJ=-dJ)) / (2 * eps)
        assert abs(fd + beta * m2[0, col]) < 1e-7


def test_row_moments_fixed_cluster_layout():
    inst = make_instance("zephyr", 84, jdist="uniform", m=1, t=2)
    net = _Net(inst, 1.0)
    sp, ed = row_spins_edges(net, 1, 0)
    cells = inst.cell_of[sp]
    assert np.all(np.diff(cells) >= 0) and np.all(cells // net.C == 1)
    assert np.all(inst.cell_of[inst.edges[ed, 0]] == inst.cell_of[inst.edges[ed, 1]])
