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
    inst = make_instance("zephyr", 53, jdist="uniform", hdist="uniform0.1", m=1, t=2)
    env = contract_env(inst, 1.0, Options(chi=4))
    res = solve(inst, 1.0, env, M=16, K=4)
    assert np.all(np.diff(res["energies"]) >= 0)
    assert np.array_equal(res["energies"], ising.energies(inst, res["states"]))


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
