"""Boundary-MPS oracle: untruncated contraction against brute force and
closed forms, invariances, and the randomized SVD against a dense SVD."""
import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle import ising
from oracle.bmps import contract_env, Options, rsvd, orth, rademacher


CASES = [("king", dict(R=2, C=3, a=2)), ("king", dict(R=4, C=4, a=1)),
         ("king", dict(R=3, C=4, a=1)), ("zephyr", dict(m=1, t=2)),
         ("king", dict(R=3, C=2, a=2, diag=False))]


@pytest.mark.parametrize("kind,kw", CASES)
@pytest.mark.parametrize("beta", [0.5, 2.0])
def test_exact_contraction_equals_brute_force(kind, kw, beta):
    inst = make_instance(kind, 31, jdist="uniform", hdist="uniform0.1", **kw)
    env = contract_env(inst, beta, Options(chi=128, cut=1e-13))
    bf = ising.brute_force(inst, beta)
    assert abs(env.logZ - bf["logZ"]) < 1e-9 * abs(bf["logZ"])


def test_chain_closed_form():
    inst = make_instance("chain", 2, jdist="uniform", hdist="zero", n=40)
    env = contract_env(inst, 1.7, Options(chi=2))
    assert abs(env.logZ - ising.logz_tree(inst.J, 40, 1.7)) < 1e-11


def test_field_only_closed_form_at_zephyr_size():
    # J = 0: every bond weight is 1 and the truncated contraction is exact
    inst = make_instance("zephyr", 3, jdist="zero", hdist="uniform0.1", m=2, t=2)
    env = contract_env(inst, 1.0, Options(chi=2))
    assert abs(env.logZ - ising.logz_field_only(inst.h, 1.0)) < 1e-10


def test_gauge_invariance():
    inst = make_instance("king", 41, jdist="uniform", hdist="uniform0.1", R=3, C=3, a=2)
    g = np.where(np.random.default_rng(3).random(inst.n_spins) < 0.5, -1.0, 1.0)
    import copy
    inst2 = copy.deepcopy(inst)
    inst2.J = inst.J * g[inst.edges[:, 0]] * g[inst.edges[:, 1]]
    inst2.h = inst.h * g
    for chi in (4, 64):
        a = contract_env(inst, 1.0, Options(chi=chi)).logZ
        b = contract_env(inst2, 1.0, Options(chi=chi)).logZ
        assert abs(a - b) < 1e-8 * abs(a)


def test_transposed_lattice_same_logz_when_exact():
    inst = make_instance("king", 43, jdist="uniform", hdist="uniform0.1", R=3, C=4, a=1)
    import copy
    t = copy.deepcopy(inst)
    r, c = np.divmod(inst.cell_of, inst.C)
    t.R, t.C = inst.C, inst.R
    t.cell_of = c * t.C + r
    a = contract_env(inst, 1.0, Options(chi=64, cut=1e-13)).logZ
    b = contract_env(t, 1.0, Options(chi=64, cut=1e-13)).logZ
    assert abs(a - b) < 1e-10 * abs(a)


def test_chi_convergence_is_monotone_in_error():
    inst = make_instance("king", 44, jdist="uniform", hdist="uniform0.1", R=4, C=4, a=2)
    ref = contract_env(inst, 1.0, Options(chi=128, cut=1e-12)).logZ
    errs = [abs(contract_env(inst, 1.0, Options(chi=chi, power=2)).logZ - ref) for chi in (2, 8, 32)]
    assert errs[2] < errs[0] and errs[2] < 1e-5 * abs(ref)


def test_rsvd_exact_when_sketch_covers_columns():
    rng = np.random.default_rng(5)
    D = rng.standard_normal((40, 12)) @ np.diag(np.logspace(0, -3, 12)) @ rng.standard_normal((12, 12))
    QU, S, Vt = rsvd(lambda X: D @ X, lambda Y: D.T @ Y, 40, 12, 5, 16, 2, 1e-12, 1, 0, 0)
    U0, S0, Vt0 = np.linalg.svd(D, full_matrices=False)
    assert np.allclose(S, S0[:5], rtol=1e-12)
    assert np.allclose((QU * S) @ Vt, (U0[:, :5] * S0[:5]) @ Vt0[:5], atol=1e-12)


def test_rsvd_sketch_recovers_low_rank():
    rng = np.random.default_rng(6)
    D = rng.standard_normal((300, 6)) @ rng.standard_normal((6, 200))
    QU, S, Vt = rsvd(lambda X: D @ X, lambda Y: D.T @ Y, 300, 200, 8, 14, 1, 1e-10, 9, 1, 2)
    assert np.allclose((QU * S) @ Vt, D, atol=1e-10 * np.abs(D).max())
    assert np.count_nonzero(S) == 6


def test_rademacher_is_counter_based_and_balanced():
    a = rademacher(64, 32, 7, 3, 4)
    b = rademacher(64, 32, 7, 3, 4)
    assert np.array_equal(a, b) and set(np.unique(a)) == {-1.0, 1.0}
    assert abs(a.mean()) < 0.05
    assert not np.array_equal(a, rademacher(64, 32, 7, 3, 5))


def test_orth_drops_numerical_null_space():
    Y = np.outer(np.arange(1.0, 6.0), np.ones(3))
    Q = orth(Y, 1e-10)
    assert np.allclose(Q[:, 1:], 0) and abs(np.linalg.norm(Q[:, 0]) - 1) < 1e-14


def test_splitmix64_matches_published_outputs():
    # SplitMix64 (Steele, Lea, Flood 2014): the stream from seed 1234567 begins
    # 6457827717110365317, 3203168211198807973, 9817491932198370423,
    # 4593380528125082431, 16408922859458223821 (Rosetta Code, "Pseudo-random
    # numbers/Splitmix64"), and the stream from seed 0 begins 0xe220a8397b1dcdaf.
    # State k of a stream is seed + k * golden.
    from oracle.bmps import splitmix64, splitmix64_finalize, SPLITMIX_GOLDEN
    from tnb_inputs import splitmix64 as inputs_splitmix64
    g = SPLITMIX_GOLDEN
    states = np.array([(1234567 + k * g) % (1 << 64) for k in range(1, 6)], dtype=np.uint64)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [int(v) for v in splitmix64_finalize(states)] == want
    assert int(splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    assert int(inputs_splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    # counter c is state (c + 1) * golden of the seed-0 stream
    c = np.arange(5, dtype=np.uint64)
    ref = splitmix64_finalize(np.array([((int(i) + 1) * g) % (1 << 64) for i in c], dtype=np.uint64))
    assert np.array_equal(splitmix64(c), ref) and np.array_equal(inputs_splitmix64(c), ref)
