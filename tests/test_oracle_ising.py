"""Pins of the spin-level oracle against closed forms and brute force."""
import numpy as np
import pytest

from tnb_inputs import make_instance, planted_loops
from oracle import ising


def _loop_energy(inst, s):
    tot = 0.0
    for (i, j), J in zip(inst.edges.tolist(), inst.J.tolist()):
        tot = tot + J * s[i] * s[j]
    for i, h in enumerate(inst.h.tolist()):
        tot = tot + h * s[i]
    return tot


def test_energies_sequential_and_exact():
    inst = make_instance("zephyr", 1, jdist="uniform", hdist="uniform0.1", m=2, t=4)
    rng = np.random.default_rng(0)
    S = rng.choice([-1, 1], size=(6, inst.n_spins)).astype(np.int8)
    E = ising.energies(inst, S)
    for k in range(6):
        assert E[k] == _loop_energy(inst, S[k].astype(float))   # bit-exact, same order


def test_energies_quarter_integer_are_exact():
    inst = make_instance("zephyr", 3, jdist="quarter", hdist="zero", m=2, t=4)
    S = np.ones((1, inst.n_spins), dtype=np.int8)
    assert ising.energies(inst, S)[0] == inst.J.sum()
    assert (ising.energies(inst, S)[0] * 4) % 1 == 0


def test_planted_ground_energy():
    inst, s, E0 = planted_loops(2, 4, 5001)
    assert ising.energies(inst, s[None, :])[0] == E0


def test_brute_force_field_only():
    inst = make_instance("king", 5, jdist="zero", hdist="uniform1", R=3, C=4, a=1)
    beta = 0.7
    bf = ising.brute_force(inst, beta)
    assert abs(bf["logZ"] - ising.logz_field_only(inst.h, beta)) < 1e-12
    assert np.allclose(bf["m1"], -np.tanh(beta * inst.h), atol=1e-13)


def test_brute_force_tree_and_high_temperature():
    inst = make_instance("chain", 6, jdist="uniform", hdist="zero", n=14)
    bf = ising.brute_force(inst, 1.3)
    assert abs(bf["logZ"] - ising.logz_tree(inst.J, 14, 1.3)) < 1e-12
    assert np.allclose(bf["m1"], 0.0, atol=1e-14)          # Z2 symmetry, class I
    assert np.allclose(bf["m2"], -np.tanh(1.3 * inst.J), atol=1e-12)  # tree edge moments
    inst2 = make_instance("king", 9, jdist="uniform", hdist="uniform0.1", R=3, C=3, a=1)
    assert abs(ising.brute_force(inst2, 0.0)["logZ"] - 9 * np.log(2)) < 1e-12


def test_brute_force_ground_state_of_free_spins():
    inst = make_instance("king", 8, jdist="zero", hdist="uniform1", R=2, C=5, a=1)
    bf = ising.brute_force(inst, 1.0)
    assert abs(bf["E_min"] + np.abs(inst.h).sum()) < 1e-12
    g = bf["ground"][0]
    s = ((g >> np.arange(inst.n_spins)) & 1) * 2 - 1
    assert np.array_equal(s, -np.sign(inst.h))
