"""Clustered Hamiltonian (Eq. 3-5) pinned by the spin-level energy."""
import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle import ising
from oracle.potts import Potts, pext, pdep


@pytest.mark.parametrize("kind,kw", [("zephyr", dict(m=2, t=4)), ("king", dict(R=3, C=3, a=3)),
                                     ("zephyr", dict(m=3, t=2))])
def test_cluster_identity(kind, kw):
    inst = make_instance(kind, 17, jdist="uniform", hdist="uniform0.1", **kw)
    P = Potts(inst)
    rng = np.random.default_rng(1)
    S = rng.choice([-1, 1], size=(8, inst.n_spins)).astype(np.int8)
    X = P.cluster_of_states(S)
    H = np.zeros(8)
    for n in range(P.R * P.C):
        if P.k[n]:
            H += P.local_energy(n)[X[:, n]]
    for (m, n) in P.inter:
        Eb = P.bond_energy(m, n)
        H += Eb[pext(X[:, m], P.B(m, n)), pext(X[:, n], P.B(n, m))]
    assert np.allclose(H, ising.energies(inst, S), atol=1e-12, rtol=0)
    assert np.array_equal(P.states_of_clusters(X), S)


def test_cluster_identity_is_bit_exact_for_quarter_couplings():
    inst = make_instance("zephyr", 3000, jdist="quarter", hdist="zero", m=2, t=4)
    P = Potts(inst)
    S = np.random.default_rng(2).choice([-1, 1], size=(4, inst.n_spins)).astype(np.int8)
    X = P.cluster_of_states(S)
    H = np.zeros(4)
    for n in range(P.R * P.C):
        if P.k[n]:
            H += P.local_energy(n)[X[:, n]]
    for (m, n) in P.inter:
        H += P.bond_energy(m, n)[pext(X[:, m], P.B(m, n)), pext(X[:, n], P.B(n, m))]
    assert np.array_equal(H, ising.energies(inst, S))


def test_projector_masks_are_the_coupled_spins():
    inst = make_instance("zephyr", 4, jdist="uniform", hdist="zero", m=2, t=4)
    P = Potts(inst)
    for (m, n), mask in P.mask.items():
        want = 0
        for (i, j) in inst.edges.tolist():
            if inst.cell_of[i] == m and inst.cell_of[j] == n:
                want |= 1 << int(P.bit[i])
            if inst.cell_of[j] == m and inst.cell_of[i] == n:
                want |= 1 << int(P.bit[j])
        assert mask == want
    # all Zephyr cross-cell projections are 2^8 or smaller
    assert max(bin(v).count("1") for v in P.mask.values()) == 8


def test_pext_pdep_roundtrip():
    x = np.arange(1 << 12)
    for mask in (0, 0b1, 0b101101, 0xF0F, 0xFFF):
        y = pext(x, mask)
        assert np.array_equal(pext(pdep(y, mask), mask), y)
        assert np.array_equal(pdep(y, mask), x & mask)
