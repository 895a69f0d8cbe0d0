"""The oracle's droplet bookkeeping (Sec. III.A, Fig. 4) against Eq. (1),
enumeration of the configuration space and a chain worked by hand."""
import numpy as np

from tnb_inputs import make_instance
from tnb_inputs.instances import Instance
from oracle import ising
from oracle.bmps import contract_env, Options
from oracle.search import solve
from oracle.droplets import DropletOptions, apply_flip, hamming, connected, cluster_bonds
from oracle.potts import Potts


def _chain3():
    # s0 - s1 - s2 on a 1 x 3 cluster lattice, E = -s0 s1 - 0.5 s1 s2 + 0.25 s2
    return Instance(n_spins=3, edges=np.array([[0, 1], [1, 2]], dtype=np.int64), J=np.array([-1.0, -0.5]),
                    h=np.array([0.0, 0.0, 0.25]), R=1, C=3, cell_of=np.arange(3, dtype=np.int64))


def test_chain_worked_by_hand():
    # Step 1 groups (x0, x1) by x1 (cluster 0 no longer touches an unfixed
    # one): within a group the factor from s2 is common, so the member with
    # s0 = s1 wins and the other is the droplet "flip s0", dE = 2 |J01| = 2.
    # The last step merges nothing, so all four final states carry it; the
    # ground state (-,-,-) has E = -1.75 and its droplet (+,-,-) E = 0.25.
    inst = _chain3()
    env = contract_env(inst, 2.0, Options(chi=8))
    res = solve(inst, 2.0, env, M=8, K=4, droplets=DropletOptions())
    assert list(res["states"][0]) == [-1, -1, -1] and res["energies"][0] == -1.75
    for drops in res["droplets"]:
        assert drops == [(((0, 1),), 2.0)]


def _check_invariants(inst, res, opts):
    P = Potts(inst)
    bonds = cluster_bonds(P)
    for X, E, drops in zip(res["X"], res["energies"], res["droplets"]):
        assert len(drops) <= opts.max_droplets
        dEs = [e for _, e in drops]
        assert dEs == sorted(dEs)
        for f, e in drops:
            s2 = P.states_of_clusters(apply_flip(X, f)[None, :])
            assert ising.energies(inst, s2)[0] - E == e
            assert connected(f, bonds) and len(f) <= opts.max_cells and e <= opts.max_dE
        for i in range(len(drops)):
            for j in range(i):
                assert hamming(drops[i][0], drops[j][0]) >= opts.min_hamming


def test_droplet_invariants_quarter_couplings():
    inst = make_instance("king", 31, jdist="quarter", hdist="zero", R=3, C=4, a=1)
    env = contract_env(inst, 1.5, Options(chi=64))
    opts = DropletOptions(max_droplets=6, max_losers=3, min_hamming=2, max_cells=4)
    res = solve(inst, 1.5, env, M=6, K=4, droplets=opts)
    assert any(res["droplets"])
    _check_invariants(inst, res, opts)


def test_unlimited_droplets_partition_the_configuration_space():
    # exact contraction, every group kept, every limit lifted: each
    # configuration is a final state or exactly one droplet state of one
    inst = make_instance("king", 7, jdist="uniform", hdist="uniform0.1", R=3, C=3, a=1)
    env = contract_env(inst, 1.0, Options(chi=64))
    n = inst.n_spins
    opts = DropletOptions(max_droplets=1 << n, max_losers=1 << n, min_hamming=1, max_cells=64,
                          connected_only=False)
    res = solve(inst, 1.0, env, M=1 << n, K=1, droplets=opts)
    P = Potts(inst)
    Xf = P.cluster_of_states(res["all_states"])
    seen = []
    for X, drops in zip(Xf, res["all_droplets"]):
        seen.append(tuple(X))
        for f, e in drops:
            Y = apply_flip(X, f)
            seen.append(tuple(Y))
            s1, s2 = P.states_of_clusters(np.stack([X, Y]))
            E1, E2 = ising.energies(inst, np.stack([s1, s2]))
            assert abs((E2 - E1) - e) <= 1e-12
    assert len(seen) == len(set(seen)) == 1 << n
