"""The oracle's loopy belief propagation (Sec. IV, Fig. 9) against brute
force on cluster trees, closed forms, and the reduced partition function."""
import numpy as np

from tnb_inputs import make_instance
from oracle import ising
from oracle.bmps import contract_env, Options, Network
from oracle.lbp import lbp, select, exact_marginals
from oracle.potts import Potts


def test_exact_on_cluster_trees():
    # a single row of clusters is a path: belief propagation is exact there
    for kind, kw in (("king", dict(R=1, C=4, a=2)), ("chain", dict(n=10))):
        inst = make_instance(kind, 17, jdist="uniform", hdist="uniform0.1", **kw)
        bel, _, change = lbp(inst, 0.8, 12)
        ref = exact_marginals(inst, 0.8, Potts(inst))
        for p, q in zip(bel, ref):
            np.testing.assert_allclose(p, q, rtol=1e-12, atol=1e-15)
        assert change < 1e-13          # converged: another sweep changes nothing


def test_infinite_temperature_and_uncoupled_cluster():
    inst = make_instance("king", 3, jdist="uniform", hdist="uniform0.1", R=3, C=3, a=2)
    bel, _, _ = lbp(inst, 0.0, 5)
    for p in bel:
        np.testing.assert_allclose(p, np.full(len(p), 1.0 / len(p)), rtol=1e-14)
    one = make_instance("king", 3, jdist="uniform", hdist="uniform0.1", R=1, C=1, a=2)
    bel, _, _ = lbp(one, 1.3, 3)
    w = Network(one, 1.3).w[0]
    np.testing.assert_allclose(bel[0], w / w.sum(), rtol=1e-14)


def test_reduction_restricts_the_partition_function():
    # keeping the LBP-most-probable states per cluster: log Z of the exact
    # contraction equals the brute-force sum over the retained configurations
    inst = make_instance("king", 9, jdist="uniform", hdist="uniform0.1", R=2, C=2, a=2)
    bel, _, _ = lbp(inst, 1.0, 8)
    keep = select(bel, 6)
    assert all(m.sum() == 6 for m in keep)
    z = contract_env(inst, 1.0, Options(chi=256), keep=keep).logZ
    P = Potts(inst)
    s = ising.all_states(inst.n_spins)
    X = P.cluster_of_states(s)
    ok = np.all([keep[n][X[:, n]] for n in range(P.R * P.C)], axis=0)
    E = ising.energies(inst, s[ok])
    ref = -1.0 * E.min() + np.log(np.exp(-1.0 * (E - E.min())).sum())
    assert abs(z - ref) <= 1e-12 * abs(ref)
