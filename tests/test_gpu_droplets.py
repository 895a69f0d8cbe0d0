"""Droplets (Sec. III.A, Fig. 4) on the GPU: the excitations kept above every
branch equal the oracle's at every step (same flip sets in the same order,
dE within 1e-12), their energies follow Eq. (1) on the completed states, and
the bookkeeping's limits are enforced."""
import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle import ising
from oracle.bmps import contract_env, Options
from oracle.search import solve
from oracle.droplets import DropletOptions
from oracle.potts import Potts

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk, torch


def _opts_kw(o):
    return dict(max_droplets=o.max_droplets, max_losers=o.max_losers, min_hamming=o.min_hamming,
                max_cells=o.max_cells, max_dE=o.max_dE, connected_only=o.connected_only)


def _flips(P, X, states, nfix):
    Y = P.cluster_of_states(np.where(states == 0, -1, states))
    return [tuple((c, int(Y[q][c] ^ X[c])) for c in range(nfix) if Y[q][c] != X[c]) for q in range(len(Y))]


CASES = [("king", dict(R=3, C=4, a=1), 6, DropletOptions(max_droplets=6, max_losers=3, min_hamming=2, max_cells=4)),
         ("king", dict(R=3, C=3, a=2), 8, DropletOptions(max_droplets=8, max_losers=4, max_cells=6)),
         ("zephyr", dict(m=1, t=2), 8, DropletOptions()),
         ("zephyr", dict(m=2, t=1), 16, DropletOptions(max_droplets=10, max_losers=5, min_hamming=3)),
         ("king", dict(R=3, C=4, a=1), 6, DropletOptions(connected_only=False, max_dE=1.5))]


@pytest.mark.parametrize("kind,kw,M,opts", CASES)
def test_droplets_match_oracle_every_step(kind, kw, M, opts):
    pk, torch = _gpu()
    inst = make_instance(kind, 301, jdist="uniform", hdist="uniform0.1", **kw)
    ref = solve(inst, 1.0, contract_env(inst, 1.0, Options(chi=64, power=2, seed=5)), M=M, K=4, trace=True,
                droplets=opts)
    cl = pk.Clusters(inst, 1.0)
    env = pk.Env(cl, pk.EnvOptions(chi=64, power_iters=2, seed=5))
    beam = pk.Beam(env, M)
    beam.enable_droplets(**_opts_kw(opts))
    P = Potts(inst)
    N = inst.n_spins
    total = 0
    for rec in ref["steps"]:
        beam.step()
        states, _ = beam.export(len(rec["X"]), N)
        states = states.cpu().numpy()
        nfix = rec["n"] + 1
        X = P.cluster_of_states(np.where(states == 0, -1, states))
        for i, exp in enumerate(rec["droplets"]):
            ds, dE = beam.droplets(i, N)
            got = _flips(P, X[i], ds.cpu().numpy(), nfix)
            assert got == [e[0] for e in exp], (rec["n"], i)
            np.testing.assert_allclose(dE.cpu().numpy(), [e[1] for e in exp], rtol=0, atol=1e-12)
            total += len(exp)
    assert total > 0


def test_droplet_energies_follow_eq1_quarter_couplings():
    # exact arithmetic: every excitation of every final branch costs exactly
    # its dE on the completed states
    pk, torch = _gpu()
    inst = make_instance("king", 33, jdist="quarter", hdist="zero", R=4, C=5, a=1)
    cl = pk.Clusters(inst, 1.5)
    env = pk.Env(cl, pk.EnvOptions(chi=16, power_iters=2, seed=5))
    beam = pk.Beam(env, 32)
    beam.enable_droplets(max_droplets=12, max_losers=6, min_hamming=1, max_cells=8)
    for _ in range(inst.R * inst.C):
        beam.step()
    npar = beam.info()[1]
    states, _ = beam.export(npar, inst.n_spins)
    states = states.cpu().numpy()
    E = ising.energies(inst, states)
    seen = 0
    for i in range(npar):
        ds, dE = beam.droplets(i, inst.n_spins)
        ds, dE = ds.cpu().numpy(), dE.cpu().numpy()
        if len(ds):
            assert np.all(np.diff(dE) >= 0)
            np.testing.assert_array_equal(ising.energies(inst, ds) - E[i], dE)
            seen += len(ds)
    assert seen > 0


def test_droplet_limits_and_order_of_calls():
    pk, torch = _gpu()
    inst = make_instance("king", 5, jdist="uniform", hdist="zero", R=2, C=3, a=1)
    cl = pk.Clusters(inst, 1.0)
    env = pk.Env(cl, pk.EnvOptions(chi=8))
    beam = pk.Beam(env, 4)
    for bad in (dict(max_droplets=17), dict(max_losers=9), dict(max_cells=65), dict(min_hamming=0),
                dict(max_losers=0)):
        with pytest.raises(pk.TnbError) as e:
            beam.enable_droplets(**bad)
        assert e.value.code == -1
    with pytest.raises(pk.TnbError):
        beam.droplets(0, inst.n_spins)          # bookkeeping off
    beam.step()
    with pytest.raises(pk.TnbError):
        beam.enable_droplets()                  # after the first step


def test_solve_returns_the_best_branch_droplets_planted():
    # planted king's lattice: the exact ground energy E0 bounds every
    # excitation state from below, and each state costs E_best + dE
    pk, torch = _gpu()
    from tnb_inputs import planted_king
    inst, s_star, E0 = planted_king(6, 6, 1, 11)
    res = pk.solve(inst, 3.0, 16, 32, K=2, droplets=dict(max_droplets=12, max_losers=6, max_cells=16))
    assert res["energies"][0] == E0
    ds, dE = res["droplet_states"], res["droplet_dE"]
    assert len(ds) > 0 and np.all(np.diff(dE) >= 0)
    E = ising.energies(inst, ds)
    np.testing.assert_array_equal(E - res["energies"][0], dE)
    assert np.all(E >= E0)
