"""The square / king's-lattice workload of App. B (one spin per site, d = 2,
chi = 16, M = 256, beta = 4) against the oracle."""
import numpy as np
import pytest

from tnb_inputs import make_instance, planted_king
from oracle import ising
from oracle.bmps import contract_env, Options
from oracle.search import solve

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk, torch


def test_planted_king_16x16_reaches_E0_and_matches_logz():
    pk, torch = _gpu()
    inst, s, E0 = planted_king(16, 16, 1, 11, loops_per_cell=1)
    o = Options(chi=16, power=2, seed=3)
    ora = contract_env(inst, 4.0, o)
    res = pk.solve(inst, 4.0, chi=16, M=256, K=4, power_iters=2, seed=3)
    assert abs(res["logZ"] - ora.logZ) <= 1e-5 * abs(ora.logZ), (res["logZ"], ora.logZ)
    assert res["energies"][0] == E0
    assert np.array_equal(res["energies"], ising.energies(inst, res["states"]))


def test_random_king_10x10_stepwise_with_near_tie_log():
    pk, torch = _gpu()
    from oracle.potts import Potts
    inst = make_instance("king", 12, jdist="uniform", hdist="uniform0.1", R=10, C=10, a=1)
    ora_env = contract_env(inst, 4.0, Options(chi=16, power=2, seed=3))
    M = 256
    ref = solve(inst, 4.0, ora_env, M=M, K=4, trace=True)
    env = pk.Env(pk.Clusters(inst, 4.0), pk.EnvOptions(chi=16, power_iters=2, seed=3))
    assert abs(env.logZ - ora_env.logZ) <= 1e-5 * abs(ora_env.logZ)
    beam = pk.Beam(env, M)
    P = Potts(inst)
    compared, diverged = 0, False
    for rec in ref["steps"]:
        p = beam.marginals().cpu().numpy()
        assert np.abs(p - rec["p"]).max() <= 1e-5, rec["n"]
        beam.step()
        states, logp = beam.export(M, inst.n_spins)
        S = states.cpu().numpy()
        got_X = P.cluster_of_states(np.where(S == 0, -1, S))[:, : rec["n"] + 1]
        compared += 1
        if not np.array_equal(got_X, rec["X"][:, : rec["n"] + 1]):
            gap = min(rec["boundary_gap"], rec["group_gap"])
            print("near tie at step %d (gap %.3e); comparison ends after %d of %d steps"
                  % (rec["n"], gap, compared, len(ref["steps"])))
            assert gap <= 1e-5
            diverged = True
            break
    if not diverged:
        st, en = beam.lowest(4, inst.n_spins)
        assert np.array_equal(en.cpu().numpy(), ref["energies"])
    assert compared >= 10
