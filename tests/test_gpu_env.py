"""Parity of the HIP boundary-MPS contraction (tnb_contract_env) with the
oracle: log Z and bond dimensions, exact and truncated."""
import numpy as np
import pytest

from tnb_inputs import make_instance, planted_loops
from oracle import ising
from oracle.bmps import contract_env, Options

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk


EXACT = [("king", dict(R=2, C=3, a=2)), ("king", dict(R=4, C=4, a=1)), ("zephyr", dict(m=1, t=2)),
         ("king", dict(R=3, C=2, a=2, diag=False)), ("chain", dict(n=12))]


@pytest.mark.parametrize("kind,kw", EXACT)
def test_exact_logz(kind, kw):
    pk = _gpu()
    inst = make_instance(kind, 201, jdist="uniform", hdist="uniform0.1", **kw)
    bf = ising.brute_force(inst, 1.0)
    cl = pk.Clusters(inst, 1.0)
    env = pk.Env(cl, pk.EnvOptions(chi=64, cut=1e-7))
    assert abs(env.logZ - bf["logZ"]) < 1e-10 * abs(bf["logZ"])


TRUNC = [("king", dict(R=4, C=4, a=2), 2), ("king", dict(R=4, C=4, a=2), 6),
         ("king", dict(R=5, C=6, a=1), 3), ("zephyr", dict(m=2, t=1), 4),
         ("zephyr", dict(m=2, t=1), 8),
         # t = 3 cells: 64 horizontal bins (several register chunks)
         ("zephyr", dict(m=1, t=3), 8)]


@pytest.mark.parametrize("kind,kw,chi", TRUNC)
def test_truncated_logz_matches_oracle(kind, kw, chi):
    pk = _gpu()
    inst = make_instance(kind, 202, jdist="uniform", hdist="uniform0.1", **kw)
    ora = contract_env(inst, 1.0, Options(chi=chi, width_extra=8, power=2, cut=1e-6, seed=777))
    cl = pk.Clusters(inst, 1.0)
    env = pk.Env(cl, pk.EnvOptions(chi=chi, sketch_extra=8, power_iters=2, cut=1e-6, seed=777))
    # target tolerance: 1e-5 relative on log Z
    assert abs(env.logZ - ora.logZ) <= 1e-5 * abs(ora.logZ), (env.logZ, ora.logZ)
    for r in range(1, inst.R):
        for k, site in enumerate(ora.psi[r]):
            assert env.site_shape(r, k) == site.shape


@pytest.mark.parametrize("chi", [16, 32])
def test_zephyr_t4_planted_logz_matches_oracle(chi):
    # 16-spin-class cells (t = 4): 256 horizontal bins in 16 register chunks, and at
    # chi = 32 the sketch (72 columns) is processed in column blocks.  With sparse planted
    # couplings chi = 16 is already exact, so parity is strict.
    pk = _gpu()
    inst, s, E0 = planted_loops(1, 4, 77, loops_per_cell=2)
    ora = contract_env(inst, 1.0, Options(chi=chi, power=2, cut=1e-7, seed=777))
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=chi, power_iters=2, cut=1e-7, seed=777))
    assert abs(env.logZ - ora.logZ) <= 1e-10 * abs(ora.logZ), (env.logZ, ora.logZ)


def test_zephyr_t4_random_logz_within_conditioning():
    # Random couplings on Z_1 (t = 4) at chi = 32: a truncated zipper can be
    # ill-conditioned (a 1e-14 relative change of J moves the oracle's own
    # log Z), so GPU and CPU rounding may lead to different truncations.  The
    # bound is ten times the conditioning measured in this test, floored at
    # the 1e-5 relative target.
    import copy
    pk = _gpu()
    inst = make_instance("zephyr", 202, jdist="uniform", hdist="uniform0.1", m=1, t=4)
    o = Options(chi=32, power=2, cut=1e-6, seed=777)
    ora = contract_env(inst, 1.0, o).logZ
    pert = copy.deepcopy(inst)
    pert.J = inst.J * (1 + 1e-14 * np.cos(np.arange(len(inst.J))))
    spread = abs(contract_env(pert, 1.0, o).logZ - ora)
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=32, power_iters=2, cut=1e-6, seed=777))
    assert abs(env.logZ - ora) <= max(1e-5 * abs(ora), 10 * spread), (env.logZ, ora, spread)


def test_field_only_closed_form_zephyr():
    # J = 0 on Z_2 (t = 1): every bond weight is 1, exact at chi = 1
    pk = _gpu()
    inst = make_instance("zephyr", 203, jdist="zero", hdist="uniform0.1", m=2, t=1)
    cl = pk.Clusters(inst, 1.0)
    env = pk.Env(cl, pk.EnvOptions(chi=1))
    assert abs(env.logZ - ising.logz_field_only(inst.h, 1.0)) < 1e-10 * abs(env.logZ)


def test_invalid_options_rejected():
    pk = _gpu()
    inst = make_instance("king", 204, R=2, C=2, a=1)
    cl = pk.Clusters(inst, 1.0)
    with pytest.raises(pk.TnbError) as e:
        pk.Env(cl, pk.EnvOptions(chi=0))
    assert e.value.code == -1


def test_sign_of_a_sign_indefinite_truncation_is_reported():
    # chi = 2 without variational sweeps at beta = 3 leaves this king's
    # lattice with a negative approximate Z; log Z is log |Z| on both sides
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    from tnb_inputs import make_instance
    from oracle.bmps import contract_env, Options
    inst = make_instance("king", 67, jdist="uniform", hdist="zero", R=4, C=4, a=2)
    ref = contract_env(inst, 3.0, Options(chi=2, power=2, var_window=0, var_sweeps=0))
    cl = pk.Clusters(inst, 3.0)
    env = pk.Env(cl, pk.EnvOptions(chi=2, var_window=0, var_sweeps=0))
    assert ref.sign == -1 and env.sign == -1
    assert abs(env.logZ - ref.logZ) <= 1e-10 * abs(ref.logZ)
    exact = pk.Env(cl, pk.EnvOptions(chi=64))
    assert exact.sign == 1
