"""FP32 environment contractions (tnb_prec TNB_F32) against the FP64 oracle.

The diagram kernels run in FP32 on the matrix cores with FP32 copies of the
Boltzmann weights; every other step stays FP64.  The tolerances below are the
stated FP32 error of each result: diagram outputs 2e-5 of their largest
magnitude (sums of up to 2^21 FP32 products), log Z 1e-6 relative where the
contraction is exact and 1e-5 (the FP64 target) under truncation, marginals
1e-5 absolute with identical kept configurations."""
import numpy as np
import pytest

from tnb_inputs import make_instance, planted_loops
from oracle import ising
from oracle.bmps import Network, RowOps, contract_env, Options
from oracle.search import solve

pytestmark = pytest.mark.gpu
TOL_DIAGRAM = 2e-5


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("r,k", [(1, 1), (1, 2), (1, 3), (2, 3), (2, 4)])
def test_fp32_diagrams_match_oracle(r, k):
    # Zephyr Z_2 t=2: all three forms of one box, in full
    pk, torch = _gpu()
    inst = make_instance("zephyr", 1000, jdist="uniform", hdist="uniform0.1", m=2, t=2)
    net = Network(inst, 1.0)
    cl = pk.Clusters(inst, 1.0)
    ops = RowOps(net, r)
    dm_in, dm_out, ds, dsb = pk.diagram_dims(cl, r, k)
    rng = np.random.default_rng(31 + r + k)
    Da = Db = 16
    Dg, S = 32, 40
    A = rng.standard_normal((dsb, Da, Db))
    Kc = rng.standard_normal((dm_out, Db, Dg))
    X = rng.standard_normal((ds, Dg, S))
    Y = rng.standard_normal((dm_in, Da, S))
    L = rng.standard_normal((dm_in, Da, Dg))
    phi = rng.standard_normal((ds, Dg, Dg))
    A_o, K_o, L_o, phi_o = (a.transpose(1, 0, 2) for a in (A, Kc, L, phi))
    run = lambda mode, K_, X_: pk.diagram_apply(cl, r, k, mode, _dev(torch, A), _dev(torch, K_), _dev(torch, X_),
                                                prec="f32").cpu().numpy()
    if k % 2 == 0:
        c = k // 2
        refs = (ops.site_apply(c, A_o, K_o, X).transpose(1, 0, 2),
                ops.site_applyT(c, A_o, K_o, Y.transpose(1, 0, 2)),
                ops.site_left(c, A_o, L_o, phi_o).transpose(1, 0, 2))
    else:
        c = (k - 1) // 2
        da, db = net.phys_dims(r)[1][k]
        refs = (ops.med_apply(c, A_o, K_o, X.reshape(db, da, Dg, S).transpose(1, 0, 2, 3)).transpose(1, 0, 2),
                ops.med_applyT(c, A_o, K_o, Y.transpose(1, 0, 2)).transpose(1, 0, 2, 3).reshape(ds, Dg, S),
                ops.med_left(c, A_o, L_o, phi_o).transpose(1, 0, 2))
    errs = [_rel(run(0, Kc, X), refs[0]), _rel(run(1, Kc, Y), refs[1]), _rel(run(2, L, phi), refs[2])]
    print("FP32 diagram r=%d k=%d relative errors (apply, transpose, left): %s" % (r, k, errs))
    assert max(errs) <= TOL_DIAGRAM and max(errs) > 0


def test_fp32_central_mediating_full_size():
    # the bench's central mediating diagram (Z_2 t=4, row 1, legs 65536 x 65536)
    pk, torch = _gpu()
    inst = make_instance("zephyr", 1000, jdist="uniform", hdist="uniform0.1", m=2, t=4)
    net = Network(inst, 1.0)
    cl = pk.Clusters(inst, 1.0)
    r, k = 1, 3
    ops = RowOps(net, r)
    dm_in, dm_out, ds, dsb = pk.diagram_dims(cl, r, k)
    da, db = net.phys_dims(r)[1][k]
    rng = np.random.default_rng(41)
    A = rng.standard_normal((dsb, 16, 16))
    Kc = rng.standard_normal((dm_out, 16, 32))
    X = rng.standard_normal((ds, 32, 40))
    got = pk.diagram_apply(cl, r, k, 0, _dev(torch, A), _dev(torch, Kc), _dev(torch, X), prec="f32").cpu().numpy()
    ref64 = pk.diagram_apply(cl, r, k, 0, _dev(torch, A), _dev(torch, Kc), _dev(torch, X)).cpu().numpy()
    rhos = np.array([0, 255, 256, dm_in - 1])
    ref = ops.med_apply((k - 1) // 2, A.transpose(1, 0, 2), Kc.transpose(1, 0, 2),
                        X.reshape(db, da, 32, 40).transpose(1, 0, 2, 3), rhos=rhos).transpose(1, 0, 2)
    e_oracle = _rel(got[rhos], ref)
    e_all = _rel(got, ref64)          # FP32 against the FP64 kernels over every row
    print("FP32 central mediating apply: %.2e against the oracle (sampled rows), %.2e against FP64 (all rows)"
          % (e_oracle, e_all))
    assert e_oracle <= TOL_DIAGRAM and e_all <= TOL_DIAGRAM


@pytest.mark.parametrize("kind,kw", [("king", dict(R=2, C=3, a=2)), ("zephyr", dict(m=1, t=2))])
def test_fp32_exact_logz(kind, kw):
    pk, torch = _gpu()
    inst = make_instance(kind, 201, jdist="uniform", hdist="uniform0.1", **kw)
    bf = ising.brute_force(inst, 1.0)
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=64, cut=1e-7, prec="f32"))
    rel = abs(env.logZ - bf["logZ"]) / abs(bf["logZ"])
    print("FP32 exact log Z %s: relative error %.2e" % (kind, rel))
    assert rel <= 1e-6


@pytest.mark.parametrize("kind,kw,chi", [("king", dict(R=4, C=4, a=2), 6), ("zephyr", dict(m=2, t=1), 8),
                                         ("zephyr", dict(m=1, t=3), 8)])
def test_fp32_truncated_logz(kind, kw, chi):
    pk, torch = _gpu()
    inst = make_instance(kind, 202, jdist="uniform", hdist="uniform0.1", **kw)
    ora = contract_env(inst, 1.0, Options(chi=chi, width_extra=8, power=2, cut=1e-6, seed=777))
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=chi, power_iters=2, cut=1e-6, seed=777, prec="f32"))
    rel = abs(env.logZ - ora.logZ) / abs(ora.logZ)
    print("FP32 truncated log Z %s chi=%d: relative error %.2e against the FP64 oracle" % (kind, chi, rel))
    assert rel <= 1e-5


def test_fp32_beam_marginals_and_states():
    # every beam step of a planted t = 4 instance with fields (exact truncation)
    pk, torch = _gpu()
    from oracle.potts import Potts
    from tnb_inputs.rng import uniform01
    inst, s, E0 = planted_loops(1, 4, 77, loops_per_cell=2)
    inst.h = 0.1 * (2 * uniform01(77, inst.n_spins, stream=2) - 1)
    ora_env = contract_env(inst, 1.0, Options(chi=16, power=2, seed=5, cut=1e-7))
    ref = solve(inst, 1.0, ora_env, M=16, K=4, trace=True)
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=16, power_iters=2, seed=5, cut=1e-7, prec="f32"))
    beam = pk.Beam(env, 16)
    P = Potts(inst)
    worst = 0.0
    for rec in ref["steps"]:
        p = beam.marginals().cpu().numpy()
        worst = max(worst, float(np.abs(p - rec["p"]).max()))
        beam.step()
        states, logp = beam.export(16, inst.n_spins)
        S = states.cpu().numpy()
        got_X = P.cluster_of_states(np.where(S == 0, -1, S))[:, : rec["n"] + 1]
        assert np.array_equal(got_X, rec["X"][:, : rec["n"] + 1])
    print("FP32 marginals: max |dp| %.2e over every step" % worst)
    assert worst <= 1e-5
