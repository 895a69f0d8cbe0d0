"""Row moments of beam states: HIP adjoint and per-branch paths against the
oracle's clamped contractions, and against each other at full size."""
import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle.bmps import contract_env, Options
from oracle.search import solve, row_moments

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk, torch


# (kind, lattice, chi, M, parents compared per step)
CASES = [("king", dict(R=2, C=3, a=2), 64, 16, 6), ("zephyr", dict(m=1, t=2), 64, 16, 4),
         ("king", dict(R=3, C=4, a=1), 4, 16, 8), ("king", dict(R=3, C=3, a=2), 3, 8, 3)]


@pytest.mark.parametrize("kind,kw,chi,M,nchk", CASES)
def test_row_moments_match_oracle_every_step(kind, kw, chi, M, nchk):
    pk, torch = _gpu()
    beta = 1.0
    inst = make_instance(kind, 401, jdist="uniform", hdist="uniform0.1", **kw)
    ora_env = contract_env(inst, beta, Options(chi=chi, power=2, seed=5))
    ref = solve(inst, beta, ora_env, M=M, K=4, trace=True)
    env = pk.Env(pk.Clusters(inst, beta), pk.EnvOptions(chi=chi, power_iters=2, seed=5))
    beam = pk.Beam(env, M)
    net = ora_env.net
    ncell = net.R * net.C
    X, L = np.zeros((1, ncell), dtype=np.int64), np.ones((1, 1))
    for step, rec in enumerate(ref["steps"]):
        r, c = divmod(step, net.C)
        sp, ed = beam.row_layout()
        m1, m2 = beam.row_moments()
        o1, o2, osp, oed = row_moments(net, ora_env, r, c, X[:nchk], L[:nchk])
        assert np.array_equal(sp, osp) and np.array_equal(ed, oed)
        g1, g2 = m1.cpu().numpy()[:nchk], m2.cpu().numpy()[:nchk]
        assert np.abs(g1 - o1).max() <= 1e-6, ("m1", step, np.abs(g1 - o1).max())
        if len(ed):
            assert np.abs(g2 - o2).max() <= 1e-6, ("m2", step, np.abs(g2 - o2).max())
        pb = beam.row_moments_per_branch().cpu().numpy()[:nchk]
        assert np.abs(pb - o1).max() <= 1e-6, ("per-branch", step, np.abs(pb - o1).max())
        beam.step()
        X, L = rec["X"], rec["L"]


def test_row_moments_zephyr_t4_adjoint_equals_per_branch():
    # full cluster size (16-spin cells of Z_2, d = 2^16) at the start of row 1
    # and mid-row: the two GPU algorithms agree.  The chi = 16 environment of
    # this random instance has negative terms, so the moments are signed
    # ratios and may leave [-1, 1]; both paths must give the same ones.
    pk, torch = _gpu()
    inst = make_instance("zephyr", 402, jdist="uniform", hdist="uniform0.1", m=2, t=4)
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=16, seed=7))
    beam = pk.Beam(env, 8)
    C = inst.C
    checked = 0
    for step in range(2 * C):
        if step in (C, C + 1):
            sp, ed = beam.row_layout()
            m1, m2 = beam.row_moments()
            pb = beam.row_moments_per_branch()
            a, b = m1.cpu().numpy(), pb.cpu().numpy()
            assert a.shape == b.shape and a.shape[1] == len(sp) > 0
            assert np.abs(a - b).max() <= 1e-8, np.abs(a - b).max()
            assert np.all(np.isfinite(m2.cpu().numpy()))
            checked += 1
        beam.step()
    assert checked == 2


@pytest.mark.parametrize("chi", [16, 32])
def test_row_moments_planted_t4_exact_truncation(chi):
    # 12-spin cells (d = 4096) on sparse planted couplings, where the
    # truncation is exact: the environment is non-negative, the moments of the
    # current cluster are the first moments of its marginal, every moment is
    # in [-1, 1], and the oracle agrees on the first parents of every step
    pk, torch = _gpu()
    from tnb_inputs import planted_loops
    from tnb_inputs.rng import uniform01
    inst, s, E0 = planted_loops(1, 4, 78, loops_per_cell=2)
    inst.h = 0.1 * (2 * uniform01(78, inst.n_spins, stream=2) - 1)
    ora_env = contract_env(inst, 1.0, Options(chi=chi, power=2, seed=5, cut=1e-7))
    ref = solve(inst, 1.0, ora_env, M=8, K=4, trace=True)
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=chi, power_iters=2, seed=5, cut=1e-7))
    beam = pk.Beam(env, 8)
    net = ora_env.net
    C = inst.C
    X, L = np.zeros((1, net.R * C), dtype=np.int64), np.ones((1, 1))
    for step, rec in enumerate(ref["steps"]):
        r, c = divmod(step, C)
        m1, m2 = beam.row_moments()
        a = m1.cpu().numpy()
        p = beam.marginals().cpu().numpy()
        k = int(np.sum(inst.cell_of == r * C + c))
        x = np.arange(p.shape[1])
        sv = ((x[:, None] >> np.arange(k)) & 1) * 2.0 - 1.0
        assert np.allclose(p @ sv, a[:, :k], atol=1e-9)
        assert np.all(np.abs(a) <= 1 + 1e-9) and np.all(np.abs(m2.cpu().numpy()) <= 1 + 1e-9)
        if c == C - 1:  # one cluster left in the row: the oracle is cheap there
            o1, o2, _, _ = row_moments(net, ora_env, r, c, X[:2], L[:2])
            assert np.abs(a[:2] - o1).max() <= 1e-8
            assert np.abs(m2.cpu().numpy()[:2] - o2).max() <= 1e-8
        beam.step()
        X, L = rec["X"], rec["L"]


def test_row_moments_argument_checks():
    pk, torch = _gpu()
    import ctypes
    from paper_2411_16431_amd import _lib as L
    inst = make_instance("king", 403, jdist="uniform", R=2, C=2, a=1)
    env = pk.Env(pk.Clusters(inst, 1.0), pk.EnvOptions(chi=4))
    beam = pk.Beam(env, 4)
    m1 = torch.empty(1, dtype=torch.float64, device="cuda")
    st = L.lib().tnb_row_moments(beam._h, ctypes.c_void_p(m1.data_ptr()), 1, None, 0, None)
    assert st == -1  # two spins in the first row, one slot given
    for _ in range(4):
        beam.step()
    sp = ctypes.c_int32()
    assert L.lib().tnb_row_layout(beam._h, ctypes.byref(sp), None, None, None, 0) == -1


@pytest.mark.parametrize("kind,kw,chi", [("king", dict(R=2, C=3, a=2), 64), ("zephyr", dict(m=1, t=2), 64),
                                         ("king", dict(R=3, C=3, a=2), 3)])
def test_first_row_logz_gradient(kind, kw, chi):
    # the autograd Function's backward (the HIP adjoint) against central finite
    # differences of its forward (log Z from tnb_contract_env), and, with an
    # exact environment, against brute-force <s_i> and <s_i s_j>
    pk, torch = _gpu()
    from oracle import ising
    inst = make_instance(kind, 404, jdist="uniform", hdist="uniform0.1", **kw)
    beta = 0.8
    opts = pk.EnvOptions(chi=chi, power_iters=2, seed=3, cut=1e-7)
    sp, ed = pk.first_row_layout(inst, beta)
    h = torch.tensor(inst.h[sp], dtype=torch.float64, requires_grad=True)
    J = torch.tensor(inst.J[ed], dtype=torch.float64, requires_grad=True)
    lz = pk.FirstRowLogZ.apply(h, J, inst, beta, opts)
    lz.backward()
    gh, gJ = h.grad.numpy(), J.grad.numpy()
    eps = 1e-5
    f = lambda hh, JJ: pk.FirstRowLogZ.apply(torch.tensor(hh), torch.tensor(JJ), inst, beta, opts).item()
    h0, J0 = inst.h[sp].copy(), inst.J[ed].copy()
    for i in (0, len(sp) // 2, len(sp) - 1):
        dh = np.zeros_like(h0)
        dh[i] = eps
        fd = (f(h0 + dh, J0) - f(h0 - dh, J0)) / (2 * eps)
        assert abs(fd - gh[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, gh[i])
    for e in (0, len(ed) - 1):
        dJ = np.zeros_like(J0)
        dJ[e] = eps
        fd = (f(h0, J0 + dJ) - f(h0, J0 - dJ)) / (2 * eps)
        assert abs(fd - gJ[e]) <= 1e-6 * (1 + abs(fd)), (e, fd, gJ[e])
    if chi == 64:
        bf = ising.brute_force(inst, beta)
        assert np.allclose(-gh / beta, bf["m1"][sp], atol=1e-8)
        assert np.allclose(-gJ / beta, bf["m2"][ed], atol=1e-8)
