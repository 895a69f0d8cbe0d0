"""Variational zipper of the oracle (Sec. III.B, "Variational zipper algorithm
for boundary MPS", Fig. 8c-d).

Pins, none of which reuses the formula under test:
  - the three forms of every diagram (apply, transpose, left transfer) are
    tied by adjoint identities on random tensors: <Y, D X> = <D^T Y, X> and
    <left(L, phi), K> = <L, D_K phi>, with D_K the box whose right
    environment is K.  apply itself is pinned to brute force through the
    untruncated contraction;
  - every variational update maximises an overlap over one site with the rest
    fixed, so the distance to the target never grows: checked update by
    update against the dense target, for the window sweep after each zipper
    step (in the zipper's own metric, where the rows of the box are an
    orthonormal basis) and for the full sweeps (in the true metric);
  - when the 2 chi stage is exact the sweeps change nothing;
  - a planted index mistake in a left transfer breaks the identity.
"""
import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle.bmps import Network, Options, RowOps, Box, site_cols, trivial_mps, zipper
import oracle.bmps as bm


def _net(kind, kw, seed=61, beta=1.0):
    inst = make_instance(kind, seed, jdist="uniform", hdist="uniform0.1", **kw)
    return Network(inst, beta)


def _rand_psi(net, r, rng, D=3):
    """Random sites of a boundary MPS below row r (bond D, open ends 1)."""
    dims = net.phys_dims(r + 1)[0]
    K = len(dims)
    out = []
    for k, d in enumerate(dims):
        Dl = 1 if k == 0 else D
        Dr = 1 if k == K - 1 else D
        out.append(rng.standard_normal((Dl, d, Dr)))
    return out


DIAGRAM_CASES = [("king", dict(R=3, C=3, a=2)), ("king", dict(R=3, C=4, a=1)),
                 ("zephyr", dict(m=1, t=2)), ("king", dict(R=3, C=3, a=2, diag=False))]


@pytest.mark.parametrize("kind,kw", DIAGRAM_CASES)
def test_diagram_forms_are_adjoint(kind, kw):
    net = _net(kind, kw)
    rng = np.random.default_rng(5)
    r = 1
    ops = RowOps(net, r)
    psi = _rand_psi(net, r, rng)
    dims, split = net.phys_dims(r)
    for k in range(len(dims)):
        probe = Box(ops, dims, split, k, psi[k], None)
        Dg, t, s = 2, 3, 2
        K = rng.standard_normal((probe.Db, probe.dm_out, Dg))
        box = Box(ops, dims, split, k, psi[k], K)
        X = rng.standard_normal((box.ds * Dg, s))
        Y = rng.standard_normal((box.n_rows, s))
        lhs, rhs = np.vdot(Y, box.apply(X)), np.vdot(box.applyT(Y), X)
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs)), (k, lhs, rhs)
        L = rng.standard_normal((box.n_rows, t))
        phi = rng.standard_normal((t, box.ds, Dg))
        lhs = np.vdot(probe.left(L, phi), K.reshape(-1, Dg))
        rhs = np.vdot(L, box.apply(site_cols(phi)))
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs)), (k, lhs, rhs)


def test_planted_mistake_in_left_transfer_breaks_the_identity(monkeypatch):
    # reading the two diagonal indices of the new site in the wrong order
    # (sigma = beta + db * alpha instead of alpha + da * beta) must be caught
    net = _net("zephyr", dict(m=1, t=2))
    rng = np.random.default_rng(8)
    ops = RowOps(net, 1)
    real = RowOps.med_left

    def wrong(self, c, A, L, phi, ells=None):
        M = self.med[c]
        da, db = M["Wdr"].shape[0], M["Wdl"].shape[0]
        t, _, g = phi.shape
        swapped = phi.reshape(t, da, db, g).transpose(0, 2, 1, 3).reshape(t, da * db, g)
        return real(self, c, A, L, swapped, ells)

    psi = _rand_psi(net, 1, rng)
    dims, split = net.phys_dims(1)
    ks = [k for k in range(1, len(dims), 2) if split[k][0] > 1 and split[k][1] > 1]
    assert ks
    for k in ks:
        probe = Box(ops, dims, split, k, psi[k], None)
        K = rng.standard_normal((probe.Db, probe.dm_out, 2))
        box = Box(ops, dims, split, k, psi[k], K)
        L = rng.standard_normal((box.n_rows, 3))
        phi = rng.standard_normal((3, box.ds, 2))
        rhs = np.vdot(L, box.apply(site_cols(phi)))
        monkeypatch.setattr(RowOps, "med_left", wrong)
        lhs = np.vdot(probe.left(L, phi), K.reshape(-1, 2))
        monkeypatch.setattr(RowOps, "med_left", real)
        assert abs(lhs - rhs) > 1e-6 * (1 + abs(rhs))


def _chain_dense(chain):
    """Dense vector of a chain [matrix (rows x t) or site, site, ...]."""
    first = chain[0]
    v = first if first.ndim == 2 else first.reshape(-1, first.shape[2])
    for s in chain[1:]:
        Dl, d, Dr = s.shape
        v = (v @ s.reshape(Dl, d * Dr)).reshape(-1, Dr)
    return v.reshape(-1)


def _bottom(kind, kw, seed=3):
    net = _net(kind, kw, seed=51)
    r = net.R - 1
    psi0 = trivial_mps(net.phys_dims(r + 1)[0])
    return net, r, psi0


WINDOW_CASES = [("king", dict(R=2, C=4, a=2), 2), ("king", dict(R=2, C=4, a=2), 3),
                ("zephyr", dict(m=1, t=2), 3), ("zephyr", dict(m=1, t=2), 5),
                ("king", dict(R=2, C=5, a=1), 1)]


@pytest.mark.parametrize("kind,kw,chi", WINDOW_CASES)
def test_window_sweep_never_moves_away_from_the_stage_target(kind, kw, chi):
    net, r, psi0 = _bottom(kind, kw)
    exact, rec = {}, []
    zipper(net, r, psi0, Options(chi=256, cut=1e-14, power=2, var_window=0, var_sweeps=0),
           truncate=False, trace=lambda d: exact.__setitem__(d["k"], _chain_dense(d["chain"]))
           if d["stage"] == "zipper" else None)
    zipper(net, r, psi0, Options(chi=chi, cut=1e-14, power=1, var_window=2, var_sweeps=0, seed=4),
           truncate=True, trace=lambda d: rec.append((d["k"], d["stage"], _chain_dense(d["chain"]))))
    by_k = {}
    for k, stage, v in rec:
        by_k.setdefault(k, []).append((stage, np.linalg.norm(v - exact[k])))
    moved = 0
    for k, seq in by_k.items():
        scale = np.linalg.norm(exact[k])
        stages = [st for st, _ in seq]
        if len(seq) == 1:
            assert stages == ["zipper"] and k == max(by_k)
            continue
        assert stages == ["zipper", "window k+1", "window k"]
        d = [x for _, x in seq]
        assert d[1] <= d[0] + 1e-10 * scale, (k, d)
        assert d[2] <= d[1] + 1e-10 * scale, (k, d)
        moved += d[2] < d[0] - 1e-8 * scale
    assert len(by_k) == 2 * net.C - 1


def test_window_sweep_improves_a_randomized_stage():
    # at chi where the randomized range finder truncates, the window sweep
    # strictly reduces the distance at some zipper stage
    net, r, psi0 = _bottom("zephyr", dict(m=1, t=2))
    exact, rec = {}, []
    zipper(net, r, psi0, Options(chi=256, cut=1e-14, power=2, var_window=0, var_sweeps=0),
           truncate=False, trace=lambda d: exact.__setitem__(d["k"], _chain_dense(d["chain"]))
           if d["stage"] == "zipper" else None)
    zipper(net, r, psi0, Options(chi=3, cut=1e-14, power=0, width_extra=0, var_window=2, var_sweeps=0, seed=4),
           truncate=True, trace=lambda d: rec.append((d["k"], d["stage"], _chain_dense(d["chain"]))))
    gains = []
    for k in exact:
        ds = [np.linalg.norm(v - exact[k]) for kk, st, v in rec if kk == k]
        if len(ds) == 3:
            gains.append((ds[0] - ds[2]) / np.linalg.norm(exact[k]))
    assert max(gains) > 1e-6


SWEEP_CASES = [("king", dict(R=2, C=4, a=2), 2), ("zephyr", dict(m=1, t=2), 4),
               ("king", dict(R=2, C=5, a=1), 1), ("zephyr", dict(m=1, t=2), 2)]


@pytest.mark.parametrize("kind,kw,chi", SWEEP_CASES)
@pytest.mark.parametrize("window", [0, 2])
def test_full_sweeps_never_move_away_from_the_target(kind, kw, chi, window):
    net, r, psi0 = _bottom(kind, kw)
    ex, ln = zipper(net, r, psi0, Options(chi=256, cut=1e-14, power=2, var_window=0, var_sweeps=0),
                    truncate=False)
    target = _chain_dense(ex) * np.exp(ln)
    dist = []
    zipper(net, r, psi0, Options(chi=chi, cut=1e-14, power=1, var_window=window, var_sweeps=2, seed=9),
           truncate=True, trace=lambda d: dist.append(np.linalg.norm(_chain_dense(d["phi"]) - target))
           if d["stage"] == "sweep" else None)
    K = 2 * net.C - 1
    assert len(dist) == (2 * K - 1) + (2 * K - 2)
    scale = np.linalg.norm(target)
    for a, b in zip(dist[:-1], dist[1:]):
        assert b <= a + 1e-10 * scale


@pytest.mark.parametrize("kind,kw", [("king", dict(R=2, C=3, a=2)), ("zephyr", dict(m=1, t=2)),
                                     ("king", dict(R=3, C=3, a=1))])
def test_sweeps_are_a_no_op_when_the_stage_is_exact(kind, kw):
    net, r, psi0 = _bottom(kind, kw)
    a, la = zipper(net, r, psi0, Options(chi=256, cut=1e-14, var_window=0, var_sweeps=0))
    b, lb = zipper(net, r, psi0, Options(chi=256, cut=1e-14, var_window=2, var_sweeps=2))
    va, vb = _chain_dense(a) * np.exp(la), _chain_dense(b) * np.exp(lb)
    assert np.linalg.norm(va - vb) <= 1e-11 * np.linalg.norm(va)


@pytest.mark.parametrize("kind,kw", [("king", dict(R=4, C=4, a=1)), ("zephyr", dict(m=1, t=2)),
                                     ("king", dict(R=3, C=2, a=2))])
def test_variational_zipper_log_z_exact_when_untruncated(kind, kw):
    # full environment with every variational step switched on, chi large
    from oracle import ising
    from oracle.bmps import contract_env
    inst = make_instance(kind, 31, jdist="uniform", hdist="uniform0.1", **kw)
    env = contract_env(inst, 1.0, Options(chi=128, cut=1e-13, var_window=2, var_sweeps=2))
    bf = ising.brute_force(inst, 1.0)
    assert abs(env.logZ - bf["logZ"]) < 1e-9 * abs(bf["logZ"])
