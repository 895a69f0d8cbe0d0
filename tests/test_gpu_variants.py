"""Every launch variant of the mediating diagram's binned stage (the
autotuner's candidates) against the oracle: forced one at a time through a
tuning table, on the Zephyr Z_2 t=2 diagrams in full and on the central
diagram of Z_2 t=4 (legs 65536 x 65536, the benchmark's launch shape) against
the default variant, whose sampled rows the diagram tests compare with the
oracle.  The binned variants differ in tiling only; the grouped ones sum the
items of a weight group first, so they agree up to rounding (1e-12)."""
import json

import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle.bmps import Network, RowOps

pytestmark = pytest.mark.gpu

CHI_B, DG, S = 16, 32, 40
TOL = 1e-12
N_VARIANTS = 5   # binned with 1, 2, 3 column tiles; grouped with 1, 2


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk, torch


@pytest.fixture(autouse=True)
def _default_variants():
    yield
    import paper_2411_16431_amd as pk
    pk.autotune(False, None)   # later tests run the default variants


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


def _inputs(pk, cl, r, k, seed):
    dm_in, dm_out, ds, dsb = pk.diagram_dims(cl, r, k)
    rng = np.random.default_rng(seed)
    return dict(A=rng.standard_normal((dsb, CHI_B, CHI_B)), K=rng.standard_normal((dm_out, CHI_B, DG)),
                X=rng.standard_normal((ds, DG, S)), Y=rng.standard_normal((dm_in, CHI_B, S)),
                L=rng.standard_normal((dm_in, CHI_B, DG)), phi=rng.standard_normal((ds, DG, DG)))


def _run_all(pk, torch, cl, r, k, t):
    A = _dev(torch, t["A"])
    return [pk.diagram_apply(cl, r, k, 0, A, _dev(torch, t["K"]), _dev(torch, t["X"])).cpu().numpy(),
            pk.diagram_apply(cl, r, k, 1, A, _dev(torch, t["K"]), _dev(torch, t["Y"])).cpu().numpy(),
            pk.diagram_apply(cl, r, k, 2, A, _dev(torch, t["L"]), _dev(torch, t["phi"])).cpu().numpy()]


def _each_variant(pk, tmp_path, record):
    """Yield v after installing a table that forces variant v on every shape
    `record` launches (shapes with fewer candidates keep their default)."""
    path = str(tmp_path / "tune.json")
    pk.autotune(True, path)
    try:
        record()
        keys = list(json.load(open(path)))
        assert keys
        for v in range(N_VARIANTS):
            with open(path, "w") as fh:
                json.dump({key: v for key in keys}, fh)
            pk.autotune(False, path)
            yield v
    finally:
        pk.autotune(False, None)


@pytest.mark.parametrize("r,k", [(1, 3), (2, 3), (1, 5)])
def test_every_variant_matches_oracle_small(tmp_path, r, k):
    pk, torch = _gpu()
    inst = make_instance("zephyr", 1000, jdist="uniform", hdist="uniform0.1", m=2, t=2)
    net = Network(inst, 1.0)
    cl = pk.Clusters(inst, 1.0)
    ops = RowOps(net, r)
    t = _inputs(pk, cl, r, k, 40 + 10 * r + k)
    c = (k - 1) // 2
    da, db = net.phys_dims(r)[1][k]
    A_o = t["A"].transpose(1, 0, 2)
    K_o = t["K"].transpose(1, 0, 2)
    refs = (ops.med_apply(c, A_o, K_o, t["X"].reshape(db, da, DG, S).transpose(1, 0, 2, 3)).transpose(1, 0, 2),
            ops.med_applyT(c, A_o, K_o, t["Y"].transpose(1, 0, 2)).transpose(1, 0, 2, 3).reshape(t["X"].shape),
            ops.med_left(c, A_o, t["L"].transpose(1, 0, 2), t["phi"].transpose(1, 0, 2)).transpose(1, 0, 2))
    for v in _each_variant(pk, tmp_path, lambda: _run_all(pk, torch, cl, r, k, t)):
        for mode, (got, ref) in enumerate(zip(_run_all(pk, torch, cl, r, k, t), refs)):
            assert _rel(got, ref) <= TOL, (v, mode, _rel(got, ref))


def test_every_variant_agrees_at_full_size(tmp_path):
    pk, torch = _gpu()
    inst = make_instance("zephyr", 1000, jdist="uniform", hdist="uniform0.1", m=2, t=4)
    cl = pk.Clusters(inst, 1.0)
    r, k = 1, 3
    t = _inputs(pk, cl, r, k, 77)
    base = _run_all(pk, torch, cl, r, k, t)    # the default variant
    for v in _each_variant(pk, tmp_path, lambda: _run_all(pk, torch, cl, r, k, t)):
        got = _run_all(pk, torch, cl, r, k, t)
        for mode in range(3):
            assert _rel(got[mode], base[mode]) <= TOL, (v, mode, _rel(got[mode], base[mode]))


def test_binned_variants_identical_with_item_split(tmp_path):
    # row 1, diagram k = 1 of Zephyr Z_2 t=4 (legs 4096 x 4096): few output
    # blocks, so the binned stage splits each class's items over workgroups.
    # The split does not depend on the variant: the binned variants (0..2)
    # agree bit for bit, the grouped ones (3, 4) up to rounding, and the
    # default variant's apply matches the oracle on sampled rows.
    pk, torch = _gpu()
    inst = make_instance("zephyr", 1000, jdist="uniform", hdist="uniform0.1", m=2, t=4)
    net = Network(inst, 1.0)
    cl = pk.Clusters(inst, 1.0)
    r, k = 1, 1
    t = _inputs(pk, cl, r, k, 91)
    outs = {}
    for v in _each_variant(pk, tmp_path, lambda: _run_all(pk, torch, cl, r, k, t)):
        outs[v] = _run_all(pk, torch, cl, r, k, t)
    for v in (1, 2):
        for mode in range(3):
            assert np.array_equal(outs[v][mode], outs[0][mode]), (v, mode)
    for v in (3, 4):
        for mode in range(3):
            assert _rel(outs[v][mode], outs[0][mode]) <= TOL, (v, mode, _rel(outs[v][mode], outs[0][mode]))
    ops = RowOps(net, r)
    da, db = net.phys_dims(r)[1][k]
    X_o = t["X"].reshape(db, da, DG, S).transpose(1, 0, 2, 3)
    rhos = np.array([0, 1, 2047, 4095])
    ref = ops.med_apply((k - 1) // 2, t["A"].transpose(1, 0, 2), t["K"].transpose(1, 0, 2), X_o, rhos=rhos)
    assert _rel(outs[0][0][rhos], ref.transpose(1, 0, 2)) <= TOL


def test_eigen_and_svd_launch_widths_agree(tmp_path):
    # the LDS eigensolver and one-sided Jacobi SVD of the Gram path (the
    # 2^16-state clusters of Zephyr t=4) at 16 and at 4 waves: the same
    # boundary MPSs up to rounding, on a planted instance whose truncation is
    # well conditioned
    import json
    pk, torch = _gpu()
    from tnb_inputs import planted_loops
    inst, _, _ = planted_loops(2, 4, 91, loops_per_cell=2)
    cl = pk.Clusters(inst, 1.0)
    base = pk.Env(cl, pk.EnvOptions(chi=16)).logZ
    path = str(tmp_path / "w.json")
    pk.autotune(True, path)
    pk.Env(cl, pk.EnvOptions(chi=16))
    keys = [k for k in json.load(open(path)) if k.startswith(("eigh", "hestenes"))]
    assert keys
    with open(path, "w") as fh:
        json.dump({k: 1 for k in keys}, fh)
    pk.autotune(False, path)
    four = pk.Env(cl, pk.EnvOptions(chi=16)).logZ
    assert abs(four - base) <= 1e-10 * abs(base)
