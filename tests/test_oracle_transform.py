"""The eight lattice symmetries of the cluster lattice (Sec. V.A): they
relabel cluster positions only, so every exact quantity is unchanged."""
import numpy as np
import pytest

from tnb_inputs import make_instance, transform, transform_cells, N_TRANSFORMS
from oracle import ising
from oracle.bmps import contract_env, Options


def test_transforms_are_the_eight_symmetries():
    R, C = 3, 5
    seen = set()
    for t in range(N_TRANSFORMS):
        R2, C2, f = transform_cells(R, C, t)
        img = tuple(f(r, c) for r in range(R) for c in range(C))
        assert sorted(img) == sorted((a, b) for a in range(R2) for b in range(C2))   # a bijection
        # king neighbours stay king neighbours
        for r in range(R):
            for c in range(C):
                for dr in (-1, 0, 1):
                    for dc in (-1, 0, 1):
                        if 0 <= r + dr < R and 0 <= c + dc < C:
                            a, b = f(r, c), f(r + dr, c + dc)
                            assert max(abs(a[0] - b[0]), abs(a[1] - b[1])) == max(abs(dr), abs(dc))
        seen.add(img)
    assert len(seen) == N_TRANSFORMS
    # t = 0 is the identity and t = 2 (half turn) applied twice is too
    _, _, f0 = transform_cells(R, C, 0)
    _, _, f2 = transform_cells(R, C, 2)
    assert all(f0(r, c) == (r, c) and f2(*f2(r, c)) == (r, c) for r in range(R) for c in range(C))


@pytest.mark.parametrize("kind,kw", [("king", dict(R=3, C=2, a=2)), ("zephyr", dict(m=1, t=2))])
def test_exact_logz_is_invariant(kind, kw):
    inst = make_instance(kind, 41, jdist="uniform", hdist="uniform0.1", **kw)
    bf = ising.brute_force(inst, 1.0)["logZ"]
    for t in range(N_TRANSFORMS):
        ti = transform(inst, t)
        assert np.array_equal(ti.J, inst.J) and ti.n_spins == inst.n_spins
        z = contract_env(ti, 1.0, Options(chi=256, power=2, cut=1e-12)).logZ
        assert abs(z - bf) <= 1e-10 * abs(bf), (t, z, bf)
