"""Several instances solved at once (solve_batch: one host thread and one
stream per instance) give exactly the results of solving them one by one."""
import numpy as np
import pytest

from tnb_inputs import planted_king, make_instance

pytestmark = pytest.mark.gpu


def test_batch_equals_one_by_one():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    insts = [planted_king(8, 8, 1, s)[0] for s in (3, 4, 5)]
    insts.append(make_instance("zephyr", 7, jdist="uniform", hdist="uniform0.1", m=1, t=2))
    one = [pk.solve(i, 2.0, 16, 32, K=4) for i in insts]
    many = pk.solve_batch(insts, 2.0, 16, 32, K=4, workers=4)
    for a, b in zip(one, many):
        assert a["logZ"] == b["logZ"]
        np.testing.assert_array_equal(a["states"], b["states"])
        np.testing.assert_array_equal(a["energies"], b["energies"])
