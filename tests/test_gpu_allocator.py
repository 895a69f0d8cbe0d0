"""Device memory through the caller's allocator (tnb_set_allocator): the same
results as with hipMalloc, every block given back, and hipMalloc restored."""
import gc

import numpy as np
import pytest

from tnb_inputs import make_instance

pytestmark = pytest.mark.gpu


def _run(pk, inst, var):
    cl = pk.Clusters(inst, 1.0)
    env = pk.Env(cl, pk.EnvOptions(chi=8, power_iters=2, seed=5, var_window=2 if var else 0,
                                   var_sweeps=1 if var else 0))
    beam = pk.Beam(env, 16)
    for _ in range(inst.R * inst.C):
        beam.step()
    st, E = beam.lowest(4, inst.n_spins)
    out = (env.logZ, E.cpu().numpy().copy(), st.cpu().numpy().copy())
    del beam, env, cl
    gc.collect()
    return out


@pytest.mark.parametrize("var", [False, True])
def test_torch_allocator_gives_the_same_results(var):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    inst = make_instance("zephyr", 305, jdist="quarter", hdist="uniform0.1", m=1, t=2)
    ref = _run(pk, inst, var)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    count = pk.use_torch_allocator()
    try:
        got = _run(pk, inst, var)
        torch.cuda.synchronize()
    finally:
        pk.use_torch_allocator(False)
    assert count["alloc"] > 0 and count["release"] == count["alloc"]
    assert torch.cuda.memory_allocated() == base
    assert got[0] == ref[0]
    np.testing.assert_array_equal(got[1], ref[1])
    np.testing.assert_array_equal(got[2], ref[2])
    # hipMalloc again after the restore: the counters stay where they were
    n = count["alloc"]
    again = _run(pk, inst, var)
    assert count["alloc"] == n and again[0] == ref[0]
