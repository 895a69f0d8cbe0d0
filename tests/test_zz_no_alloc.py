"""tnb_energies_noalloc (the instance staged in the library's static device
array instead of allocated buffers) against tnb_energies, through the C ABI:
two calls in a row, the second on a smaller instance and fewer states, every
energy equal bit for bit."""
import ctypes

import numpy as np
import pytest

from tnb_inputs import make_instance

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    from paper_2411_16431_amd import _lib as L
    from paper_2411_16431_amd.api import HostInstance, _stream
    return pk, torch, L, HostInstance, _stream


def _states(torch, n, K, seed):
    rng = np.random.default_rng(seed)
    s = np.where(rng.random((K, n)) < 0.5, -1, 1).astype(np.int8)
    return torch.from_numpy(s).cuda()


def test_noalloc_energies_equal_allocating_call_twice():
    pk, torch, L, HostInstance, _stream = _gpu()
    big = make_instance("zephyr", 501, jdist="uniform", hdist="uniform0.1", m=2, t=4)
    small = make_instance("king", 502, jdist="quarter", hdist="uniform0.1", R=3, C=3, a=2)
    assert small.n_spins < big.n_spins and len(small.J) < len(big.J)
    for inst, K, seed in ((big, 300, 1), (small, 7, 2)):
        S = _states(torch, inst.n_spins, K, seed)
        ref = pk.energies(inst, S)
        out = torch.full((K,), float("nan"), dtype=torch.float64, device="cuda")
        hi = HostInstance(inst)
        code = L.lib().tnb_energies_noalloc(ctypes.byref(hi.c), ctypes.c_void_p(S.data_ptr()), K,
                                            ctypes.c_void_p(out.data_ptr()), _stream())
        assert code == 0, L.lib().tnb_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (inst.n_spins, (out - ref).abs().max().item())


def test_noalloc_rejects_instance_beyond_staging_area():
    # 16 bytes per edge + 8 per spin above 2 MiB: refused on the host before any copy
    pk, torch, L, HostInstance, _stream = _gpu()
    inst = make_instance("chain", 503, jdist="uniform", hdist="uniform0.1", n=100000)
    S = torch.ones((1, inst.n_spins), dtype=torch.int8, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    hi = HostInstance(inst)
    code = L.lib().tnb_energies_noalloc(ctypes.byref(hi.c), ctypes.c_void_p(S.data_ptr()), 1,
                                        ctypes.c_void_p(out.data_ptr()), _stream())
    assert code == -5
    assert b"staging" in L.lib().tnb_last_error()
