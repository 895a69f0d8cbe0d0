"""The C-ABI library: builds, loads and exports every declared entry point
(no GPU needed), and rejects malformed input on the host."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tnbb.h")).read()
    return sorted(set(re.findall(r"\b(tnb_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2411_16431_amd as pk
    if not os.path.exists(pk.library_path()):
        pytest.skip("libtnbb.so not built")
    exported = set(pk.exported_symbols())
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing
    from paper_2411_16431_amd import _lib
    lib = _lib.lib()
    for name in _declared():
        assert hasattr(lib, name)


def test_header_declares_the_boundary_calls():
    decl = _declared()
    for name in ("tnb_build_clusters", "tnb_contract_env", "tnb_marginals", "tnb_branch_step",
                 "tnb_energies"):
        assert name in decl


def test_set_allocator_checks_its_argument_on_the_host():
    # installing or clearing an allocator touches no device
    import ctypes
    import paper_2411_16431_amd as pk
    if not os.path.exists(pk.library_path()):
        pytest.skip("libtnbb.so not built")
    from paper_2411_16431_amd import _lib
    lib = _lib.lib()
    half = _lib.TnbAllocator(_lib.ALLOC_FN(lambda n, u: None), ctypes.cast(None, _lib.RELEASE_FN), None)
    assert lib.tnb_set_allocator(ctypes.byref(half)) == -1     # TNB_EINVAL
    assert lib.tnb_set_allocator(None) == 0
