"""ctypes declarations of include/tnbb.h (argument marshalling only)."""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtnbb.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P = ctypes.POINTER


class TnbInstance(ctypes.Structure):
    _fields_ = [("n_spins", c_int32), ("n_edges", c_int32),
                ("edge_i", P(c_int32)), ("edge_j", P(c_int32)),
                ("J", P(c_double)), ("h", P(c_double)),
                ("rows", c_int32), ("cols", c_int32), ("cell_of", P(c_int32))]


class TnbEnvOpts(ctypes.Structure):
    _fields_ = [("chi", c_int32), ("sketch_extra", c_int32), ("power_iters", c_int32),
                ("cut", c_double), ("seed", ctypes.c_uint64), ("var_window", c_int32),
                ("var_sweeps", c_int32), ("prec", c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class TnbDropletOpts(ctypes.Structure):
    _fields_ = [("max_droplets", c_int32), ("max_losers", c_int32), ("min_hamming", c_int32),
                ("max_cells", c_int32), ("max_dE", ctypes.c_double), ("connected_only", c_int32)]


class TnbAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "tnb_energies": (c_int32, [P(TnbInstance), c_void_p, c_int64, c_void_p, c_void_p]),
    "tnb_energies_noalloc": (c_int32, [P(TnbInstance), c_void_p, c_int64, c_void_p, c_void_p]),
    "tnb_build_clusters": (c_int32, [P(TnbInstance), c_double, c_void_p, P(c_void_p)]),
    "tnb_cluster_energies": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_void_p]),
    "tnb_bond_energies": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int64, P(c_int32),
                                    P(c_int32), c_void_p]),
    "tnb_contract_env": (c_int32, [c_void_p, P(TnbEnvOpts), c_void_p, P(c_void_p), P(c_double)]),
    "tnb_env_site_shape": (c_int32, [c_void_p, c_int32, c_int32, P(c_int32), P(c_int32), P(c_int32)]),
    "tnb_diagram_dims": (c_int32, [c_void_p, c_int32, c_int32, P(c_int32), P(c_int32), P(c_int32),
                                   P(c_int32)]),
    "tnb_diagram_apply": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_int32, c_int32,
                                    c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_int64, c_void_p]),
    "tnb_beam_create": (c_int32, [c_void_p, c_int32, P(c_void_p)]),
    "tnb_beam_info": (c_int32, [c_void_p, P(c_int32), P(c_int32), P(c_int32)]),
    "tnb_marginals": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_void_p]),
    "tnb_branch_step": (c_int32, [c_void_p, P(c_double), c_void_p]),
    "tnb_beam_export": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, P(c_int32), c_void_p]),
    "tnb_beam_lowest": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, P(c_int32), c_void_p]),
    "tnb_beam_droplets_enable": (c_int32, [c_void_p, P(TnbDropletOpts)]),
    "tnb_env_logz": (c_int32, [c_void_p, P(ctypes.c_double), P(c_int32)]),
    "tnb_lbp_marginals": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.c_int64, P(ctypes.c_double), c_void_p]),
    "tnb_reduce_clusters": (c_int32, [c_void_p, c_int32, c_int32, c_void_p]),
    "tnb_beam_droplets": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, P(c_int32), c_void_p]),
    "tnb_select_lowest": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, P(c_int32),
                                    c_void_p]),
    "tnb_row_layout": (c_int32, [c_void_p, P(c_int32), P(c_int32), c_void_p, c_void_p, c_int32]),
    "tnb_row_moments": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
    "tnb_row_moments_per_branch": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "tnb_autotune": (c_int32, [c_int32, ctypes.c_char_p]),
    "tnb_profile_enable": (c_int32, [c_int32]),
    "tnb_profile_query": (c_int32, [ctypes.c_char_p, P(c_double), P(c_int64), P(c_double), P(c_double)]),
    "tnb_profile_names": (c_int32, [ctypes.c_char_p, c_int64]),
    "tnb_set_allocator": (c_int32, [P(TnbAllocator)]),
    "tnb_destroy": (None, [c_void_p]),
    "tnb_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtnbb.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib
