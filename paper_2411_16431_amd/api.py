"""Python face of libtnbb: numpy/torch arrays in, handles and tensors out.

Device memory comes from torch (the caller's tensors) and work is queued on
torch's current stream; every computation runs inside libtnbb.
"""
import ctypes
import math
import re
import subprocess
from dataclasses import dataclass

import numpy as np

from . import _lib as L


class TnbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libtnbb status %d: %s" % (code, msg))
        self.code = code


def _check(code):
    if code != 0:
        raise TnbError(code, L.lib().tnb_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def library_path():
    return L.LIB_PATH


def exported_symbols():
    """Dynamic symbols exported by libtnbb.so whose name starts with tnb_."""
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return sorted(set(re.findall(r"\b(tnb_[a-z_]+)\b", out)))


class HostInstance:
    """Keeps the host arrays of an instance alive for a C call."""

    def __init__(self, inst):
        self.ei = np.ascontiguousarray(inst.edges[:, 0], dtype=np.int32)
        self.ej = np.ascontiguousarray(inst.edges[:, 1], dtype=np.int32)
        self.J = np.ascontiguousarray(inst.J, dtype=np.float64)
        self.h = np.ascontiguousarray(inst.h, dtype=np.float64)
        self.cell = np.ascontiguousarray(inst.cell_of, dtype=np.int32)
        ip = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
        self.c = L.TnbInstance(int(inst.n_spins), len(self.J), ip(self.ei, ctypes.c_int32),
                               ip(self.ej, ctypes.c_int32), ip(self.J, ctypes.c_double),
                               ip(self.h, ctypes.c_double), int(inst.R), int(inst.C),
                               ip(self.cell, ctypes.c_int32))


def energies(inst, states):
    """Eq. (1) on the device; states: torch int8 cuda tensor [K, N] of +-1."""
    import torch
    K = states.shape[0]
    out = torch.empty(K, dtype=torch.float64, device=states.device)
    hi = HostInstance(inst)
    _check(L.lib().tnb_energies(ctypes.byref(hi.c), ctypes.c_void_p(states.data_ptr()), K,
                                ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


class _Handle:
    _h = None

    def close(self):
        if self._h:
            L.lib().tnb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Clusters(_Handle):
    """tnb_build_clusters: local tables, projectors, bond tables, weights."""

    def __init__(self, inst, beta):
        self.inst, self.beta = inst, beta
        hi = HostInstance(inst)
        h = ctypes.c_void_p()
        _check(L.lib().tnb_build_clusters(ctypes.byref(hi.c), float(beta), _stream(), ctypes.byref(h)))
        self._h = h

    def lbp_marginals(self, iters):
        """tnb_lbp_marginals: (list of per-cluster belief tensors, largest
        message change of the last iteration)."""
        import torch
        ks = np.bincount(np.asarray(self.inst.cell_of), minlength=self.inst.R * self.inst.C)
        sizes = [1 << int(k) for k in ks]
        p = torch.empty(sum(sizes), dtype=torch.float64, device="cuda")
        ch = ctypes.c_double()
        _check(L.lib().tnb_lbp_marginals(self._h, int(iters), ctypes.c_void_p(p.data_ptr()), p.numel(),
                                         ctypes.byref(ch), _stream()))
        return list(torch.split(p, sizes)), ch.value

    def reduce(self, keep, iters):
        """tnb_reduce_clusters: keep the `keep` most probable states of every
        cluster by LBP beliefs; the others get weight 0 (Sec. IV)."""
        _check(L.lib().tnb_reduce_clusters(self._h, int(keep), int(iters), _stream()))

    def local_energy(self, n):
        import torch
        k = int(np.sum(np.asarray(self.inst.cell_of) == n))
        out = torch.empty(1 << k, dtype=torch.float64, device="cuda")
        _check(L.lib().tnb_cluster_energies(self._h, n, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                            _stream()))
        return out

    def bond_energy(self, m, n):
        import torch
        r, c = ctypes.c_int32(), ctypes.c_int32()
        code = L.lib().tnb_bond_energies(self._h, m, n, None, 0, ctypes.byref(r), ctypes.byref(c),
                                         _stream())
        out = torch.empty(r.value * c.value, dtype=torch.float64, device="cuda")
        _check(L.lib().tnb_bond_energies(self._h, m, n, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                         ctypes.byref(r), ctypes.byref(c), _stream()))
        return out.reshape(r.value, c.value)


PRECS = {"f64": 0, "f32": 1}
MARG_MODES = {"vector": 0, "spin": 1, "adjoint": 2}


@dataclass
class EnvOptions:
    chi: int = 16
    sketch_extra: int = 8
    power_iters: int = 2
    cut: float = 1e-6
    seed: int = 12345
    var_window: int = 2
    var_sweeps: int = 1
    prec: str = "f64"      # "f64" or "f32": arithmetic of the diagram contractions

    def c(self):
        return L.TnbEnvOpts(self.chi, self.sketch_extra, self.power_iters, self.cut, self.seed,
                            self.var_window, self.var_sweeps, PRECS[self.prec])


class Env(_Handle):
    """tnb_contract_env: boundary MPSs and log Z."""

    def __init__(self, clusters, opts):
        self.clusters = clusters
        h = ctypes.c_void_p()
        lz = ctypes.c_double()
        o = opts.c()
        _check(L.lib().tnb_contract_env(clusters._h, ctypes.byref(o), _stream(), ctypes.byref(h),
                                        ctypes.byref(lz)))
        self._h = h
        self.logZ = lz.value
        sg = ctypes.c_int32()
        _check(L.lib().tnb_env_logz(self._h, None, ctypes.byref(sg)))
        self.sign = sg.value   # sign of the approximate Z (log Z is log |Z|)

    def site_shape(self, r, k):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.lib().tnb_env_site_shape(self._h, r, k, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value


class Beam(_Handle):
    """tnb_beam_create / tnb_marginals / tnb_branch_step / tnb_beam_export."""

    def __init__(self, env, M):
        self.env = env
        h = ctypes.c_void_p()
        _check(L.lib().tnb_beam_create(env._h, int(M), ctypes.byref(h)))
        self._h = h

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.lib().tnb_beam_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def enable_droplets(self, max_droplets=16, max_losers=8, min_hamming=1, max_cells=64, max_dE=math.inf,
                        connected_only=True):
        """tnb_beam_droplets_enable: keep the excitations the boundary merge
        finds above every branch (before the first step)."""
        o = L.TnbDropletOpts(int(max_droplets), int(max_losers), int(min_hamming), int(max_cells), float(max_dE),
                             1 if connected_only else 0)
        _check(L.lib().tnb_beam_droplets_enable(self._h, ctypes.byref(o)))

    def droplets(self, i, n_spins, max_count=16):
        """tnb_beam_droplets: (states int8 [k, N], dE [k]) of branch i."""
        import torch
        st = torch.empty((max(max_count, 1), n_spins), dtype=torch.int8, device="cuda")
        dE = torch.empty(max(max_count, 1), dtype=torch.float64, device="cuda")
        cnt = ctypes.c_int32()
        _check(L.lib().tnb_beam_droplets(self._h, int(i), int(max_count), ctypes.c_void_p(st.data_ptr()),
                                         ctypes.c_void_p(dE.data_ptr()), ctypes.byref(cnt), _stream()))
        return st[:cnt.value], dE[:cnt.value]

    def marginals(self, mode="vector"):
        """tnb_marginals: 'vector' p_b(x) [parents, d]; 'spin' <s_i>_b of the
        next cluster [parents, k]; 'adjoint' <s_i>_b of the unfixed row spins
        [parents, len(row_layout()[0])]."""
        import torch
        _, npar, d = self.info()
        if mode == "vector":
            cols = d
        elif mode == "spin":
            cols = int(round(math.log2(d)))
        else:
            cols = len(self.row_layout()[0])
        out = torch.empty((npar, max(cols, 1)), dtype=torch.float64, device="cuda")
        _check(L.lib().tnb_marginals(self._h, MARG_MODES[mode], ctypes.c_void_p(out.data_ptr()), out.numel(),
                                     _stream()))
        return out[:, :cols]

    def step(self):
        pd = ctypes.c_double()
        _check(L.lib().tnb_branch_step(self._h, ctypes.byref(pd), _stream()))
        return pd.value

    def row_layout(self):
        """(spins, edges) of the row moments at the current step (numpy int32)."""
        ns, ne = ctypes.c_int32(), ctypes.c_int32()
        _check(L.lib().tnb_row_layout(self._h, ctypes.byref(ns), ctypes.byref(ne), None, None, 0))
        cap = max(ns.value, ne.value, 1)
        sp = np.zeros(cap, dtype=np.int32)
        ed = np.zeros(cap, dtype=np.int32)
        _check(L.lib().tnb_row_layout(self._h, ctypes.byref(ns), ctypes.byref(ne),
                                      sp.ctypes.data_as(ctypes.c_void_p), ed.ctypes.data_as(ctypes.c_void_p), cap))
        return sp[:ns.value], ed[:ne.value]

    def row_moments(self, edges=True):
        """Adjoint row moments: (m1 [parents, spins], m2 [parents, edges] or None)."""
        import torch
        _, npar, _ = self.info()
        sp, ed = self.row_layout()
        m1 = torch.empty((npar, len(sp)), dtype=torch.float64, device="cuda")
        m2 = torch.empty((npar, len(ed)), dtype=torch.float64, device="cuda") if edges else None
        _check(L.lib().tnb_row_moments(self._h, ctypes.c_void_p(m1.data_ptr()), m1.numel(),
                                       ctypes.c_void_p(m2.data_ptr()) if m2 is not None else None,
                                       m2.numel() if m2 is not None else 0, _stream()))
        return m1, m2

    def row_moments_per_branch(self):
        """<s_i>_b of the same layout by one clamped contraction per branch."""
        import torch
        _, npar, _ = self.info()
        sp, _ = self.row_layout()
        m1 = torch.empty((npar, len(sp)), dtype=torch.float64, device="cuda")
        _check(L.lib().tnb_row_moments_per_branch(self._h, ctypes.c_void_p(m1.data_ptr()), m1.numel(), _stream()))
        return m1

    def lowest(self, K, n_spins):
        """tnb_beam_lowest: (states int8 [k, N], energies [k]) of a finished beam."""
        import torch
        st = torch.empty((max(K, 1), n_spins), dtype=torch.int8, device="cuda")
        E = torch.empty(max(K, 1), dtype=torch.float64, device="cuda")
        cnt = ctypes.c_int32()
        _check(L.lib().tnb_beam_lowest(self._h, int(K), ctypes.c_void_p(st.data_ptr()),
                                       ctypes.c_void_p(E.data_ptr()), ctypes.byref(cnt), _stream()))
        return st[:cnt.value], E[:cnt.value]

    def export(self, K, n_spins):
        import torch
        st = torch.empty((K, n_spins), dtype=torch.int8, device="cuda")
        lp = torch.empty(K, dtype=torch.float64, device="cuda")
        cnt = ctypes.c_int32()
        _check(L.lib().tnb_beam_export(self._h, int(K), ctypes.c_void_p(st.data_ptr()),
                                       ctypes.c_void_p(lp.data_ptr()), ctypes.byref(cnt), _stream()))
        return st[:cnt.value], lp[:cnt.value]


def diagram_dims(clusters, r, k):
    """(dm_in, dm_out, ds, ds_below) of the box at site k of row r (tnb_diagram_dims)."""
    a, b, c, d = (ctypes.c_int32() for _ in range(4))
    _check(L.lib().tnb_diagram_dims(clusters._h, int(r), int(k), ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c), ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def diagram_apply(clusters, r, k, mode, A, K, X, prec="f64"):
    """tnb_diagram_apply on float64 cuda tensors: A [ds_below][Da][Db],
    K [dm_out][Db][Dg] (modes 0, 1) or [dm_in][Da][Dg] (mode 2), X as in the
    header; returns the output tensor."""
    import torch
    dm_in, dm_out, ds, _ = diagram_dims(clusters, r, k)
    Da, Db = A.shape[1], A.shape[2]
    Dg = K.shape[2]
    if mode == 0:
        s = X.shape[2]
        shape = (dm_in, Da, s)
    elif mode == 1:
        s = X.shape[2]
        shape = (ds, Dg, s)
    else:
        s = X.shape[2]
        shape = (dm_out, Db, s)
    for t in (A, K, X):
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    out = torch.empty(shape, dtype=torch.float64, device=A.device)
    _check(L.lib().tnb_diagram_apply(clusters._h, int(r), int(k), int(mode), PRECS[prec], ctypes.c_void_p(A.data_ptr()),
                                     int(Da), int(Db), ctypes.c_void_p(K.data_ptr()), int(Dg),
                                     ctypes.c_void_p(X.data_ptr()), int(s), ctypes.c_void_p(out.data_ptr()),
                                     out.numel(), _stream()))
    return out


def solve(inst, beta, chi, M, K=8, droplets=None, **env_kw):
    """Whole pipeline on the device: clusters, boundary MPSs, every beam step,
    export of the final candidates and their energies; returns the K lowest.
    droplets: keyword arguments of Beam.enable_droplets; the excitations of
    the branch that holds the lowest energy are then returned as
    "droplet_states" / "droplet_dE" (Fig. 4)."""
    import torch
    cl = Clusters(inst, beta)
    env = Env(cl, EnvOptions(chi=chi, **env_kw))
    beam = Beam(env, M)
    if droplets is not None:
        beam.enable_droplets(**droplets)
    n_steps = inst.R * inst.C
    pd = -math.inf
    marg = 0
    for _ in range(n_steps):
        _, npar, d = beam.info()
        marg += npar * int(round(math.log2(d)))
        pd = beam.step()
    states, E = beam.lowest(K, inst.n_spins)
    out = dict(states=states.cpu().numpy(), energies=E.cpu().numpy(), logZ=env.logZ, p_d_log=pd, env=env,
               beam=beam, spin_marginals=marg)
    if droplets is not None:
        npar = beam.info()[1]
        fin, _ = beam.export(npar, inst.n_spins)
        best = int(torch.argmin(energies(inst, fin)).item())   # first branch of lowest energy
        ds, dE = beam.droplets(best, inst.n_spins, droplets.get("max_droplets", 16))
        out["droplet_states"], out["droplet_dE"] = ds.cpu().numpy(), dE.cpu().numpy()
    return out


def solve_batch(instances, beta, chi, M, K=8, workers=None, **env_kw):
    """solve() for several instances at once: each runs on its own host thread
    and its own stream, so the kernels of different instances (short, launch-
    bound ones above all) overlap on the device.  Results are those of
    solve() one by one, in the order of `instances`."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    workers = workers or min(len(instances), 8)
    dev = torch.cuda.current_device()

    def run(inst):
        torch.cuda.set_device(dev)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            out = solve(inst, beta, chi, M, K, **env_kw)
        s.synchronize()
        return out

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(run, instances))


_ALLOC_KEEP = []


def use_torch_allocator(on=True):
    """Route the library's device memory through PyTorch's caching allocator
    (tnb_set_allocator), on the current device and stream; on=False restores
    hipMalloc.  Returns the number of allocations made through it so far
    through the returned counter dict (tests)."""
    import torch
    if not on:
        _check(L.lib().tnb_set_allocator(None))
        return None
    count = {"alloc": 0, "release": 0}

    def _alloc(nbytes, user):
        count["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  torch.cuda.current_stream())

    def _release(ptr, user):
        count["release"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    a = L.TnbAllocator(L.ALLOC_FN(_alloc), L.RELEASE_FN(_release), None)
    _ALLOC_KEEP.append((a, _alloc, _release))   # the library may call them until the process ends
    _check(L.lib().tnb_set_allocator(ctypes.byref(a)))
    return count


def autotune(measure, path=None):
    """tnb_autotune: measure (True) or reuse (False) the fastest launch
    variant per shape; path: JSON cache of the choices."""
    _check(L.lib().tnb_autotune(1 if measure else 0, path.encode() if path else None))


def select_lowest(states, E, K):
    """tnb_select_lowest on cuda tensors: the K lowest distinct of the given
    configurations (int8 [n, N]) and energies ([n]), by energy then spin vector."""
    import torch
    n, N = states.shape
    out = torch.empty((max(K, 1), N), dtype=torch.int8, device=states.device)
    Eo = torch.empty(max(K, 1), dtype=torch.float64, device=states.device)
    cnt = ctypes.c_int32()
    _check(L.lib().tnb_select_lowest(ctypes.c_void_p(states.data_ptr()), ctypes.c_void_p(E.data_ptr()), int(n),
                                     int(N), int(K), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(Eo.data_ptr()),
                                     ctypes.byref(cnt), _stream()))
    return out[:cnt.value], Eo[:cnt.value]


def solve_transformed(inst, beta, chi, M, K=8, transforms=range(8), **env_kw):
    """The method on each lattice symmetry of the instance (Sec. V.A: the
    search runs row by row in a fixed direction, so the eight orientations of
    the cluster lattice give different approximations), with the K lowest
    distinct states pooled over all runs.  Returns the pooled states and
    energies, log Z per transformation and its spread (max - min, zero for an
    exact contraction), and each run's best energy."""
    import torch
    from tnb_inputs import transform
    S, E, logz, best = [], [], {}, {}
    for t in transforms:
        res = solve(transform(inst, t), beta, chi, M, K, **env_kw)
        S.append(torch.from_numpy(res["states"]).cuda())
        E.append(torch.from_numpy(res["energies"]).cuda())
        logz[t], best[t] = res["logZ"], float(res["energies"][0])
    st, en = select_lowest(torch.cat(S).contiguous(), torch.cat(E).contiguous(), K)
    vals = list(logz.values())
    return dict(states=st.cpu().numpy(), energies=en.cpu().numpy(), logZ=logz, logZ_spread=max(vals) - min(vals),
                best_energy=best)


def first_row_layout(inst, beta=1.0):
    """(spins, edges) of the first row of clusters: the inputs of FirstRowLogZ."""
    env = Env(Clusters(inst, beta), EnvOptions(chi=1))
    return Beam(env, 1).row_layout()


def _first_row_logz_and_moments(inst, beta, opts, h_row, J_row, spins, edges):
    import copy
    k = copy.copy(inst)
    k.h = np.array(inst.h, dtype=np.float64, copy=True)
    k.J = np.array(inst.J, dtype=np.float64, copy=True)
    k.h[spins] = h_row
    k.J[edges] = J_row
    env = Env(Clusters(k, beta), opts)
    m1, m2 = Beam(env, 1).row_moments()
    return env.logZ, m1[0], m2[0]


class FirstRowLogZ:
    """log Z of an instance as a function of the fields and intra-cluster
    couplings of its first row of clusters (Eq. 10), with a hand-written
    backward: the adjoint of the row contraction gives
    d log Z / d h_i = -beta <s_i> and d log Z / d J_ij = -beta <s_i s_j>
    (tnb_row_moments at the first step).  The boundary MPS below the first row
    does not depend on these inputs, so the gradient is complete for them.

    apply(h_row, J_row, inst, beta, opts) with h_row, J_row float64 tensors in
    the order of first_row_layout(inst)."""

    @staticmethod
    def apply(h_row, J_row, inst, beta, opts):
        return _first_row_fn().apply(h_row, J_row, inst, beta, opts)


_FN = None


def _first_row_fn():
    global _FN
    if _FN is None:
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, h_row, J_row, inst, beta, opts):
                spins, edges = first_row_layout(inst, beta)
                if h_row.numel() != len(spins) or J_row.numel() != len(edges):
                    raise ValueError("h_row/J_row must follow first_row_layout(inst)")
                lz, m1, m2 = _first_row_logz_and_moments(inst, beta, opts, h_row.detach().cpu().numpy(),
                                                         J_row.detach().cpu().numpy(), spins, edges)
                ctx.beta = float(beta)
                ctx.save_for_backward(m1.to(h_row.device), m2.to(J_row.device))
                return torch.tensor(lz, dtype=torch.float64, device=h_row.device)

            @staticmethod
            def backward(ctx, g):
                m1, m2 = ctx.saved_tensors
                return -ctx.beta * g * m1, -ctx.beta * g * m2, None, None, None

        _FN = _F
    return _FN


def profile_enable(on=True):
    """Start (clearing earlier records) or stop per-kernel event timing."""
    _check(L.lib().tnb_profile_enable(1 if on else 0))


def profile_query(name):
    """(total_ms, launches, flops, bytes) of one instrumented kernel."""
    ms, n, fl, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(L.lib().tnb_profile_query(name.encode(), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                     ctypes.byref(by)))
    return ms.value, n.value, fl.value, by.value


def profile_names():
    buf = ctypes.create_string_buffer(4096)
    _check(L.lib().tnb_profile_names(buf, 4096))
    return [x for x in buf.value.decode().split(",") if x]
