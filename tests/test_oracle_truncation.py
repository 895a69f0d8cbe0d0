"""Truncated boundary MPS of the oracle against the mathematics of MPS
truncation (Sec. III.B, "Variational zipper algorithm for boundary MPS", Fig. 8).

The zipper first compresses T_r Psi_{r+1} to bond 2 chi.  Where that stage is
exact, its result is right-canonical, and the left-to-right SVD sweep down to
chi is the TT-SVD of the exact state.  Two bounds then fix the distance of the
truncated state from the exact one, with eps_k the best rank-chi error of the
k-th unfolding of the exact state:
  - upper (TT-SVD, Oseledets 2011, Thm. 2.2): ||Psi_chi - Psi|| <= sqrt(sum_k eps_k^2);
  - lower (Eckart-Young): any MPS of bond <= chi is at least max_k eps_k away.
The lower bound holds in every regime, including where the randomized stage
truncates too.  The exact state is the untruncated zipper, whose log Z is
pinned to brute force elsewhere; the unfoldings are plain numpy SVDs.
"""
import numpy as np
import pytest

from tnb_inputs import make_instance
from oracle.bmps import Network, Options, trivial_mps, zipper


def _dense(sites):
    v = np.ones((1, 1))
    for s in sites:
        Dl, d, Dr = s.shape
        v = (v @ s.reshape(Dl, d * Dr)).reshape(-1, Dr)
    return v.reshape(-1)


def _bottom_row(kind, kw, chi, truncate, seed=3):
    inst = make_instance(kind, 51, jdist="uniform", hdist="uniform0.1", **kw)
    net = Network(inst, 1.0)
    r = net.R - 1
    psi0 = trivial_mps(net.phys_dims(r + 1)[0])
    sites, ln = zipper(net, r, psi0, Options(chi=chi, cut=1e-14, power=2, seed=seed), truncate=truncate)
    return _dense(sites) * np.exp(ln), net.phys_dims(r)[0], sites


def _tail_errors(E, dims, chi):
    eps = []
    for k in range(1, len(dims)):
        s = np.linalg.svd(E.reshape(int(np.prod(dims[:k])), -1), compute_uv=False)
        eps.append(np.sqrt(np.sum(s[chi:] ** 2)))
    return np.array(eps)


# (kind, lattice, chi) where the rank-2chi stage is exact but chi truncates
EXACT_STAGE = [("king", dict(R=2, C=3, a=2), 2), ("king", dict(R=2, C=3, a=2), 3),
               ("king", dict(R=3, C=3, a=2), 2), ("king", dict(R=2, C=4, a=2), 2),
               ("king", dict(R=2, C=4, a=2), 3), ("zephyr", dict(m=1, t=2), 8)]


@pytest.mark.parametrize("kind,kw,chi", EXACT_STAGE)
def test_truncation_within_tt_svd_bounds(kind, kw, chi):
    E, dims, _ = _bottom_row(kind, kw, 256, truncate=False)
    Z, _, _ = _bottom_row(kind, kw, chi, truncate=False)
    scale = np.linalg.norm(E)
    assert np.linalg.norm(Z - E) <= 1e-12 * scale  # the 2 chi stage is exact here
    T, _, sites = _bottom_row(kind, kw, chi, truncate=True)
    assert max(s.shape[2] for s in sites[:-1]) <= chi
    eps = _tail_errors(E, dims, chi)
    err = np.linalg.norm(T - E)
    assert eps.max() > 1e-6 * scale  # a real truncation
    assert err <= np.sqrt(np.sum(eps ** 2)) * (1 + 1e-9) + 1e-12 * scale
    assert err >= eps.max() * (1 - 1e-9) - 1e-12 * scale


@pytest.mark.parametrize("chi", [2, 3, 4, 6])
def test_truncation_never_beats_eckart_young(chi):
    # Zephyr t=2 cells: at these chi the randomized stage truncates as well
    E, dims, _ = _bottom_row("zephyr", dict(m=1, t=2), 256, truncate=False)
    T, _, _ = _bottom_row("zephyr", dict(m=1, t=2), chi, truncate=True)
    eps = _tail_errors(E, dims, chi)
    assert eps.max() > 0
    assert np.linalg.norm(T - E) >= eps.max() * (1 - 1e-9)


def test_planted_mistake_in_sweep_breaks_the_upper_bound(monkeypatch):
    # a truncation that keeps the wrong singular triplets (the smallest chi
    # instead of the largest) must fail the upper bound: the pin can fail
    import oracle.bmps as bm
    real_svd = np.linalg.svd

    def reversed_svd(a, full_matrices=True, compute_uv=True):
        if not compute_uv:
            return real_svd(a, full_matrices=full_matrices, compute_uv=False)
        U, S, Vt = real_svd(a, full_matrices=full_matrices)
        n = len(S)
        if n < 2:
            return U, S, Vt
        return U[:, :n][:, ::-1], S[::-1].copy(), Vt[:n][::-1]

    E, dims, _ = _bottom_row("king", dict(R=2, C=3, a=2), 256, truncate=False)
    monkeypatch.setattr(bm.np.linalg, "svd", reversed_svd)
    try:
        T, _, _ = _bottom_row("king", dict(R=2, C=3, a=2), 2, truncate=True)
    finally:
        monkeypatch.setattr(bm.np.linalg, "svd", real_svd)
    eps = _tail_errors(E, dims, 2)
    assert np.linalg.norm(T - E) > np.sqrt(np.sum(eps ** 2)) * 1.01
