"""The lattice symmetries on the GPU path (Sec. V.A) and the pooled
selection over several runs."""
import numpy as np
import pytest

from tnb_inputs import make_instance, transform, N_TRANSFORMS
from oracle import ising
from oracle.bmps import contract_env, Options

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_16431_amd as pk
    return pk, torch


def test_exact_contraction_is_invariant_and_pooled_search_exact():
    pk, torch = _gpu()
    inst = make_instance("king", 402, jdist="uniform", hdist="uniform0.1", R=2, C=3, a=2)
    bf = ising.brute_force(inst, 1.0)
    res = pk.solve_transformed(inst, 1.0, chi=64, M=4096, K=3, cut=1e-7)
    for t, z in res["logZ"].items():
        assert abs(z - bf["logZ"]) <= 1e-10 * abs(bf["logZ"]), (t, z)
    assert res["logZ_spread"] <= 1e-10 * abs(bf["logZ"])
    assert abs(res["energies"][0] - bf["E_min"]) < 1e-12
    assert np.array_equal(res["energies"], ising.energies(inst, res["states"]))


def test_truncated_logz_per_transform_matches_oracle():
    # each orientation is a different approximation; the GPU and the oracle
    # must agree on every one of them
    pk, torch = _gpu()
    inst = make_instance("zephyr", 403, jdist="uniform", hdist="uniform0.1", m=2, t=1)
    res = pk.solve_transformed(inst, 1.0, chi=4, M=16, K=4, power_iters=2, seed=9)
    for t in range(N_TRANSFORMS):
        ora = contract_env(transform(inst, t), 1.0, Options(chi=4, power=2, seed=9)).logZ
        assert abs(res["logZ"][t] - ora) <= 1e-5 * abs(ora), (t, res["logZ"][t], ora)
    assert res["energies"][0] <= min(res["best_energy"].values())
    print("log Z spread over the 8 orientations at chi=4: %.3e" % res["logZ_spread"])


def test_select_lowest_matches_host_order():
    pk, torch = _gpu()
    rng = np.random.default_rng(5)
    n, N = 200, 37
    S = np.where(rng.random((n, N)) < 0.5, -1, 1).astype(np.int8)
    S[50:60] = S[0:10]                          # duplicates
    E = np.round(rng.standard_normal(n) * 4) / 4
    E[50:60] = E[0:10]
    order = np.lexsort(tuple(S[:, ::-1].T) + (E,))
    seen, ref = set(), []
    for i in order:
        if S[i].tobytes() not in seen:
            seen.add(S[i].tobytes())
            ref.append(i)
    for K in (1, 7, len(ref), len(ref) + 3):
        st, en = pk.select_lowest(torch.from_numpy(S).cuda(), torch.from_numpy(E).cuda(), K)
        k = min(K, len(ref))
        assert np.array_equal(st.cpu().numpy(), S[ref[:k]]) and np.array_equal(en.cpu().numpy(), E[ref[:k]])
