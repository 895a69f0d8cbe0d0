#!/usr/bin/env python3
"""Benchmark of the boundary-MPS branch-and-bound hot path on one MI355X.

One step = the whole path on one synthetic instance: cluster tables and
Boltzmann weights, all boundary MPSs (zipper + randomized SVD), every beam
step (right environments, conditional marginals, merge and top-M), export of
the final states and their energies.  The metric counts spin marginals: for
every parent b at every beam step, the k marginals <s_i>_b of the cluster
being fixed, which its conditional distribution p_b(x) determines.

Prints one JSON line.  With --gpus N > 1 it exits: the implementation runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # plain method on Zephyr Z_2 (t=4, 160 spins), J ~ U[-1,1], h ~ U[-0.1,0.1],
    # beta = 1, chi = 16, beam M = 64, 8 states returned, FP64.
    "zephyr_z2_t4_plain": dict(kind="zephyr", kw=dict(m=2, t=4), seed=1000, jdist="uniform",
                               hdist="uniform0.1", beta=1.0, chi=16, M=64, K=8),
    # App. B workload: king's lattice 50 x 50 with one spin per site (d = 2),
    # tile-planted so that the exact ground energy E0 is known; beta = 4,
    # chi = 16, M = 256
    "king_50x50_planted": dict(kind="king_planted", kw=dict(R=50, C=50, a=1), seed=1000, jdist="planted",
                               hdist="zero", beta=4.0, chi=16, M=256, K=8),
    # small sibling used for quick checks (t = 2 cells of 8 spins)
    "zephyr_z2_t2_plain": dict(kind="zephyr", kw=dict(m=2, t=2), seed=1000, jdist="uniform",
                               hdist="uniform0.1", beta=1.0, chi=16, M=64, K=8),
}

# MI355X: FP64 vector and FP64 MFMA peaks are equal; FP32 MFMA (dense) and FP32 vector are 157.3
PEAK = {"alu_fp64_tflops": 78.6, "fp32_tflops": 157.3, "hbm_gbs": 8000.0}
MFMA_KERNELS = {"medf_Y2", "medf_W2", "medf_Y2g", "medf_W2g", "medf_G2", "medf_out", "medf_G2g", "medf_outg",
                "medf_lbin", "medf_lbing", "medf_lacc", "medf_laccg", "renv_V", "adj_v", "site_apply", "site_applyT", "site_left", "gemm"}


def peak_of(name):
    """Peak of a timed kernel: FP32 for the *_f32 diagram kernels, else FP64."""
    return PEAK["fp32_tflops"] if name.endswith("_f32") else PEAK["alu_fp64_tflops"]


def unit_class(name):
    return "mfma" if name.replace("_f32", "") in MFMA_KERNELS else "alu"
# library timer -> the kernel instance rocprofv3 reports for it
# (a prefix where the timer's launches use several tile variants of one kernel)
ROCPROF_NAME = {"medf_Y2": "medf_bin_pipe<0, 1, 0, double>", "medf_W2": "medf_bin_pipe<1, 1, 0, double>",
                "medf_lbin": "medf_bin_pipe<0, 1, 1, double>", "medf_G2g": "gemm_mfma_kernel<1,",
                "medf_outg": "gemm_mfma_kernel<2,", "medf_Y2g": "gemm_mfma_kernel<3,",
                "medf_W2g": "gemm_mfma_kernel<4,", "medf_lbing": "gemm_mfma_kernel<5,",
                "medf_Y2w": "medf_wsum_kernel<0,",
                "medf_W2w": "medf_wsum_kernel<1,"}

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by the same counters on a plain copy of known size.
# Valid only for the kernel source they were taken on: one hash over the file
# with the GEMM body and the file with its operand maps and launches.
KERNEL_SRC = [os.path.join(ROOT, "paper_2411_16431_amd", "csrc", f) for f in ("gemm_mfma.hip", "env.hip")]
TUNING_FILE = os.path.join(ROOT, "paper_2411_16431_amd", "tuning_mi355x.json")


def source_sha(hashlib):
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))) as fh:
            rec = json.load(fh)
        sha = source_sha(hashlib)
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("workload") != workload or rec.get("source_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def kernel_table(prof, steps):
    """Every timed kernel: time per step, launches, achieved rate and its
    fraction of the FP64 peak (matrix cores and vector units peak alike on
    MI355X) and of HBM bandwidth, from the algorithmic flop and byte counts."""
    out = {}
    for name, (ms, n, fl, by) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        if n == 0 or ms <= 0:
            continue
        sec = ms / 1000.0
        tf, gbs = fl / sec / 1e12, by / sec / 1e9
        out[name] = {"ms_per_step": ms / steps, "launches_per_step": n / steps, "avg_ms": ms / n,
                     "unit_class": unit_class(name), "tflops": tf, "peak_tflops": peak_of(name),
                     "frac_peak": tf / peak_of(name), "gbs": gbs, "frac_hbm": gbs / PEAK["hbm_gbs"]}
    return out


def write_traffic(fetch_csv, write_csv, timer, workload, copy_bytes=8 << 27):
    """HBM bytes per launch of one kernel from two rocprofv3 --pmc passes
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by the same
    counter's reading for the plain 1 GiB device copy that ends the run
    (--copy-calibration); the record goes to profiles/ with the hash of the
    kernel source it was taken on."""
    import csv
    import hashlib

    def read(path, counter):
        per = {}
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                d = int(row["Dispatch_Id"])
                name, v = row["Kernel_Name"], float(row["Counter_Value"])
                per.setdefault(d, [name, 0.0])[1] += v
        return per

    kname = ROCPROF_NAME[timer]
    out = {"kernel": timer, "rocprof_kernel": kname, "workload": workload}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = read(path, counter)
        copies = [v for d, (n, v) in sorted(per.items()) if "copy" in n.lower()]
        mine = [v for n, v in per.values() if kname in n]
        if not copies or not mine:
            raise SystemExit("no %s dispatches of %s or of the copy in %s" % (counter, kname, path))
        factor = copies[-1] * 1024.0 / copy_bytes
        key = "fetch" if counter == "FETCH_SIZE" else "write"
        out[key + "_bytes_per_launch"] = sum(mine) / len(mine) * 1024.0 / factor
        out[key + "_factor"] = factor
        out["launches"] = len(mine)
    out["hbm_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    out["source_sha256"] = source_sha(hashlib)
    out["commands"] = [
        "rocprofv3 --pmc %s --output-format csv -d gpurun_out/pmc_%s -o %s -- python3 bench.py --steps 1 "
        "--warmup 0 --no-cpu-baseline --no-planted --no-f32 --copy-calibration" % (c, c.split("_")[0].lower(),
                                                                          c.split("_")[0].lower())
        for c in ("FETCH_SIZE", "WRITE_SIZE")]
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (timer, workload))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zephyr_z2_t4_plain", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32-contraction comparison")
    ap.add_argument("--power-iters", type=int, default=2)
    ap.add_argument("--no-planted", action="store_true",
                    help="skip the planted-instance energy gap (profiling runs: keeps rocprof's kernel averages to the timed workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a plain 1 GiB device copy, the reference dispatch for HBM byte counters")
    ap.add_argument("--autotune", metavar="JSON",
                    help="measure the launch variants of every new shape during warm-up and write the table here")
    ap.add_argument("--tuning", default=TUNING_FILE,
                    help="launch-variant table used when not measuring (default: the committed MI355X table)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no run: turn two rocprofv3 counter files of the dominant kernel into profiles/*_traffic.json")
    ap.add_argument("--traffic-kernel", default="medf_G2g")
    ap.add_argument("--batch", type=int, default=0,
                    help="also solve this many instances of the workload (seeds seed..seed+n-1) at once with "
                         "solve_batch, after the timed region, and report their aggregate rate")
    return ap.parse_args()


def make(wl, seed=None):
    """The workload's instance, and its exact ground energy when planted (else None)."""
    from tnb_inputs import make_instance, planted_king
    seed = wl["seed"] if seed is None else seed
    if wl["kind"] == "king_planted":
        inst, _, E0 = planted_king(wl["kw"]["R"], wl["kw"]["C"], wl["kw"]["a"], seed, loops_per_cell=1)
        return inst, E0
    return make_instance(wl["kind"], seed, jdist=wl["jdist"], hdist=wl["hdist"], **wl["kw"]), None


def batch_rate(pk, torch, wl, env_kw, n):
    """n instances of the workload solved one by one and then at once
    (solve_batch, one stream per instance): aggregate spin marginals/s."""
    insts = [make(wl, wl["seed"] + i)[0] for i in range(n)]
    kw = dict(chi=wl["chi"], M=wl["M"], K=wl["K"], **env_kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [pk.solve(i, wl["beta"], **kw) for i in insts]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    par = pk.solve_batch(insts, wl["beta"], workers=n, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    marg = sum(r["spin_marginals"] for r in seq)
    same = all(a["logZ"] == b["logZ"] and (a["energies"] == b["energies"]).all() for a, b in zip(seq, par))
    return {"instances": n, "one_by_one_s": t1 - t0, "batch_s": t2 - t1,
            "one_by_one_spin_marginals_per_s": marg / (t1 - t0), "batch_spin_marginals_per_s": marg / (t2 - t1),
            "speedup": (t1 - t0) / (t2 - t1), "results_identical": bool(same)}


def cpu_baseline(inst, wl, counts, marg_per_step, power):
    """Oracle (plain numpy FP64) timed on slices of the same workload and
    extrapolated to one step: one site diagram application, a slice of the
    rho loop of one mediating application (scaled to the full loop), and the
    marginals of one parent; multiplied by the counts of one GPU step."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle.bmps import Network, RowOps
    rng = np.random.default_rng(0)
    net = Network(inst, wl["beta"])
    r = 1
    ops = RowOps(net, r)
    chi = wl["chi"]
    s = 2 * chi + 8
    # largest site and mediating diagram of row 1
    c_site = max(range(net.C), key=lambda c: len(ops.site[c]["x"]))
    S = ops.site[c_site]
    dvd = int(S["vd"].max()) + 1
    A = rng.standard_normal((chi, dvd, chi))
    K = rng.standard_normal((chi, S["dR"], 2 * chi))
    X = rng.standard_normal((S["Wv"].shape[0], 2 * chi, s))
    t0 = time.perf_counter()
    ops.site_apply(c_site, A, K, X)
    t_site = time.perf_counter() - t0
    c_med = max(range(net.C - 1), key=lambda c: ops.med[c]["dR"] * ops.med[c]["dL"])
    Md = ops.med[c_med]
    n_sl = 4
    full_dR = Md["dR"]
    Md_slice = dict(Md)
    Md_slice["dR"] = n_sl
    ops.med[c_med] = Md_slice
    A2 = rng.standard_normal((chi, Md["da2"] * (int(Md["b2"].max()) + 1), chi))
    K2 = rng.standard_normal((chi, Md["dL"], 2 * chi))
    X2 = rng.standard_normal((Md["Wdr"].shape[0], Md["Wdl"].shape[0], 2 * chi, s))
    t0 = time.perf_counter()
    ops.med_apply(c_med, A2, K2, X2)
    t_med = (time.perf_counter() - t0) * full_dR / n_sl
    ops.med[c_med] = Md
    site_calls = counts.get("site", 0)
    med_calls = counts.get("med", 0)
    t_step = site_calls * t_site + med_calls * t_med
    threads = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas") or 1
    sample = ("oracle RowOps.site_apply on the largest cell of row 1 (%.2f s) and %d of %d rho "
              "iterations of the largest mediating diagram of row 1 (%.2f s extrapolated to the full "
              "loop), times the %d site and %d mediating diagram applications of one step; beam "
              "steps not included (extrapolated lower bound on the oracle's time)" %
              (t_site, n_sl, full_dR, t_med, site_calls, med_calls))
    return dict(value=marg_per_step / t_step, unit="spin marginals/s", cores=int(threads),
                kind="oracle", sample=sample, seconds_per_step_extrapolated=t_step)


def cpu_baseline_full(inst, wl, marg_per_step):
    """Oracle end to end on the same instance (feasible for d = 2 clusters):
    all boundary MPSs and the whole beam search, timed on the host cores."""
    from threadpoolctl import threadpool_info
    from oracle.bmps import contract_env, Options
    from oracle.search import solve
    t0 = time.perf_counter()
    env = contract_env(inst, wl["beta"], Options(chi=wl["chi"], power=2, seed=4242))
    ref = solve(inst, wl["beta"], env, M=wl["M"], K=wl["K"])
    dt = time.perf_counter() - t0
    threads = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas") or 1
    return dict(value=marg_per_step / dt, unit="spin marginals/s", cores=int(threads), kind="oracle",
                sample="oracle contract_env and solve end to end on the benchmark instance (%.1f s)" % dt,
                seconds_per_step=dt), float(ref["energies"][0]), env.logZ


def adjoint_compare(pk, torch, env, wl, inst):
    """All row moments of one beam state (the start of row 1, where the beam is
    full) by the adjoint sweep and by one clamped contraction per branch; both
    include the forward right environments of the row."""
    import numpy as np
    beam = pk.Beam(env, wl["M"])
    for _ in range(inst.C):
        beam.step()
    _, npar, _ = beam.info()
    sp, ed = beam.row_layout()
    beam.row_moments()  # layout upload and buffers
    torch.cuda.synchronize()
    t_adj = []
    for _ in range(3):
        t0 = time.perf_counter()
        m1, m2 = beam.row_moments()
        torch.cuda.synchronize()
        t_adj.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    pb = beam.row_moments_per_branch()
    torch.cuda.synchronize()
    t_pb = time.perf_counter() - t0
    n = npar * len(sp)
    ta = float(np.median(t_adj))
    return {"state": "start of row 1 (beam full)", "parents": int(npar), "row_spins": int(len(sp)),
            "row_couplings": int(len(ed)), "adjoint_ms": ta * 1e3, "per_branch_ms": t_pb * 1e3,
            "adjoint_spin_marginals_per_s": n / ta, "per_branch_spin_marginals_per_s": n / t_pb,
            "speedup": t_pb / ta, "pair_moments_per_s_adjoint": npar * len(ed) / ta,
            "max_abs_diff_adjoint_vs_per_branch": float((m1 - pb).abs().max().item())}


def fp32_compare(pk, torch, inst, wl, env_kw, res64, steps):
    """The same solve with FP32 diagram contractions: time per step and the
    error of each result against the FP64 path (log Z, returned energies and
    states)."""
    kw = dict(env_kw, prec="f32")
    pk.solve(inst, wl["beta"], chi=wl["chi"], M=wl["M"], K=wl["K"], **kw)  # warm-up
    torch.cuda.synchronize()
    pk.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = pk.solve(inst, wl["beta"], chi=wl["chi"], M=wl["M"], K=wl["K"], **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    pk.profile_enable(False)
    prof = {name: pk.profile_query(name) for name in pk.profile_names()}
    import numpy as np
    same = (res["states"].shape == res64["states"].shape and np.array_equal(res["states"], res64["states"]))
    return {"ms_per_step": dt * 1e3, "value": res["spin_marginals"] / dt, "logZ": res["logZ"],
            "logZ_rel_err_vs_f64": abs(res["logZ"] - res64["logZ"]) / abs(res64["logZ"]),
            "best_energy": float(res["energies"][0]), "best_energy_f64": float(res64["energies"][0]),
            "returned_states_equal_f64": bool(same), "kernels": kernel_table(prof, steps)}


def planted_gap(pk, wl, env_kw):
    """Energy gap d_E = (E - E0) / (2 |E0|) (Eq. 14) on a planted instance of
    the same lattice, chi and beam, whose exact ground energy E0 is the sum of
    its loop minima: the oracle cannot solve the random workload at t = 4, so
    this is the stand-in for the gap against an exact reference."""
    if wl["kind"] != "zephyr":
        return None
    from tnb_inputs import planted_loops
    m, t = wl["kw"]["m"], wl["kw"]["t"]
    inst, _, E0 = planted_loops(m, t, 91, loops_per_cell=2)
    res = pk.solve(inst, wl["beta"], chi=wl["chi"], M=wl["M"], K=1, **env_kw)
    E = float(res["energies"][0])
    return {"instance": "planted loops, Zephyr Z_%d t=%d, seed 91, 2 loops per cell" % (m, t),
            "E0_exact": float(E0), "best_energy": E, "d_E": (E - E0) / (2 * abs(E0))}


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.traffic_kernel, args.workload)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); got --gpus %d"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    import paper_2411_16431_amd as pk
    wl = WORKLOADS[args.workload]
    inst, E0 = make(wl)
    env_kw = dict(power_iters=args.power_iters, seed=4242)
    if args.autotune:
        pk.autotune(True, args.autotune)
    elif args.tuning and os.path.exists(args.tuning):
        pk.autotune(False, args.tuning)

    def one():
        return pk.solve(inst, wl["beta"], chi=wl["chi"], M=wl["M"], K=wl["K"], **env_kw)

    for i in range(args.warmup):
        one()
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if args.autotune:
        pk.autotune(False, args.autotune)  # timed steps use the measured table
    pk.profile_enable(True)
    t0 = time.perf_counter()
    res = None
    for i in range(args.steps):
        res = one()
        print("step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pk.profile_enable(False)
    ms_step = (t1 - t0) * 1000.0 / args.steps
    marg = res["spin_marginals"]
    value = marg * args.steps / (t1 - t0)
    # dominant kernel over the timed region
    prof = {}
    for name in pk.profile_names():
        prof[name] = pk.profile_query(name)
    dom = max(prof, key=lambda n: prof[n][0]) if prof else None
    roof = None
    if dom:
        ms, n, fl, by = prof[dom]
        avg_s = ms / 1000.0 / n
        roof = {"bound": unit_class(dom), "kernel": dom, "achieved": fl / n / avg_s / 1e12,
                "peak": peak_of(dom), "unit": "TFLOP/s",
                "frac": fl / n / avg_s / 1e12 / peak_of(dom),
                "traffic": measured_traffic(dom, args.workload), "traffic_unit": "bytes per launch",
                "algorithmic_bytes_per_launch": by / n,
                "avg_ms": ms / n, "launches_per_step": n / args.steps,
                "share_of_step": ms / args.steps / ms_step}
    counts = {"site": (prof.get("site_apply", (0, 0))[1] + prof.get("site_applyT", (0, 0))[1]) / args.steps,
              "med": sum(prof.get(nm, (0, 0))[1] for nm in ("med_apply", "med_applyT", "medf_Y2", "medf_W2",
                                                                "medf_Y2g", "medf_W2g")) / args.steps}
    adj = adjoint_compare(pk, torch, res["env"], wl, inst)
    batch = batch_rate(pk, torch, wl, env_kw, args.batch) if args.batch > 1 else None
    f32 = None if args.no_f32 else fp32_compare(pk, torch, inst, wl, env_kw, res, args.steps)
    print("fp32 comparison done", file=sys.stderr, flush=True)
    planted = None if (args.no_planted or E0 is not None) else planted_gap(pk, wl, env_kw)
    print("adjoint comparison done", file=sys.stderr, flush=True)
    cpu, gap_oracle, exact = None, None, None
    best = float(res["energies"][0])
    if E0 is not None:
        exact = {"E0": float(E0), "best_energy": best, "d_E": (best - E0) / (2 * abs(E0))}
    if not args.no_cpu_baseline:
        if wl["kind"] == "king_planted":
            cpu, e_ora, z_ora = cpu_baseline_full(inst, wl, marg)
            gap_oracle = {"oracle_best_energy": e_ora, "d_E": (best - e_ora) / (2 * abs(e_ora)),
                          "oracle_logZ": z_ora, "logZ_rel_diff": abs(res["logZ"] - z_ora) / abs(z_ora)}
        else:
            cpu = cpu_baseline(inst, wl, counts, marg, args.power_iters)
    out = {
        "metric": "beam marginals/sec and best energy gap vs oracle, adjoint+batched vs plain",
        "value": value, "unit": "spin marginals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "spins": int(inst.n_spins),
                   "lattice": [int(inst.R), int(inst.C)], "beta": wl["beta"], "chi": wl["chi"],
                   "beam_M": wl["M"], "returned_K": wl["K"], "mode": "plain (per-step marginals, no adjoint)",
                   "power_iters": args.power_iters},
        "best_energy": best, "energy_gap_vs_oracle": gap_oracle, "energy_gap_exact": exact,
        "energy_gap_planted": planted,
        "logZ": res["logZ"], "logZ_sign": res["env"].sign, "spin_marginals_per_step": marg,
        "roofline": roof, "cpu_baseline": cpu, "adjoint": adj, "fp32": f32, "batch": batch,
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])},
        "kernels": kernel_table(prof, args.steps),
        "tuning": args.autotune or (args.tuning if args.tuning and os.path.exists(args.tuning) else None),
    }
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        n = 1 << 27  # 1 GiB of FP64
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("copy calibration: %d bytes read, %d bytes written" % (8 * n, 8 * n), file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
