"""Benchmark of the Gini MDS hot path on one MI355X.

A step is one descent iteration of the image workload (n = 10000 points,
m = 784 coordinates, nu = 2, latent p = 2 with the Gini latent distance):
the fused stress forward + backward over the upper triangle of Delta with the
latent re-ranking, the deterministic reduction and the update of Z.  Delta is
built once before timing (its build time is reported separately), inputs are
resident in HBM when the timed region starts.

Printed as ONE JSON line:
  value            pair-evals/s = n(n-1)/2 / seconds per step
  roofline         the stress-tile kernel: algorithmic bytes per launch
                   (4 B per pair of the triangle + Z read + G written) over
                   its average launch time (HIP events on its stream)
  sweep            the nu-sweep workload (16 problems x 8 nu = 128 instances):
                   instance-iterations/s of the batched solve vs the plain
                   one-instance-per-launch path
  select           Algorithm 1's nu selection (gini_select_nu) on the
                   Gaussian-mixture workload, end to end
  extras           the Sammon-loss descent step and classical MDS on the same
                   Delta
  cpu_baseline     the FP64 oracle's stress + gradient on a bounded sample

--workload heavy measures the heavy-tailed set instead (n = 50000 Student-t
rows, m = 64, p = 3; Delta is 10 GB) and reports that workload only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "stress fwd+bwd pair-evals/s and HBM GB/s at n=10k; batched vs plain iters/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--sweep-iters", type=int, default=200)
    ap.add_argument("--plain-iters", type=int, default=40)
    ap.add_argument("--persistent-iters", type=int, default=10)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-select", action="store_true")
    ap.add_argument("--workload", choices=["images", "heavy"], default="images",
                    help="images: n = 10^4 image rows, p = 2 (the default); heavy: n = 5*10^4 Student-t rows, "
                         "m = 64, p = 3 (one line for this workload only)")
    ap.add_argument("--p", type=int, default=0,
                    help="latent dimensions of the heavy workload (default 3; 2 measures the pure-HBM p = 2 case)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the Sammon-loss and classical-MDS measurements on the image workload")
    ap.add_argument("--cpu-seconds", type=float, default=5.0)
    ap.add_argument("--mode", choices=["auto", "persistent", "batched"], default="auto")
    ap.add_argument("--tile", type=int, default=256)
    ap.add_argument("--sweep-mode", choices=["auto", "persistent", "batched", "split"], default="auto")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain device copy of 256 MiB (calibration of memory counters)")
    ap.add_argument("--sweep-tile", type=int, default=0)
    return ap.parse_args()


PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2605_25124_amd", "csrc", f)
                  for f in ("k_stress.hip", "stress_impl.hpp", "common.hpp", "kernels.hpp")]


def measured_traffic(kernel, n, p, tile):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary under profiles/ taken at this n, p and tile on the current kernel
    sources, or None when there is none."""
    digest = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()
    try:
        names = sorted(os.listdir(PROFILES))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            fields = dict(re.findall(r"^(\w+): (\S+)$", f.read(), re.M))
        if (fields.get("kernel") == kernel and fields.get("source_sha256") == digest
                and fields.get("n") == str(n) and fields.get("p") == str(p) and fields.get("tile") == str(tile)
                and "traffic_bytes_per_launch" in fields):
            return float(fields["traffic_bytes_per_launch"])
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """nproc and the CPU model name of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_leg(args, w, D, Z0, nu, p, gm, dev, mixture=False):
    """The oracle timed on a bounded sample of the workload, one thread pinned
    to one core: its dissimilarity build on the first `ns` rows (the real Gini
    Delta of the sample), then descent steps on that Delta for about
    --cpu-seconds; both extrapolated to the full n by n^2 (labelled as such).
    Then the GPU's results against the oracle on the same inputs: ranks
    (count of mismatches), Delta (error over the condition scale on sampled
    pairs, and the plain relative error), the stress and the gradient (per
    entry over the term-magnitude sums) on a subsample of points."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_2605_25124_amd import synth

    n, m = w.X.shape
    ns = 700
    old_aff = os.sched_getaffinity(0)
    core = min(old_aff)
    os.sched_setaffinity(0, {core})
    try:
        Xs = w.X[:ns]
        t0 = time.perf_counter()
        Dso = O.dissim(Xs, [nu], O.MATCH32)[0]
        t_delta = time.perf_counter() - t0
        Zs = w.Z0[0][:ns, :p].astype(np.float64)
        reps, t0 = 0, time.perf_counter()
        while True:
            Zs, _ = O.solve(Dso, Zs, nu, 1, O.LATENT_GINI, O.MATCH32)   # stress + gradient + step
            reps += 1
            if reps >= 10 and time.perf_counter() - t0 >= args.cpu_seconds:
                break
        t_steps = time.perf_counter() - t0
        # the small workload in full: Delta of 200 x 10 rows and 100 descent steps
        ws = synth.workload_small()
        t0 = time.perf_counter()
        Dsm = O.dissim(ws.X, [2.0], O.MATCH32)[0]
        O.solve(Dsm, ws.Z0[0].astype(np.float64), 2.0, ws.iters, O.LATENT_GINI, O.MATCH32)
        t_small = time.perf_counter() - t0
        # the Gaussian-mixture workload: its Delta (3 nu) in full, then 20
        # descent steps at each nu (of the 500 the workload runs)
        mix = None
        if mixture:
            wg = synth.workload_gmm()
            t0 = time.perf_counter()
            Dg = O.dissim(wg.X, wg.nus, O.MATCH32)
            t_gd = time.perf_counter() - t0
            ks = 20
            t0 = time.perf_counter()
            for q, nug in enumerate(wg.nus):
                O.solve(Dg[q], wg.Z0[q].astype(np.float64), nug, ks, O.LATENT_GINI, O.MATCH32)
            t_gs = time.perf_counter() - t0
            mix = {"workload": f"Gaussian mixture n={wg.X.shape[0]} m={wg.X.shape[1]}, nu in {wg.nus}",
                   "delta_s": round(t_gd, 2), "steps_per_nu": ks, "steps_s": round(t_gs, 2),
                   "extrapolated_full_s": {"note": f"Delta measured; descent scaled from {ks} to {wg.iters} "
                                                   f"steps per nu, not measured",
                                           "value": round(t_gd + t_gs * wg.iters / ks, 1)}}
    finally:
        os.sched_setaffinity(0, old_aff)
    sp = ns * (ns - 1) // 2
    full = n * (n - 1) // 2
    step_rate = reps * sp / t_steps
    cpu = {"value": round(step_rate, 1), "unit": "pair-evals/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 oracle, one thread pinned to one core: Gini Delta of the first {ns} rows of the "
                     f"workload ({sp} pairs, m={m}) in {t_delta:.2f} s, then {reps} descent steps on it (stress + "
                     f"gradient + update, p={p} Gini latent) in {t_steps:.1f} s; small_workload_full_s: Delta of "
                     f"the 200 x 10 workload and its 100 descent steps",
           "dissim_pairs_per_s": round(sp / t_delta, 1),
           "small_workload_full_s": round(t_small, 3),
           "mixture_workload": mix,
           "extrapolated_n2": {"note": f"n^2 extrapolation from the {ns}-row sample to n={n}, not measured",
                               "dissim_build_s": round(t_delta * full / sp, 1),
                               "descent_step_s": round(full / step_rate, 3)},
           "host": host_cpu()}

    # ---- errors of the GPU results against the oracle, on the same inputs
    g = np.random.Generator(np.random.PCG64(4242))
    err = {}
    # ranks: rows of pair differences fl32(x_i - x_j), the vectors ranked inside Delta
    pi, pj = g.integers(0, n, 256), g.integers(0, n, 256)
    V = (w.X[pi] - w.X[pj]).astype(np.float32)
    tr = gm.gini_rank(torch.from_numpy(V).to(dev)).cpu().numpy()
    err["ranks"] = {"rows": int(V.shape[0]), "d": int(m), "mismatches": int((tr != O.rank2_rows(V)).sum())}
    # Delta on sampled pairs of the full matrix
    pi, pj = g.integers(0, n, 2000), g.integers(0, n, 2000)
    keep = pi != pj
    pi, pj = pi[keep], pj[keep]
    got = D[torch.from_numpy(pi).to(dev), torch.from_numpy(pj).to(dev)].cpu().numpy().astype(np.float64)
    ref = O.dissim_pairs(w.X, pi, pj, [nu], O.MATCH32)[:, 0]
    S = np.empty(len(pi))
    for q in range(len(pi)):
        z = (w.X[pi[q]].astype(np.float32) - w.X[pj[q]].astype(np.float32)).astype(np.float64)
        _, a = O.gini_dist_grad(z, nu)
        S[q] = float(np.sum(np.abs(z * a)))
    big = np.abs(ref) >= 1e-3 * np.abs(ref).max()
    err["delta"] = {"pairs": int(len(pi)), "max_err_over_scale": float(np.max(np.abs(got - ref) / S)),
                    "max_rel_err": float(np.max(np.abs(got - ref)[big] / np.abs(ref)[big])), "tolerance": 1e-5}
    # stress and gradient on a 2000-point subsample (the GPU's Delta entries as the input of both)
    k = min(n, 2000)
    idx = np.sort(g.choice(n, k, replace=False))
    ti = torch.from_numpy(idx).to(dev)
    Dk = D.index_select(0, ti).index_select(1, ti).contiguous()
    Zk = Z0.index_select(0, ti).contiguous()
    G, sig = gm.gini_stress_bwd(Dk, Zk, nu, gm.LATENT_GINI)
    Dh, Zh = Dk.cpu().numpy().astype(np.float64), Zk.cpu().numpy()
    s_ref, G_ref = O.stress(Dh, Zh, nu, O.LATENT_GINI, O.MATCH32)
    B = O.grad_scale(Dh, Zh, nu, O.LATENT_GINI, O.MATCH32)
    Gn = G.cpu().numpy().astype(np.float64)
    s_gpu = float(sig[0].double() + sig[1].double())
    err["sigma"] = {"points": k, "rel_err": abs(s_gpu - s_ref) / abs(s_ref), "tolerance": 1e-4}
    err["grad"] = {"points": k, "max_err_over_scale": float(np.max(np.abs(Gn - G_ref) / (B + 1e-300))),
                   "rel_2norm": float(np.linalg.norm(Gn - G_ref) / np.linalg.norm(G_ref)), "tolerance": 1e-4}
    return cpu, err


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported (the method's "
              f"multi-GPU split is described in the design notes, not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_ref:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_read": a.numel() * 4, "copy_ref_bytes_written": b.numel() * 4,
                          "copies": 5}), flush=True)
        return

    from paper_2605_25124_amd import ginimds as gm
    from paper_2605_25124_amd import synth

    dev = torch.device("cuda:0")
    heavy = args.workload == "heavy"
    if heavy:                                            # its own workload only
        args.no_sweep = args.no_select = args.no_extras = True
    w = synth.workload_heavy() if heavy else synth.workload_images(args.n)
    n = w.X.shape[0]
    m = w.X.shape[1]
    pairs = n * (n - 1) // 2
    X = torch.from_numpy(w.X).to(dev)
    Z0 = torch.from_numpy(w.Z0[0]).to(dev)
    if heavy and args.p:
        if not 2 <= args.p <= w.Z0[0].shape[1]:
            raise SystemExit(f"--p must be 2..{w.Z0[0].shape[1]} for the heavy workload")
        Z0 = Z0[:, :args.p].contiguous()
    p = Z0.shape[1]
    nu = 2.0
    torch.cuda.synchronize()
    log(f"workload {w.name}: {pairs} pairs")

    # ---- Delta, built once (one-off; reported, not part of a step)
    gm.gini_dissim(X[:256], [nu])                       # warm the library / tables
    torch.cuda.synchronize()
    gm.gini_profile_enable(0, True)
    t0 = time.perf_counter()
    D = gm.gini_dissim(X, [nu])[0]
    torch.cuda.synchronize()
    dissim_s = time.perf_counter() - t0
    prof = gm.gini_profile_read(0)
    gm.gini_profile_enable(0, False)
    log(f"dissim build {dissim_s * 1e3:.1f} ms (kernels {prof['dissim_ms']:.1f} ms)")

    # ---- launch mode for the single large instance
    def inst(Z, hist=None):
        return gm.Instance(D, Z, nu, gm.LATENT_GINI, 0.0, hist)

    if args.mode == "auto":
        best = gm.gini_autotune([inst(Z0.clone())], 30)
    else:
        best = {"flags": gm.SOLVE_PERSISTENT if args.mode == "persistent" else gm.SOLVE_BATCHED,
                "tile": args.tile, "grid": 0}
    mode_name = "persistent" if best["flags"] == gm.SOLVE_PERSISTENT else "batched"
    log(f"mode {mode_name} tile {best['tile']} grid {best['grid']}")

    Zw = Z0.clone()
    gm.gini_mds_solve([inst(Zw)], args.warmup, best["flags"], best["tile"], best["grid"])
    torch.cuda.synchronize()

    # ---- timed region: K descent steps (no instrumentation inside)
    Z = Z0.clone()
    hist = torch.zeros(args.steps, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gm.gini_mds_solve([inst(Z, hist)], args.steps, best["flags"], best["tile"], best["grid"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el * 1e3 / args.steps
    value = pairs / (el / args.steps)
    h = hist.cpu().numpy()
    log(f"{args.steps} steps: {ms_step * 1e3:.1f} us/step, sigma {h[0]:.6e} -> {h[-1]:.6e}")
    # ---- the same K steps again with HIP events around every launch (per-kernel times)
    Z = Z0.clone()
    gm.gini_profile_enable(0, True)
    gm.gini_mds_solve([inst(Z)], args.steps, best["flags"], best["tile"], best["grid"])
    torch.cuda.synchronize()
    prof = gm.gini_profile_read(0)
    gm.gini_profile_enable(0, False)

    # dominant kernel and its algorithmic traffic per launch
    alg_bytes = 4.0 * pairs + 4.0 * n * p + 4.0 * n * p
    if prof["tile_launches"] > 0:
        kname = "k_stress_units"
        launches = prof["tile_launches"]
        avg_ms = prof["tile_ms"] / launches
    else:
        kname = "k_solve_persistent"
        launches = args.steps                      # one launch covers every step
        avg_ms = prof["persistent_ms"] / max(args.steps, 1)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, n, p, best["tile"]) if mode_name == "batched" else None,
            "kernel": kname,
            "avg_launch_us": round(avg_ms * 1e3, 2), "alg_bytes_per_launch": alg_bytes,
            "reduce_avg_us": round(prof["reduce_ms"] * 1e3 / max(prof["reduce_launches"], 1), 2)}
    if kname == "k_stress_units":
        # the step without the per-call fixed cost and launch gaps: its two kernels
        roof["step_kernels_us"] = round(roof["avg_launch_us"] + roof["reduce_avg_us"], 2)
    log(f"roofline {kname}: {avg_ms * 1e3:.1f} us/launch -> {achieved:.0f} GB/s")

    # ---- the Sammon loss and classical MDS on the same Delta (n = 10^4)
    extras = None
    if not args.no_extras:
        ds = gm.gini_sum(D)
        eta = gm.gini_sammon_step(D, p, nu)
        def sammon_inst(Zs):
            return gm.Instance(D, Zs, nu, gm.LATENT_GINI, eta, None, None, None, gm.LOSS_SAMMON, ds)
        ks = 100
        gm.gini_mds_solve([sammon_inst(Z0.clone())], 5, gm.SOLVE_BATCHED, best["tile"])
        torch.cuda.synchronize()
        Zs = Z0.clone()
        t0 = time.perf_counter()
        gm.gini_mds_solve([sammon_inst(Zs)], ks, gm.SOLVE_BATCHED, best["tile"])
        torch.cuda.synchronize()
        t_sam = (time.perf_counter() - t0) / ks
        gm.gini_profile_enable(0, True)
        gm.gini_mds_solve([sammon_inst(Z0.clone())], ks, gm.SOLVE_BATCHED, best["tile"])
        torch.cuda.synchronize()
        prof_s = gm.gini_profile_read(0)
        gm.gini_profile_enable(0, False)
        sam_us = prof_s["tile_ms"] / max(1, prof_s["tile_launches"]) * 1e3
        gm.gini_classical_mds(D[:512, :512].contiguous(), p)            # warm the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ev, cm_iters = gm.gini_classical_mds(D, p)
        torch.cuda.synchronize()
        t_cm = time.perf_counter() - t0
        extras = {
            "sammon": {"workload": f"images n={n}, nu=2, p=2 Gini latent, Sammon stress, {ks} descent steps",
                       "ms_per_step": round(t_sam * 1e3, 5), "pair_evals_per_s": round(pairs / t_sam, 1),
                       "units_avg_us": round(sam_us, 2),
                       "units_gbs_algorithmic": round(alg_bytes / (sam_us * 1e-6) / 1e9, 1)},
            "classical_mds": {"workload": f"images n={n}, nu=2 Delta, p=2, subspace iteration",
                              "seconds": round(t_cm, 4), "iterations": cm_iters,
                              "delta_pass_gbs": round(cm_iters * 4.0 * n * n / t_cm / 1e9, 1),
                              "eigenvalues": [round(float(v), 3) for v in ev]}}
        log(f"sammon {t_sam * 1e6:.1f} us/step (units {sam_us:.1f} us); classical MDS {t_cm * 1e3:.1f} ms, "
            f"{cm_iters} iterations")

    # ---- CPU baseline and errors against the oracle (needs D; run before the
    # sweep frees it)
    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        cpu, errors = cpu_leg(args, w, D, Z0, nu, p, gm, dev, mixture=not heavy)
        log(f"cpu oracle {cpu['value']:.3e} pair-evals/s; errors {json.dumps(errors)}")

    # ---- nu-sweep: batched persistent vs plain
    sweep = None
    if not args.no_sweep:
        del D
        torch.cuda.empty_cache()
        probs = synth.workload_sweep()
        Ds, Z0s, nus = [], [], []
        t0 = time.perf_counter()
        for pr in probs:
            Dk = gm.gini_dissim(torch.from_numpy(pr.X).to(dev), pr.nus)
            for k, nuk in enumerate(pr.nus):
                Ds.append(Dk[k])
                Z0s.append(torch.from_numpy(pr.Z0[k]).to(dev))
                nus.append(nuk)
        torch.cuda.synchronize()
        sweep_build = time.perf_counter() - t0
        n_inst = len(Ds)

        def insts():
            return [gm.Instance(Ds[k], Z0s[k].clone(), nus[k]) for k in range(n_inst)]

        if args.sweep_mode == "auto":
            tuned = gm.gini_autotune(insts(), 20)
        else:
            tuned = {"flags": {"persistent": gm.SOLVE_PERSISTENT, "batched": gm.SOLVE_BATCHED,
                               "split": gm.SOLVE_BATCHED | gm.SOLVE_SPLIT}[args.sweep_mode],
                     "tile": args.sweep_tile or 64, "grid": 0}
        log(f"sweep: {n_inst} instances, build {sweep_build:.2f} s, tuned {tuned}")
        I1 = insts()
        gm.gini_mds_solve(I1, 5, tuned["flags"], tuned["tile"], tuned["grid"])
        I1 = insts()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gm.gini_mds_solve(I1, args.sweep_iters, tuned["flags"], tuned["tile"], tuned["grid"])
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        batched_rate = n_inst * args.sweep_iters / tb
        # per-kernel times of the same iterations (HIP events around every launch)
        sweep_kernels = None
        if tuned["flags"] & gm.SOLVE_BATCHED:
            I1 = insts()
            gm.gini_profile_enable(0, True)
            gm.gini_mds_solve(I1, 20, tuned["flags"], tuned["tile"], tuned["grid"])
            torch.cuda.synchronize()
            pr_s = gm.gini_profile_read(0)
            gm.gini_profile_enable(0, False)
            sweep_kernels = {"units_us": round(pr_s["tile_ms"] * 1e3 / max(pr_s["tile_launches"], 1), 2),
                             "reduce_us": round(pr_s["reduce_ms"] * 1e3 / max(pr_s["reduce_launches"], 1), 2)}
        I2 = insts()
        gm.gini_mds_solve(I2, 2, gm.SOLVE_PLAIN, tuned["tile"])
        I2 = insts()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gm.gini_mds_solve(I2, args.plain_iters, gm.SOLVE_PLAIN, tuned["tile"])
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        plain_rate = n_inst * args.plain_iters / tp
        # the persistent single-launch mode, few iterations (it pays one
        # device-scope release per work unit)
        I3 = insts()
        gm.gini_mds_solve(I3, 1, gm.SOLVE_PERSISTENT, tuned["tile"])
        I3 = insts()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gm.gini_mds_solve(I3, args.persistent_iters, gm.SOLVE_PERSISTENT, tuned["tile"])
        torch.cuda.synchronize()
        persistent_rate = n_inst * args.persistent_iters / (time.perf_counter() - t0)
        sweep = {"workload": "16 Gaussian-mixture problems n~U{100..3000} m~U{4..64} x 8 nu in [1.1,4], p=2",
                 "instances": n_inst, "batched_mode": "persistent" if tuned["flags"] == gm.SOLVE_PERSISTENT
                 else ("batched, two streams" if tuned["flags"] & gm.SOLVE_SPLIT else "batched")
                 + (", caller's order" if tuned["flags"] & gm.SOLVE_CALLER_ORDER else ""),
                 "tile": tuned["tile"], "grid": tuned["grid"],
                 "batched_iters_per_s": round(batched_rate, 1), "plain_iters_per_s": round(plain_rate, 1),
                 "persistent_iters_per_s": round(persistent_rate, 1),
                 "sweep_iteration_us": round(1e6 * n_inst / batched_rate, 1),
                 "sweep_iteration_kernels": sweep_kernels,
                 "speedup": round(batched_rate / plain_rate, 2), "batched_iters": args.sweep_iters,
                 "plain_iters": args.plain_iters, "dissim_build_s": round(sweep_build, 3)}
        log(f"sweep batched {batched_rate:.0f} it/s, plain {plain_rate:.0f} it/s, x{batched_rate / plain_rate:.2f}")

    # ---- Algorithm 1 (nu selection) on the Gaussian-mixture workload
    select = None
    if not args.no_select:
        wg = synth.workload_gmm()
        Xg = torch.from_numpy(wg.X).to(dev)
        Zg = torch.from_numpy(wg.Z0[0]).to(dev)
        gm.gini_select_nu(Xg, wg.nus, Zg, 5)                   # warm the library (tables, workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bi, ks_mean, _, _ = gm.gini_select_nu(Xg, wg.nus, Zg, wg.iters)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        select = {"workload": f"Gaussian mixture n={wg.X.shape[0]} m={wg.X.shape[1]}, nu in {wg.nus}, p=2 Gini "
                              f"latent, {wg.iters} descent steps per nu, one fold",
                  "seconds": round(ts, 4), "nu_star": wg.nus[bi],
                  "ks_mean": [round(float(v), 6) for v in ks_mean]}
        log(f"select: nu* = {wg.nus[bi]} in {ts * 1e3:.1f} ms, KS {select['ks_mean']}")

    out = {"metric": METRIC, "value": round(value, 1), "unit": "pair-evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": (f"heavy-tailed n={n} m={m} (iid Student-t, 3 degrees of freedom), nu=2, "
                                   f"p={p} Gini latent, raw stress, fixed-step descent") if heavy else
                                  (f"images n={n} m={m} (28x28 blobs, uint8 + N(0,32^2) noise), nu=2, "
                                   f"p={p} Gini latent, raw stress, fixed-step descent"),
                      "n": n, "m": m, "p": p, "nu": nu, "mode": mode_name, "tile": best["tile"],
                      "parallelism": "single GPU"},
           "hbm_gbs_algorithmic": round(achieved, 1),
           "dissim_build_s": round(dissim_s, 4),
           "roofline": roof, "sweep": sweep, "select": select, "extras": extras, "cpu_baseline": cpu,
           "errors": errors}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
