"""Benchmark of the DMK point code on one MI355X.

One step = one dmk_eval over the whole hot path (charge gather, upward pass,
root window, plane-wave stages of every level, leaf evaluation, residual
sums, scatter) on a plan built once outside the timed region, with points
and charges resident in HBM.  The timed run is the mixed-precision path in
batched mode (the eval core replayed from a HIP graph, residual sums on a
concurrent stream); the plain FP64 path (eager launches) is timed beside it
on the same points.  A separate eager pass with HIP events around every
launch gives the per-stage times and the roofline of the dominant kernel.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--precision fp64|mixed] [--no-batched] [--no-compare]
                  [--no-cpu-baseline] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s, 3D Laplace DMK at 1e-6 rel ℓ2: mixed+batched vs plain FP64, 1 GPU"
PEAK = {"hbm": (8000.0, "GB/s"), "alu64": (78.6, "TFLOP/s"), "alu32": (157.3, "TFLOP/s")}  # fp32 MFMA dense: also 157.3
# bound of each stage: memory streams vs arithmetic on the vector ALUs
STAGE_BOUND = {"gather": "hbm", "finalize": "hbm", "pwshift": "hbm", "upward": "alu", "root": "alu",
               "proxy2pw": "alu", "local": "alu", "pw2grid": "alu", "leaf": "alu", "residual": "alu"}
STAGE_KERNEL = {"gather": "k_gather_q", "upward": "k_upward_q", "root": "k_root_stage",
                "proxy2pw": "k_proxy2pw_mfma", "local": "k_local_mfma_q", "pwshift": "k_pwshift",
                "pw2grid": "k_local_mfma_q", "leaf": "k_leaf_mfma", "residual": "k_residual",
                "finalize": "k_finalize"}
STAGE_KERNEL2 = {"gather": "k_gather_q2", "upward": "k_upward2", "root": "k_root2", "proxy2pw": "k_proxy2pw2",
                 "local": "k_local_pw2", "pwshift": "k_pwshift2", "pw2grid": "k_local_pw2", "leaf": "k_leaf2",
                 "residual": "k_residual2", "finalize": "k_finalize2"}
WORKLOADS = {
    "cfg3_clustered_10m": "3-D Laplace, N=1e7 clustered (70% on the unit sphere, 30% in 3 Gaussian "
                          "blobs sigma=1e-3), charges U[-1,1], leaf<=64, tol 1e-6",
    "cfg2_uniform_1m": "3-D Laplace, N=1e6 uniform in the unit cube, charges U[-1,1], leaf<=64, tol 1e-6",
    "cfg1_uniform_2k": "3-D Laplace, N=2000 uniform in the unit cube, leaf<=50, tol 1e-6",
    "cfg4_batch2d_512": "2-D batch of 512 independent problems, N_b = exp(U[ln 1e3, ln 2e5]) "
                        "(1.79e7 points), U[0,1]^2 or 0.5+0.01 N(0,I) per problem, charges U[-1,1], leaf<=64, "
                        "tol 1e-6; kernel -log(r)/(2 pi) or K_0(10 r) (--kernel)",
    "cfg5_volume_8gauss": "3-D volume potential on [-1/2,1/2]^3 of rho = sum of 8 Gaussians exp(-|x-c|^2/s^2), "
                          "s = exp(U[ln 1e-3, ln 1e-1]), c ~ U[-0.3,0.3]^3; adaptive tree of 8^3 Chebyshev leaves "
                          "(density resolved to 3e-8 of its peak, leaves <= 4 s at each centre), 4.0e7 nodes; "
                          "Gaussian split at tol 1e-3, PSWF split at 1e-6 (--vol-tol; same tree) (--precision: mixed = FP32 far-field transforms and near-field "
                          "products, FP64 asymptotic part and sums)",
}
METRIC_2D = "points/s, 2-D DMK batch of 512 problems at 1e-6 rel l2, 1 GPU"
METRIC_VOL = "points/s, 3-D volume potential DMK (box code) at tol {tol:g}, 1 GPU"
STAGE_KERNEL_VOL = {"upward": "k_vol_upward", "root": "k_root_stage", "proxy2pw": "k_proxy2pw_mfma",
                    "pwshift": "k_pwshift", "pw2grid": "k_local_mfma_q", "leaf": "k_vol_leaf", "residual": "k_vol_near",
                    "finalize": "k_vol_finalize"}
# volume workload: density, refinement and tree limits.  The tree refines
# while a leaf's Chebyshev tail exceeds tol * rho_scale; the product is held
# at 3e-8 for both tolerances, so tol 1e-3 and 1e-6 run on the same tree.
VOL_SEED, VOL_RHO_SCALE, VOL_MAX_LEVEL = 5, 3e-5, 16


def vol_rho_scale(tol):
    return VOL_RHO_SCALE * 1e-3 / tol


# HBM bytes per launch of the dominant kernel, from two rocprofv3 PMC runs of
# this script (--pmc FETCH_SIZE, then --pmc WRITE_SIZE, with --copy-calibration):
# FETCH_SIZE scaled by 2.0, WRITE_SIZE by 1.0, the factors that make the
# elementwise copy of 1 GiB read and write exactly 1 GiB.  Keyed by workload,
# precision and kernel, and valid only for the kernel source it was measured
# on (digest of csrc/eval.hip); otherwise traffic is reported as null.
TRAFFIC = {
    ("cfg3_clustered_10m", "mixed", "k_local_mfma_q"): (1.4569e+10, "63a94a33aab9e114"),
    ("cfg3_clustered_10m", "mixed", "k_upward_q"): (5.1550e+09, "63a94a33aab9e114"),
    ("cfg3_clustered_10m", "mixed", "k_pwshift"): (1.7208e+10, "63a94a33aab9e114"),
}


def per_level(kname, args):
    """the kernel name under --level-launches (the per-level launches drop the _q suffix)"""
    return kname[:-2] if (args.level_launches and kname.endswith("_q")) else kname


def eval_src_digest():
    import hashlib
    path = os.path.join(ROOT, "paper_2308_00292_amd", "csrc", "eval.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline_2d(off, pts, q, ns, tol, kern, lam, seed=7):
    """The oracle on whole problems of the batch, drawn at random until about
    15 s of eval work is done; points/s over the problems it ran."""
    import oracle
    rng = np.random.default_rng(seed)
    pr = oracle.params2_for(tol)
    ps = oracle.PSWF(pr.c)
    done, te = 0, 0.0
    order = rng.permutation(len(off) - 1)
    nprob = 0
    for b in order:
        pb, qb = pts[off[b]:off[b + 1]], q[off[b]:off[b + 1]]
        tr = oracle.Tree(pb, ns)
        t0 = time.perf_counter()
        oracle.dmk_eval(tr, pr, ps, qb, kern=kern, lam=lam)
        te += time.perf_counter() - t0
        done += len(qb)
        nprob += 1
        if te > 15.0:
            break
    return {"value": done / te, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{nprob} whole problems of the batch drawn at random ({done} points), eval phase "
                      f"{te:.2f} s, trees excluded, FP64, tol {tol:g}"}


def morton_runs(pts, m, rng, nrun=8):
    """indices of nrun runs of about m/nrun consecutive points in Morton order
    (10 bits per axis), at random places: spatially compact pieces of the set
    at its own local density, so the oracle's tree over them is as deep
    there as the full tree (a uniform random subset would be sparser and its
    tree shallower)"""
    n = len(pts)
    lo = pts.min(0)
    ext = float((pts.max(0) - lo).max()) or 1.0
    c = np.clip(((pts - lo) / ext * 1024).astype(np.int64), 0, 1023)

    def spread(v):  # 10 bits -> every third bit of 30
        v = (v | (v << 16)) & 0x030000FF
        v = (v | (v << 8)) & 0x0300F00F
        v = (v | (v << 4)) & 0x030C30C3
        return (v | (v << 2)) & 0x09249249

    order = np.argsort((spread(c[:, 0]) << 2) | (spread(c[:, 1]) << 1) | spread(c[:, 2]), kind="stable")
    k = max(1, m // nrun)
    starts = np.sort(rng.choice(max(1, n - k + 1), nrun, replace=False))
    idx = np.unique(np.concatenate([order[s0:s0 + k] for s0 in starts]))
    return idx


def cpu_baseline(pts, q, ns, tol, seed=7):
    """The oracle (plain FP64 C, OpenMP over all host threads) on Morton runs
    of the same point set (morton_runs), sized for roughly 15 s of eval work
    on all threads, then on one thread for roughly 8 s."""
    import oracle
    rng = np.random.default_rng(seed)
    n = len(q)
    idx = morton_runs(pts, min(n, 50_000), rng)
    _, _, te = oracle.dmk_run(pts[idx], q[idx], tol, ns)
    rate = len(idx) / te
    idx = morton_runs(pts, int(min(n, max(100_000, min(3_000_000, rate * 15.0)))), rng)
    m = len(idx)
    _, tp, te = oracle.dmk_run(pts[idx], q[idx], tol, ns)
    cores = oracle.num_threads()
    res = {"value": m / te, "unit": "points/s", "cores": cores, "kind": "oracle",
           "sample": f"8 runs of consecutive points in Morton order at random places ({m} of the {n} points, "
                     f"the full set's local density), eval phase {te:.2f} s, plan {tp:.2f} s excluded, "
                     f"FP64, tol {tol:g}"}
    prev = oracle.set_threads(1)
    try:
        idx1 = morton_runs(pts, int(max(20_000, min(m, (m / te) / cores * 8.0))), rng)
        _, _, te1 = oracle.dmk_run(pts[idx1], q[idx1], tol, ns)
    finally:
        oracle.set_threads(prev)
    res["single_thread"] = {"value": len(idx1) / te1, "cores": 1,
                            "sample": f"8 Morton runs, {len(idx1)} points, eval phase {te1:.2f} s"}
    return res


def cpu_baseline_vol(sig, cen, amp, feat, tol):
    """The volume oracle (plain FP64 C, OpenMP) on the same density with the
    tree cut at level 4 (tol 1e-3) or 3 (tol 1e-6; same refinement rule
    otherwise): points/s of its eval phase."""
    import oracle
    import dmk_inputs
    vp = oracle.vparams_for(tol, 8)
    f = lambda x: dmk_inputs.gaussian_mixture(x, sig, cen, amp)
    cut = 4 if tol == 1e-3 else 3  # 10 to 30 s of eval on 16 threads either way
    T = oracle.VTree(vp, f, vol_rho_scale(tol), 1, cut, features=feat)
    rho = f(T.nodes())
    t0 = time.perf_counter()
    T.eval(rho)
    te = time.perf_counter() - t0
    n = T.nleaf * 512
    return {"value": n / te, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"same density, tree cut at level {cut} ({T.nleaf} leaves, {n} nodes), eval phase {te:.2f} s, "
                      f"tree excluded, FP64, tol {tol:g}"}


def run_volume(args):
    import torch

    import dmk_inputs
    import paper_2308_00292_amd as dmk
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from vol_exact import gauss_mixture_potential  # closed-form reference of the sampled check

    sig, cen, amp = dmk_inputs.vol_gaussians(VOL_SEED)
    f = lambda x: dmk_inputs.gaussian_mixture(x, sig, cen, amp)
    feat = dmk_inputs.gaussian_features(sig, cen)
    prec = dmk.DMK_FP64 if args.precision == "fp64" else dmk.DMK_MIXED
    log(f"[bench] volume plan ({args.precision})")
    t0 = time.perf_counter()
    lvl = dmk.DMK_FLAG_LEVEL_LAUNCHES if args.level_launches else 0
    vtol = args.vol_tol
    plan = dmk.VolPlan(f, tol=vtol, q=8, rho_scale=vol_rho_scale(vtol), min_level=1, max_level=VOL_MAX_LEVEL,
                       features=feat, precision=prec, flags=lvl)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    n = plan.n
    lev, _ = plan.leaves()
    log(f"[bench] plan {t_plan:.2f} s: {plan.nleaf} leaves, {n} nodes")
    xyz = plan.nodes()
    rho = torch.zeros(n, dtype=torch.float64, device="cuda")
    for s_, c_, a_ in zip(sig, cen, amp):
        cc = torch.tensor(c_, dtype=torch.float64, device="cuda")
        rho += a_ * torch.exp(-((xyz - cc) ** 2).sum(dim=1) / (s_ * s_))
    out = torch.empty_like(rho)
    for _ in range(args.warmup):
        plan.eval(rho, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        plan.eval(rho, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms_step * 1e-3)
    log(f"[bench] {ms_step:.3f} ms/step -> {value:.4g} points/s")
    plan.stage_timing(True)
    nst = max(2, min(args.steps, 5))
    for _ in range(nst):
        plan.eval(rho, out)
    torch.cuda.synchronize()
    stage_ms, launches = plan.stage_times()
    plan.stage_timing(False)
    flops, byts = plan.stage_work()
    dom = max(stage_ms, key=lambda k: stage_ms[k])
    avg_ms = stage_ms[dom] / max(1, launches[dom])
    hbm = STAGE_BOUND[dom] == "hbm"
    per_launch = (byts[dom] if hbm else flops[dom]) * nst / max(1, launches[dom])
    achieved = per_launch / (avg_ms * 1e-3) / (1e9 if hbm else 1e12)
    # every stage, the near field included, computes in FP32 in a mixed plan
    peak, unit = PEAK["hbm"] if hbm else (PEAK["alu64"] if prec == dmk.DMK_FP64 else PEAK["alu32"])
    roof = {"bound": STAGE_BOUND[dom], "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": None, "kernel": per_level(STAGE_KERNEL_VOL.get(dom, dom), args), "stage": dom, "avg_launch_ms": avg_ms,
            "launches_per_step": launches[dom] / nst}
    stages = {}
    for k in stage_ms:
        ms = stage_ms[k] / nst
        if ms <= 0:
            continue
        ent = {"ms": round(ms, 4)}
        if flops[k] > 0:
            ent["tflops"] = round(flops[k] / (ms * 1e-3) / 1e12, 3)
        if byts[k] > 0:
            ent["gbps"] = round(byts[k] / (ms * 1e-3) / 1e9, 1)
        stages[k] = ent
    u = out.cpu().numpy()
    idx = np.random.default_rng(3).choice(n, args.sample_targets // 2, replace=False)
    ex = gauss_mixture_potential(xyz.cpu().numpy()[idx], sig, cen, amp)
    err = float(np.linalg.norm(u[idx] - ex) / np.linalg.norm(ex))
    log(f"[bench] sampled rel l2 vs closed form ({len(idx)} nodes): {err:.3e}")
    plan.close()
    fp64 = None
    if not args.no_compare and prec != dmk.DMK_FP64:
        p64 = dmk.VolPlan(f, tol=vtol, q=8, rho_scale=vol_rho_scale(vtol), min_level=1, max_level=VOL_MAX_LEVEL,
                          features=feat, precision=dmk.DMK_FP64, flags=lvl)
        out64 = torch.empty_like(rho)
        for _ in range(args.warmup):
            p64.eval(rho, out64)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            p64.eval(rho, out64)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms64 = ev0.elapsed_time(ev1) / args.steps
        u64 = out64.cpu().numpy()
        p64.close()
        fp64 = {"points_per_s": n / (ms64 * 1e-3), "ms_per_step": ms64,
                "sampled_rel_l2_vs_closed_form": float(np.linalg.norm(u64[idx] - ex) / np.linalg.norm(ex)),
                "rel_l2_vs_main": float(np.linalg.norm(u - u64) / np.linalg.norm(u64))}
        log(f"[bench] FP64 volume {ms64:.3f} ms/step -> {fp64['points_per_s']:.4g} points/s")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (volume oracle)")
        cpu = cpu_baseline_vol(sig, cen, amp, feat, vtol)
        log(f"[bench] cpu baseline {cpu['value']:.4g} points/s on {cpu['cores']} threads")
    res = {
        "metric": METRIC_VOL.format(tol=vtol), "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64" if prec == dmk.DMK_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["cfg5_volume_8gauss"], "name": "cfg5_volume_8gauss", "n_points": n,
                   "precision": args.precision, "fp64": fp64,
                   "schedule": "per-level launches" if args.level_launches else "queue-fed over all levels",
                   "leaves": plan.nleaf, "levels": np.bincount(lev).tolist(), "q": 8, "p": 18, "nf": 12, "tol": vtol,
                   "split": "PSWF (residual: fitted Gaussians + log-t quadrature)" if vtol == 1e-6 else "Gaussian",
                   "t_plan_s": round(t_plan, 3), "sampled_rel_l2_vs_closed_form": err, "stage_ms_per_step": stages},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg3_clustered_10m", choices=list(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--kernel", default="log", choices=["log", "k0"],
                    help="2-D workloads: -log(r)/(2 pi) or K_0(10 r)")
    ap.add_argument("--no-batched", action="store_true",
                    help="launch every stage eagerly instead of replaying the captured graph")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain FP64 (eager) comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--vol-tol", type=float, default=1e-3, choices=[1e-3, 1e-6],
                    help="volume workload: 1e-3 (Gaussian split) or 1e-6 (PSWF split), same tree")
    ap.add_argument("--sample-targets", type=int, default=200)
    ap.add_argument("--level-launches", action="store_true",
                    help="launch the upward and local stages one tree level at a time instead of the "
                         "queue-fed kernels over all levels (DMK_FLAG_LEVEL_LAUNCHES)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run an elementwise copy of 1 GiB first (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "cfg5_volume_8gauss":
        run_volume(args)
        return

    import torch

    import dmk_inputs
    import paper_2308_00292_amd as dmk

    tol = 1e-6
    prec = dmk.DMK_FP64 if args.precision == "fp64" else dmk.DMK_MIXED
    batched = not args.no_batched
    log(f"[bench] generating {args.workload}")
    offsets = None
    kern, lam = dmk.DMK_LAPLACE, 0.0
    if args.workload == "cfg4_batch2d_512":
        offsets, pts, q = dmk_inputs.batch_2d(512, 4)
        ns = 64
        if args.kernel == "k0":
            kern, lam = dmk.DMK_YUKAWA, 10.0
    else:
        pts, q, ns = dmk_inputs.make(args.workload)
    n = len(q)
    dev = torch.device("cuda:0")
    tp_ = torch.from_numpy(pts).to(dev)
    tq = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    if args.copy_calibration:
        # x * 1 through torch's elementwise kernel: reads and writes exactly 2^30 bytes
        src = torch.ones(2**28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 x (read 1 GiB, write 1 GiB)")

    def timed(plan, steps, warmup):
        out = torch.empty(n, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            plan.eval(tq, out)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            plan.eval(tq, out)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, out

    log(f"[bench] plan ({args.precision}{', batched' if batched else ''})")
    t0 = time.perf_counter()
    lvl = dmk.DMK_FLAG_LEVEL_LAUNCHES if args.level_launches else 0
    plan = dmk.Plan(tp_, tol=tol, leaf_max=ns, precision=prec, offsets=offsets, kernel=kern, lam=lam,
                    flags=(dmk.DMK_FLAG_BATCHED if batched else 0) | lvl)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    info = plan.info()
    log(f"[bench] plan {t_plan:.2f} s: levels {info['nlevels']} boxes {info['nbox']} leaves {info['nleaf']}")
    log("[bench] timed region")
    ms_step, out = timed(plan, args.steps, args.warmup)
    value = n / (ms_step * 1e-3)
    log(f"[bench] {ms_step:.3f} ms/step -> {value:.4g} points/s")

    def breakdown(plan, out, prec, pname):
        """per-stage times (HIP events around every launch, eager) and the
        roofline of the dominant stage's kernel"""
        plan.stage_timing(True)
        nst = max(2, min(args.steps, 5))
        for _ in range(nst):
            plan.eval(tq, out)
        torch.cuda.synchronize()
        stage_ms, launches = plan.stage_times()
        plan.stage_timing(False)
        flops, byts = plan.stage_work()
        dom = max(stage_ms, key=lambda k: stage_ms[k])
        avg_ms = stage_ms[dom] / max(1, launches[dom])
        per_launch = (byts[dom] if STAGE_BOUND[dom] == "hbm" else flops[dom]) * nst / max(1, launches[dom])
        if STAGE_BOUND[dom] == "hbm":
            achieved = per_launch / (avg_ms * 1e-3) / 1e9
            peak, unit = PEAK["hbm"]
        else:
            achieved = per_launch / (avg_ms * 1e-3) / 1e12
            peak, unit = PEAK["alu64" if prec == dmk.DMK_FP64 else "alu32"]
        kname = STAGE_KERNEL[dom] if offsets is None else STAGE_KERNEL2[dom]
        kname = per_level(kname, args)
        bound = STAGE_BOUND[dom]
        if "_mfma" in kname:
            bound = "mfma"  # matrix-core products: the dense MFMA peaks equal the vector ones (FP32 157.3, FP64 78.6)
        tr = TRAFFIC.get((args.workload, pname, kname))
        traffic = tr[0] if (tr is not None and tr[1] == eval_src_digest()) else None
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic, "kernel": kname, "stage": dom,
                "avg_launch_ms": avg_ms, "launches_per_step": launches[dom] / nst}
        stages = {}
        for k in stage_ms:
            ms = stage_ms[k] / nst
            ent = {"ms": round(ms, 4)}
            if ms > 0 and flops[k] > 0:
                ent["tflops"] = round(flops[k] / (ms * 1e-3) / 1e12, 3)
            if ms > 0 and byts[k] > 0:
                ent["gbps"] = round(byts[k] / (ms * 1e-3) / 1e9, 1)
            stages[k] = ent
        return roof, stages

    roof, stages = breakdown(plan, out, prec, args.precision)
    u_main = out.cpu().numpy()
    queue_timeouts = plan.info()["queue_timeouts"]
    plan.close()
    del plan

    plain = None
    if not args.no_compare:
        log("[bench] plain FP64 comparison (eager launches)")
        p64 = dmk.Plan(tp_, tol=tol, leaf_max=ns, precision=dmk.DMK_FP64, offsets=offsets, kernel=kern, lam=lam,
                       flags=lvl)
        ms64, out64 = timed(p64, args.steps, args.warmup)
        u64 = out64.cpu().numpy()
        roof64, stages64 = breakdown(p64, out64, dmk.DMK_FP64, "fp64")
        p64.close()
        del p64
        plain = {"points_per_s": n / (ms64 * 1e-3), "ms_per_step": ms64, "roofline": roof64,
                 "stage_ms_per_step": stages64}
        log(f"[bench] plain FP64 {ms64:.3f} ms/step -> {plain['points_per_s']:.4g} points/s")

    # sampled parity against direct summation by the oracle
    import oracle
    rng = np.random.default_rng(11)
    if offsets is None:
        sidx = rng.choice(n, min(n, args.sample_targets), replace=False)
        ud = oracle.direct(pts, q, sidx)
    else:
        # targets of 8 random problems, direct sums over their own problem
        sidx, ud = [], []
        for b in rng.choice(len(offsets) - 1, 8, replace=False):
            o0, o1 = offsets[b], offsets[b + 1]
            ti = rng.choice(o1 - o0, min(o1 - o0, args.sample_targets // 8), replace=False)
            ud.append(oracle.direct2(kern, lam, pts[o0:o1], q[o0:o1], ti))
            sidx.append(o0 + ti)
        sidx, ud = np.concatenate(sidx), np.concatenate(ud)
    err = float(np.linalg.norm(u_main[sidx] - ud) / np.linalg.norm(ud))
    log(f"[bench] sampled rel l2 vs direct sum ({len(sidx)} targets): {err:.3e}")
    if plain is not None:
        plain["sampled_rel_l2_vs_direct"] = float(np.linalg.norm(u64[sidx] - ud) / np.linalg.norm(ud))
        plain["rel_l2_vs_main"] = float(np.linalg.norm(u_main - u64) / np.linalg.norm(u64))

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = (cpu_baseline(pts, q, ns, tol) if offsets is None
               else cpu_baseline_2d(offsets, pts, q, ns, tol, kern, lam))
        log(f"[bench] cpu baseline {cpu['value']:.4g} points/s on {cpu['cores']} threads")

    res = {
        "metric": METRIC if offsets is None else METRIC_2D, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64" if prec == dmk.DMK_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload, "n_points": n,
                   "tol": tol, "leaf_max": ns, "precision": args.precision, "batched": batched,
                   "schedule": ("per-level launches" if (args.level_launches or offsets is not None)
                                else "queue-fed over all levels"),
                   "kernel": ("1/(4 pi r)" if offsets is None else
                              ("-log(r)/(2 pi)" if kern == dmk.DMK_LAPLACE else "K_0(10 r)")),
                   "levels": info["nlevels"], "boxes": info["nbox"], "leaves": info["nleaf"], "residual_candidate_pairs": info["npairs"],
                   "p": info["p"], "nf": info["nf"], "t_plan_s": round(t_plan, 3),
                   "end_to_end_points_per_s": n / (t_plan + ms_step * 1e-3),
                   "sampled_rel_l2_vs_direct": err, "stage_ms_per_step": stages,
                   "plain_fp64": plain, "queue_timeouts": queue_timeouts,
                   "speedup_vs_plain_fp64": (value / plain["points_per_s"]) if plain else None},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
