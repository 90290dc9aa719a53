"""Benchmark of the incomplete-LU hot path on one MI355X.

Workload: 3D 7-point Laplacian on a 128^3 grid (n = 2,097,152, nnz = 14,581,760),
FP64 CSR in natural ordering, b ~ U[-1, 1] from a seed; with it the 96^3 upwind
convection-diffusion matrix (n = 884,736) for the GMRES half of the metric.  One
step is one pass of the whole hot path over these inputs, already resident in HBM:

  128^3: ILU(0) numeric factor with its FP32 copy
         one FP64 apply and one FP32-factor apply of M^{-1} (level ordering)
         one spmv (level ordering)
         PCG to a 1e-10 relative residual with FP64 factors, then with FP32 factors
  96^3:  ILU(1, tau = 1e-3) factor with FP32 and BF16 copies, then FGMRES(30) to
         1e-10 with FP64, FP32 and BF16 factors

`value` is the factor + FP64 apply throughput in GB/s of algorithmic bytes
(factor 20 nnz_LU + 8 n, apply 12 nnz_LU + 16 n + 32 n: b in, y out, y in, x out)
over the whole ilu_factor call (every kernel it launches: arming, the factor, the
spmv value gather, the FP32 cast) plus the whole apply call, medians of 20 calls
each with the 256 MB last-level cache flushed before every call ("cold"); the warm
figure is reported beside it.  Durations come from HIP events the library records
on the launch stream around each call and each kernel.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --workload convdiff3d_96 | random_1m | batch512   (other workloads)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ILU factor + L/U apply GB/s & GMRES time to 1e-10, FP64 vs FP32-factor form"
HBM_PEAK_GBS = 8000.0

# HBM traffic of the solve kernels per launch on this workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) over one bench step,
# scaled by what the same counters read for the calibration copy kernels.  Valid
# only for the kernel source it was taken with: a different hash reports null.
PMC_TRAFFIC = dict(
    kernels_sha256="c6dbd0da594b7ddef98eb472e211bf4b515bb86fd4a8788bbc6ee5512f133dbe",
    fetch_scale=1.9986, write_scale=0.9944,
    forward=dict(f64=(194165, 51157), f32=(166217, 37773)),
    backward=dict(f64=(193308, 81933), f32=(151189, 66715)),
    factor=(217397, 323584),
)


def kernels_sha256():
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1812_06160_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_model(n, nnz_lu, nnz_l, nnz_b, s_v=8, s_x=8, nrhs=1):
    nnz_u = nnz_lu - nnz_l
    return dict(
        factor=20 * nnz_lu + 8 * n,
        apply=(4 + s_v) * nnz_lu + 16 * n + nrhs * 4 * s_x * n,
        forward=(4 + s_v) * nnz_l + 8 * n + nrhs * 2 * s_x * n,
        backward=(4 + s_v) * nnz_u + 8 * n + nrhs * 2 * s_x * n,
        spmv=12 * nnz_b + 4 * (n + 1) + nrhs * 2 * s_x * n,
    )


def host_cpu():
    """CPU model and current clock of this host (Linux /proc/cpuinfo)."""
    model, mhz = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and model is None:
                    model = v.strip()
                elif k == "cpu MHz" and mhz is None:
                    mhz = float(v)
                if model is not None and mhz is not None:
                    break
    except OSError:
        pass
    return model, mhz


def cpu_baseline(A, b_perm, b, A3, b3, budget_s=12.0):
    """The oracle (serial FP64 C, one core) on the same inputs: ILU(0) factor + FP64
    apply of the 128^3 matrix (median of up to 5 runs), PCG to 1e-10 on it, and
    ILU(1, 1e-3) + FGMRES(30) to 1e-10 on the 96^3 convection-diffusion matrix."""
    import oracle as O
    t0 = time.perf_counter()
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    t_an = time.perf_counter() - t0
    tf, ta, reps = [], [], 0
    f = None
    while reps < 5 and (reps < 1 or sum(tf) + sum(ta) < budget_s):
        t0 = time.perf_counter()
        f = O.factor(an, A.val)
        t1 = time.perf_counter()
        O.apply(an, f.val, b_perm, permuted=True)
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        ta.append(t2 - t1)
        reps += 1
    t0 = time.perf_counter()
    _, it_cg, _, _ = O.pcg(an, O.b_values(an, A.val), f.val, b)
    t_cg = time.perf_counter() - t0
    an3 = O.analyze(A3.n, A3.row_ptr, A3.col_idx, k_max=1)
    t0 = time.perf_counter()
    f3 = O.factor(an3, A3.val, k=1, tau=1e-3)
    t_f3 = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it_gm, rr_gm, _ = O.fgmres(an3, O.b_values(an3, A3.val), f3.val, b3)
    t_gm = time.perf_counter() - t0
    return dict(t_factor=float(np.median(tf)), t_apply=float(np.median(ta)), reps=reps, t_analyze=t_an,
                pcg_s=t_cg, pcg_iters=it_cg, cd_factor_s=t_f3, gmres_s=t_gm, gmres_iters=it_gm)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0, help="grid scale (1.0 = 128^3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sched", default="tiled", choices=["tiled", "syncfree", "level"],
                    help="launch scheme of the factor")
    ap.add_argument("--solve-sched", default="tiled", choices=["tiled", "syncfree", "level"],
                    help="launch scheme of the triangular solves")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="a tuning knob of the handles (ilu_set_tuning), repeatable")
    ap.add_argument("--workload", default="laplace3d_128",
                    choices=["laplace3d_128", "laplace2d_64", "convdiff3d_96", "random_1m", "batch512", "heavy_1m",
                             "ordering", "levels"])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "laplace3d_128":
        import bench_workloads
        bench_workloads.run(args)
        return

    import torch
    import synth
    import paper_1812_06160_amd as jv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    jv.load()
    log("generating workload ...")
    A, b = synth.workload(2, scale=args.scale)
    n = A.n
    log(f"n={n} nnz={A.nnz}; analysis ...")
    t0 = time.perf_counter()
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    t_analyze = time.perf_counter() - t0
    ilu.set_schedule(args.sched, args.solve_sched)
    for kv in args.tune:
        key, val = kv.split("=")
        ilu.set_tuning(key, int(val))
    info = ilu.info()
    sched = ilu.schedule()
    nnz_l = int((sched["diag_pos"] - sched["lu_row_ptr"][:-1]).sum())
    a_d = torch.from_numpy(A.val).cuda()
    b_d = torch.from_numpy(b).cuda()
    perm = torch.from_numpy(sched["perm"].astype(np.int64)).cuda()
    bp_d = b_d[perm].contiguous()
    x_d = torch.empty_like(bp_d)
    y_d = torch.empty_like(bp_d)
    B64 = bytes_model(n, info["nnz_lu"], nnz_l, info["nnz_b"], s_v=8)
    B32 = bytes_model(n, info["nnz_lu"], nnz_l, info["nnz_b"], s_v=4)

    # the GMRES half of the metric: 96^3 convection-diffusion, ILU(1, tau = 1e-3)
    A3, b3 = synth.workload(3)
    log(f"convdiff3d_96: n={A3.n} nnz={A3.nnz}; analysis ...")
    cd = jv.Ilu(A3.n, A3.row_ptr, A3.col_idx, k_max=1)
    for kv in args.tune:
        key, val = kv.split("=")
        cd.set_tuning(key, int(val))
    a3_d = torch.from_numpy(A3.val).cuda()
    b3_d = torch.from_numpy(b3).cuda()
    cd_info = cd.info()

    def step():
        ilu.factor(a_d, casts=("f32",))
        ilu.apply(bp_d, x=x_d, permuted=True)
        ilu.apply(bp_d, x=x_d, prec="f32", permuted=True)
        ilu.spmv(bp_d, y=y_d, permuted=True)
        torch.cuda.synchronize()
        t = [time.perf_counter()]
        _, i64 = ilu.pcg(b_d, rtol=1e-10, prec="f64")
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        _, i32 = ilu.pcg(b_d, rtol=1e-10, prec="f32")
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        cd.factor(a3_d, k=1, tau=1e-3, casts=("f32", "bf16"))
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        g = {}
        for prec in ("f64", "f32", "bf16"):
            _, gi = cd.gmres(b3_d, rtol=1e-10, restart=30, prec=prec)
            torch.cuda.synchronize()
            t.append(time.perf_counter())
            g[prec] = (t[-1] - t[-2], gi)
        return dict(pcg64=(t[1] - t[0], i64), pcg32=(t[2] - t[1], i32), cd_factor=t[3] - t[2], gmres=g)

    log("warmup ...")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # stage timings: each stage measured in isolation with the library's events
    ilu.profile(True, capacity=1 << 16)
    stage = {}
    reps = 10
    for name, fn in (("factor", lambda: ilu.factor(a_d, casts=("f32",))),
                     ("apply64", lambda: ilu.apply(bp_d, x=x_d, permuted=True)),
                     ("apply32", lambda: ilu.apply(bp_d, x=x_d, prec="f32", permuted=True)),
                     ("spmv", lambda: ilu.spmv(bp_d, y=y_d, permuted=True))):
        ilu.profile_read()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        stage[name] = ilu.profile_read()

    # per-call distributions, warm and cold (the 256 MB MALL flushed by a 1 GiB
    # write before each call), and cold_clean (flushed by a 1 GiB read instead, so
    # the call does not also pay for writing back the flush's dirty lines): p10 /
    # median / p90 of 20 calls; the factor and apply entries are whole calls (every
    # kernel they launch)
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    dist = {}
    for name, fn, keys in (("factor_call", lambda: ilu.factor(a_d, casts=("f32",)), ("factor_call",)),
                           ("apply_f64_call", lambda: ilu.apply(bp_d, x=x_d, permuted=True), ("apply_call",)),
                           ("factor_kernel", lambda: ilu.factor(a_d, casts=("f32",)), ("factor",)),
                           ("apply_f64_kernels", lambda: ilu.apply(bp_d, x=x_d, permuted=True),
                            ("forward", "backward")),
                           ("spmv", lambda: ilu.spmv(bp_d, y=y_d, permuted=True), ("spmv",))):
        for mode in ("warm", "cold", "cold_clean"):
            vals = []
            for _ in range(20):
                if mode == "cold":
                    flush.add_(1.0)
                elif mode == "cold_clean":
                    flush.sum()
                torch.cuda.synchronize()
                ilu.profile_read()
                fn()
                torch.cuda.synchronize()
                p = ilu.profile_read()
                vals.append(1e3 * sum(p[k][0] for k in keys))
            q = np.percentile(vals, [10, 50, 90])
            dist.setdefault(name, {})[mode] = [round(float(v), 2) for v in q]
    del flush

    # timed steps (events stay on: they are the live per-kernel durations)
    log(f"timing {args.steps} steps ...")
    ilu.profile_read()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        r = step()
        te = time.perf_counter()
        recs.append(r)
        log(f"  step {i}: {1e3 * (te - ts):.1f} ms  pcg64 {r['pcg64'][1]['iters']} it  "
            f"pcg32 {r['pcg32'][1]['iters']} it  gmres {[r['gmres'][p][1]['iters'] for p in ('f64', 'f32', 'bf16')]}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    prof = ilu.profile_read()

    # modified ILU(0) on the same matrix (outside the timed steps): factor time and PCG
    ilu.profile_read()
    for _ in range(5):
        ilu.factor(a_d, casts=(), milu=True)
    torch.cuda.synchronize()
    pm = ilu.profile_read()
    t_a = time.perf_counter()
    _, im = ilu.pcg(b_d, rtol=1e-10, prec="f64")
    torch.cuda.synchronize()
    milu = dict(factor_us=round(1e3 * pm["factor"][0] / max(pm["factor"][1], 1), 2),
                pcg_f64=dict(seconds=round(time.perf_counter() - t_a, 5), iters=im["iters"],
                             true_relres=im["true_relres"]))
    ilu.factor(a_d, casts=("f32",))

    def avg(p, key):
        ms, cnt = p[key]
        return ms / max(cnt, 1), cnt

    t_factor, _ = avg(stage["factor"], "factor")
    t_factor_call, _ = avg(stage["factor"], "factor_call")
    t_fwd64, _ = avg(stage["apply64"], "forward")
    t_bwd64, _ = avg(stage["apply64"], "backward")
    t_app64_call, _ = avg(stage["apply64"], "apply_call")
    t_fwd32, _ = avg(stage["apply32"], "forward")
    t_bwd32, _ = avg(stage["apply32"], "backward")
    t_spmv, _ = avg(stage["spmv"], "spmv")
    t_apply64 = t_fwd64 + t_bwd64
    t_apply32 = t_fwd32 + t_bwd32
    # headline: whole calls, cold medians (us); warm medians beside it
    fb = B64["factor"] + B64["apply"]
    cold_us = dist["factor_call"]["cold"][1] + dist["apply_f64_call"]["cold"][1]
    warm_us = dist["factor_call"]["warm"][1] + dist["apply_f64_call"]["warm"][1]
    value = fb / (cold_us * 1e-6) / 1e9
    value_warm = fb / (warm_us * 1e-6) / 1e9

    # dominant kernel over the timed steps (kernel stages only)
    tot = {k: v[0] for k, v in prof.items() if k in ("factor", "forward", "backward", "spmv")}
    dom = max(tot, key=tot.get)
    dom_ms, dom_cnt = avg(prof, dom)
    # per-launch algorithmic bytes of that kernel over the timed steps: the FP64 and
    # FP32-factor applies alternate, so weight by the launches of each
    n_it64 = sum(r["pcg64"][1]["iters"] for r in recs)
    n_it32 = sum(r["pcg32"][1]["iters"] for r in recs)
    if dom in ("forward", "backward"):
        c64 = args.steps * 1 + n_it64 + len(recs)      # apply64 per step + PCG applies
        c32 = args.steps * 1 + n_it32 + len(recs)
        per_launch = (c64 * B64[dom] + c32 * B32[dom]) / max(c64 + c32, 1)
    else:
        per_launch = B64[dom]
    achieved = per_launch / (dom_ms * 1e-3) / 1e9
    traffic = None
    if dom in ("forward", "backward", "factor") and kernels_sha256() == PMC_TRAFFIC["kernels_sha256"]:
        def scaled(fw):
            return 1024.0 * (fw[0] * PMC_TRAFFIC["fetch_scale"] + fw[1] * PMC_TRAFFIC["write_scale"])
        t = PMC_TRAFFIC[dom]
        if dom == "factor":
            traffic = int(scaled(t))
        else:
            traffic = int((c64 * scaled(t["f64"]) + c32 * scaled(t["f32"])) / max(c64 + c32, 1))
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom,
                    launches=dom_cnt, avg_us=round(dom_ms * 1e3, 2),
                    bytes_per_launch=int(per_launch))

    from paper_1812_06160_amd.calibrate import calibrate
    calib = calibrate(1 << 30)
    roofline["measured_read_gbs"] = calib["read_gbs"]
    roofline["frac_of_measured"] = round(achieved / calib["read_gbs"], 4)
    roofline["hop_ns"] = calib["hop_ns_same_xcd"]
    roofline["latency_floor_us"] = round((info["n_levels"] if dom == "forward" else info["n_ulevels"])
                                         * calib["hop_ns_same_xcd"] * 1e-3, 1) if dom in ("forward", "backward") else None

    def med(xs):
        return round(float(np.median(xs)), 5)

    pcg = dict(f64=dict(seconds=med([r["pcg64"][0] for r in recs]), iters=recs[-1]["pcg64"][1]["iters"],
                        true_relres=recs[-1]["pcg64"][1]["true_relres"]),
               f32_factor=dict(seconds=med([r["pcg32"][0] for r in recs]), iters=recs[-1]["pcg32"][1]["iters"],
                               true_relres=recs[-1]["pcg32"][1]["true_relres"]))
    pcg["speedup_f32_over_f64"] = round(pcg["f64"]["seconds"] / pcg["f32_factor"]["seconds"], 3)
    gm = {}
    for prec in ("f64", "f32", "bf16"):
        gm[prec] = dict(seconds=med([r["gmres"][prec][0] for r in recs]),
                        iters=recs[-1]["gmres"][prec][1]["iters"],
                        true_relres=recs[-1]["gmres"][prec][1]["true_relres"])
    gm["speedup_f32_over_f64"] = round(gm["f64"]["seconds"] / gm["f32"]["seconds"], 3)
    gm["speedup_bf16_over_f64"] = round(gm["f64"]["seconds"] / gm["bf16"]["seconds"], 3)
    gm["factor_call_s"] = med([r["cd_factor"] for r in recs])
    gm["config"] = dict(workload="convdiff3d_96: 96^3 first-order upwind convection-diffusion, velocity "
                                 "(1, 0.5, 0.25), cell Peclet 10, ILU(1, tau=1e-3), FGMRES(30) to 1e-10",
                        n=A3.n, nnz=A3.nnz, nnz_lu=cd_info["nnz_lu"], levels=cd_info["n_levels"])
    out = dict(
        metric=METRIC, value=round(value, 2), unit="GB/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(1e3 * t_total / args.steps, 3), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="laplace3d_128: 3D 7-point Laplacian, 128^3 grid, natural ordering, FP64 CSR, "
                             "ILU(0), b ~ U[-1,1]",
                    n=n, nnz=A.nnz, nnz_lu=info["nnz_lu"], levels=info["n_levels"], schedule=args.sched,
                    solve_schedule=args.solve_sched),
        value_def="(factor + FP64 apply algorithmic bytes) / (median cold ilu_factor call + median cold "
                  "apply call), whole calls with every kernel they launch",
        value_warm=round(value_warm, 2),
        roofline=roofline,
        stages_us=dict(factor_call=round(1e3 * t_factor_call, 2), factor=round(1e3 * t_factor, 2),
                       apply_f64_call=round(1e3 * t_app64_call, 2),
                       forward_f64=round(1e3 * t_fwd64, 2),
                       backward_f64=round(1e3 * t_bwd64, 2), forward_f32=round(1e3 * t_fwd32, 2),
                       backward_f32=round(1e3 * t_bwd32, 2), spmv=round(1e3 * t_spmv, 2)),
        stages_gbs=dict(factor_call=round(B64["factor"] / t_factor_call / 1e6, 1),
                        factor=round(B64["factor"] / t_factor / 1e6, 1),
                        apply_f64=round(B64["apply"] / t_apply64 / 1e6, 1),
                        apply_f32=round(B32["apply"] / t_apply32 / 1e6, 1),
                        spmv=round(B64["spmv"] / t_spmv / 1e6, 1),
                        spmv_cold=round(B64["spmv"] / dist["spmv"]["cold"][1] / 1e3, 1),
                        spmv_cold_clean=round(B64["spmv"] / dist["spmv"]["cold_clean"][1] / 1e3, 1)),
        rows_per_s=dict(factor=round(n / (t_factor_call * 1e-3), 1)),
        calls_us_p10_p50_p90=dist,
        pcg=pcg,
        gmres_convdiff3d_96=gm,
        milu=milu,
        analyze_s=round(t_analyze, 3),
        calibration=calib,
    )
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        bperm = np.ascontiguousarray(b[sched["perm"]])
        cb = cpu_baseline(A, bperm, b, A3, b3)
        cval = fb / (cb["t_factor"] + cb["t_apply"]) / 1e9
        model, mhz = host_cpu()
        out["cpu_baseline"] = dict(
            value=round(cval, 3), unit="GB/s", cores=1, kind="oracle",
            sample=f"serial FP64 oracle, one host core: ILU(0) factor + one FP64 apply of the full 128^3 "
                   f"Laplacian, median of {cb['reps']} runs (factor {cb['t_factor']:.3f} s, apply "
                   f"{cb['t_apply']:.3f} s); PCG to 1e-10 on it ({cb['pcg_iters']} it, {cb['pcg_s']:.2f} s); "
                   f"ILU(1, 1e-3) of convdiff3d_96 ({cb['cd_factor_s']:.3f} s) and FGMRES(30) to 1e-10 "
                   f"({cb['gmres_iters']} it, {cb['gmres_s']:.2f} s)",
            pcg_f64_s=round(cb["pcg_s"], 3), gmres_f64_s=round(cb["gmres_s"], 3),
            cpu_model=model, cpu_mhz=mhz, host_cpus=os.cpu_count())
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
