"""Benchmark of the incomplete-LU hot path on one MI355X.

Workload: 3D 7-point Laplacian on a 128^3 grid (n = 2,097,152, nnz = 14,581,760),
FP64 CSR in natural ordering, b ~ U[-1, 1] from a seed.  One step is one pass of
the whole hot path over that input, already resident in HBM:

  ILU(0) numeric factor (+ FP32/BF16 copies of the factor)
  one FP64 apply and one FP32-factor apply of M^{-1} (level ordering)
  one spmv (level ordering)
  PCG to a 1e-10 relative residual with FP64 factors, then with FP32 factors

`value` is the factor + FP64 apply throughput in GB/s of algorithmic bytes:
factor 20 nnz_LU + 8 n, apply 12 nnz_LU + 16 n + 32 n (b in, y out, y in, x out).
Kernel durations come from HIP events the library records around each kernel
launch on its own stream during the timed steps.

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
    kernels_sha256="a9eee54bbd52941742d98d9ad40a00e2d4778a8832d729e5a085bc9e9ac1763b",
    fetch_scale=1.9987, write_scale=0.9945,
    forward=dict(f64=(209072, 66171), f32=(159291, 50766)),
    backward=dict(f64=(211735, 94306), f32=(150668, 77626)),
    factor=(281816, 146456),
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


def cpu_baseline(A, b, budget_s=12.0):
    """The oracle (serial FP64 C, one core) on the same matrix: factor + FP64 apply."""
    import oracle as O
    t0 = time.perf_counter()
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    t_an = time.perf_counter() - t0
    tf, ta, reps = [], [], 0
    while reps < 5 and (reps < 1 or sum(tf) + sum(ta) < budget_s):
        t0 = time.perf_counter()
        f = O.factor(an, A.val)
        t1 = time.perf_counter()
        O.apply(an, f.val, b, permuted=True)
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        ta.append(t2 - t1)
        reps += 1
    return an, dict(t_factor=float(np.median(tf)), t_apply=float(np.median(ta)), reps=reps, t_analyze=t_an)


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
    ap.add_argument("--workload", default="laplace3d_128",
                    choices=["laplace3d_128", "laplace2d_64", "convdiff3d_96", "random_1m", "batch512", "heavy_1m",
                             "ordering"])
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

    def step():
        ilu.factor(a_d, casts=("f32",))
        ilu.apply(bp_d, x=x_d, permuted=True)
        ilu.apply(bp_d, x=x_d, prec="f32", permuted=True)
        ilu.spmv(bp_d, y=y_d, permuted=True)
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        _, i64 = ilu.pcg(b_d, rtol=1e-10, prec="f64")
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        _, i32 = ilu.pcg(b_d, rtol=1e-10, prec="f32")
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        return i64, i32, t_b - t_a, t_c - t_b

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
    # write before each call): p10 / median / p90 of 20 calls per stage
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    dist = {}
    for name, fn, keys in (("factor", lambda: ilu.factor(a_d, casts=()), ("factor",)),
                           ("apply_f64", lambda: ilu.apply(bp_d, x=x_d, permuted=True), ("forward", "backward")),
                           ("spmv", lambda: ilu.spmv(bp_d, y=y_d, permuted=True), ("spmv",))):
        for mode in ("warm", "cold"):
            vals = []
            for _ in range(20):
                if mode == "cold":
                    flush.add_(1.0)
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
    pcg64, pcg32 = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        i64, i32, d64, d32 = step()
        te = time.perf_counter()
        pcg64.append((d64, i64))
        pcg32.append((d32, i32))
        log(f"  step {i}: {1e3 * (te - ts):.1f} ms  pcg64 {i64['iters']} it  pcg32 {i32['iters']} it")
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

    def avg(p, key):
        ms, cnt = p[key]
        return ms / max(cnt, 1), cnt

    t_factor, _ = avg(stage["factor"], "factor")
    t_fwd64, _ = avg(stage["apply64"], "forward")
    t_bwd64, _ = avg(stage["apply64"], "backward")
    t_fwd32, _ = avg(stage["apply32"], "forward")
    t_bwd32, _ = avg(stage["apply32"], "backward")
    t_spmv, _ = avg(stage["spmv"], "spmv")
    t_apply64 = t_fwd64 + t_bwd64
    t_apply32 = t_fwd32 + t_bwd32
    value = (B64["factor"] + B64["apply"]) / ((t_factor + t_apply64) * 1e-3) / 1e9

    # dominant kernel over the timed steps
    tot = {k: v[0] for k, v in prof.items()}
    dom = max(tot, key=tot.get)
    dom_ms, dom_cnt = avg(prof, dom)
    # per-launch algorithmic bytes of that kernel over the timed steps: the FP64 and
    # FP32-factor applies alternate, so weight by the launches of each
    n_it64 = sum(p[1]["iters"] for p in pcg64)
    n_it32 = sum(p[1]["iters"] for p in pcg32)
    if dom in ("forward", "backward"):
        c64 = args.steps * 1 + n_it64 + len(pcg64)      # apply64 per step + PCG applies
        c32 = args.steps * 1 + n_it32 + len(pcg32)
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
    out = dict(
        metric=METRIC, value=round(value, 2), unit="GB/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(1e3 * t_total / args.steps, 3), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="laplace3d_128: 3D 7-point Laplacian, 128^3 grid, natural ordering, FP64 CSR, "
                             "ILU(0), b ~ U[-1,1]",
                    n=n, nnz=A.nnz, nnz_lu=info["nnz_lu"], levels=info["n_levels"], schedule=args.sched,
                    solve_schedule=args.solve_sched),
        roofline=roofline,
        stages_us=dict(factor=round(1e3 * t_factor, 2), forward_f64=round(1e3 * t_fwd64, 2),
                       backward_f64=round(1e3 * t_bwd64, 2), forward_f32=round(1e3 * t_fwd32, 2),
                       backward_f32=round(1e3 * t_bwd32, 2), spmv=round(1e3 * t_spmv, 2)),
        stages_gbs=dict(factor=round(B64["factor"] / t_factor / 1e6, 1),
                        apply_f64=round(B64["apply"] / t_apply64 / 1e6, 1),
                        apply_f32=round(B32["apply"] / t_apply32 / 1e6, 1),
                        spmv=round(B64["spmv"] / t_spmv / 1e6, 1)),
        rows_per_s=dict(factor=round(n / (t_factor * 1e-3), 1)),
        calls_us_p10_p50_p90=dist,
        pcg=dict(f64=dict(seconds=round(float(np.median([p[0] for p in pcg64])), 5),
                          iters=pcg64[-1][1]["iters"], true_relres=pcg64[-1][1]["true_relres"]),
                 f32_factor=dict(seconds=round(float(np.median([p[0] for p in pcg32])), 5),
                                 iters=pcg32[-1][1]["iters"], true_relres=pcg32[-1][1]["true_relres"])),
        milu=milu,
        analyze_s=round(t_analyze, 3),
        calibration=calib,
    )
    out["pcg"]["speedup_f32_over_f64"] = round(out["pcg"]["f64"]["seconds"] / out["pcg"]["f32_factor"]["seconds"], 3)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        bperm = np.ascontiguousarray(b[sched["perm"]])
        _, cb = cpu_baseline(A, bperm)
        cval = (B64["factor"] + B64["apply"]) / (cb["t_factor"] + cb["t_apply"]) / 1e9
        out["cpu_baseline"] = dict(value=round(cval, 3), unit="GB/s", cores=1, kind="oracle",
                                   sample=f"serial FP64 oracle: ILU(0) factor + one FP64 apply of the full "
                                          f"128^3 Laplacian, median of {cb['reps']} runs "
                                          f"(factor {cb['t_factor']:.3f} s, apply {cb['t_apply']:.3f} s); "
                                          f"PCG not run on the CPU",
                                   host_cpus=os.cpu_count())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
