#!/usr/bin/env python3
"""Benchmark of the probing / multi-shift Krylov log det + gradient on one MI355X.

Workload (the configuration the headline metric is quoted on): the 2-D
512 x 512 lattice with Q = (0.05 I + L)^2 (13-point operator), distance-4
modular colouring (41 probes), N = 20 contour shifts, gradient with respect
to kappa^2 (dQ/dkappa^2 = 2 (kappa^2 I + L)), mixed form (vectors stored in
FP32, all arithmetic in FP64), tol 1e-5 per shifted system and 1e-6 for the
base system.  One step = one full log det + gradient evaluation through the
C ABI with the operator already resident on the device.

Printed: one JSON line with the whole-job throughput (evaluations per second),
the roofline of the dominant kernel (the fused 2-D pass), the plain FP64 form
timed beside it, the error of the timed result against a tight FP64 run of
the same library, and the CPU reference timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pass2d_lattice512_sq_traffic.json")
KERNEL_SOURCES = ["paper_1105_5256_amd/csrc/pass2d.hip", "paper_1105_5256_amd/csrc/tail.h",
                  "paper_1105_5256_amd/csrc/ldq_internal.h"]


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP64-form, CSR-form and accuracy runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM counters)")
    return ap.parse_args()


def cpu_baseline(wl, iters_total, sample_iters=200):
    """The CPU oracle (textbook CG-M with per-shift vectors, FP64) on a bounded
    sample: the first `sample_iters` iterations of probe 0, scaled by the
    workload's total probe-iterations."""
    import numpy as np
    from oracle import colouring, exact, krylov, lattice, shifts

    shape, kappa2 = wl["shape"], wl["kappa2"]
    M = lattice.shifted_laplacian(shape, kappa2)
    Q = lattice.squared(M)
    C, co = colouring.find_modular(2, 2 * wl["k"])
    col = colouring.modular_colouring(shape, C, co)
    v = (col == 0).astype(np.float64)
    lo, hi = exact.spectrum_closed_form(shape, kappa2, 2)
    sig, _ = shifts.log_shifts(lo, hi, 20)
    t0 = time.perf_counter()
    x, X, it = krylov.cg_m(Q, v, sig, tol=1e-30, maxiter=sample_iters)
    _ = x @ (2 * (M @ v))
    dt = time.perf_counter() - t0
    per_iter = dt / it
    eval_s = per_iter * iters_total
    threads = 1
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        pass
    return {"value": 1.0 / eval_s, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"first {it} CG-M iterations (20 shifts, per-shift vectors, FP64) of probe 0 of 41 "
                      f"on the 512x512 13-point lattice, {dt:.1f} s, scaled by the workload's "
                      f"{iters_total} probe-iterations; scipy sparse products and numpy updates run "
                      f"single-threaded (BLAS pool {threads} threads, {os.cpu_count()} host cores)"}


def csr_forms(ctx, wl, nsteps, ref_val, ref_grad):
    """The same workload with Q and dQ/dkappa2 given as CSR matrices (the
    general sparse passes), the same colouring and enclosure as the stencil
    form, timed in the mixed and FP64 forms."""
    import torch

    from paper_1105_5256_amd import ldq, workloads

    shape, kappa2 = wl["shape"], wl["kappa2"]
    n = shape[0] * shape[1]
    lat = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, kappa2))
    col, _ = ldq.ldq_colouring(ctx.handle, lat, wl["k"], ldq.LDQ_COLOUR_MODULAR)
    lo, hi = ldq.ldq_spectrum_bounds(ctx.handle, lat)
    rp, ci, v = workloads.lattice2d_sq_csr(*shape, kappa2=kappa2)
    Q = ctx.op(ldq.ldq_op_csr(ctx.handle, n, rp, ci, v))
    rp, ci, v = workloads.lattice2d_5pt_csr(*shape, kappa2=kappa2, scale=2.0)
    dQ = ctx.op(ldq.ldq_op_csr(ctx.handle, n, rp, ci, v))
    res = {}
    for name, prec, tol, gtol in [("csr_mixed", ldq.LDQ_MIXED, 1e-5, 1e-6), ("csr_fp64", ldq.LDQ_FP64, 1e-5, 1e-6)]:
        opts = ldq.ldq_options_default(k=wl["k"], nshifts=20, tol=tol, grad_tol=gtol, precision=prec,
                                       colouring=ldq.LDQ_COLOUR_USER, user_colours=col, lambda_min=lo,
                                       lambda_max=hi)
        ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            cv, cg, ci_ = ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], opts)
        torch.cuda.synchronize()
        cdt = (time.perf_counter() - t0) / nsteps
        res[name] = {"evals_per_s": round(1.0 / cdt, 3), "ms": round(cdt * 1e3, 3),
                     "gbs": round(ci_["bytes_model"] / ci_["loop_seconds"] / 1e9, 1),
                     "iters_max": ci_["iters_max"],
                     "rel_err_vs_tight_fp64": {"logdet": abs(cv - ref_val) / abs(ref_val),
                                               "grad": abs(cg[0] - ref_grad) / abs(ref_grad)}}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(on several GPUs the probes would be split between ranks and their terms summed with one all-reduce of a few doubles; this build measures one GPU)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1105_5256_amd import ldq, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = workloads.lattice2d_sq(512, kappa2=0.05, k=4)
    shape, kappa2 = wl["shape"], wl["kappa2"]
    ctx = ldq.Context(0)
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, kappa2))
    dQ = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, kappa2, scale=2.0))
    mixed = ldq.ldq_options_default(k=4, nshifts=20, tol=1e-5, grad_tol=1e-6, precision=ldq.LDQ_MIXED)

    for _ in range(args.warmup):
        ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], mixed)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        val, grad, info = ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], mixed)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt

    kern_s = sum(i["loop_seconds"] for i in infos)
    kern_bytes = sum(i["bytes_model"] for i in infos)
    launches = sum(i["passes"] for i in infos)
    achieved = kern_bytes / kern_s / 1e9
    last = infos[-1]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "pass2d_fast<float, R=2, no observations, 1 gradient> (fused 2-D pass)",
                "avg_launch_us": round(kern_s / launches * 1e6, 2),
                "bytes_per_launch": round(kern_bytes / launches),
                "bytes_model": "16 B per site per active probe (r and p read and written once, FP32)"}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            roofline["traffic"] = tr["bytes_per_launch"]
            roofline["traffic_note"] = tr.get("note", "")

    out = {
        "metric": "log det Q evals/s + SpMM HBM GB/s at rel. err 1e-4 vs FP64; fwd+grad",
        "value": round(value, 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lattice512_sq: 2-D 512x512 lattice, Q = (0.05 I + L)^2 (13-point), "
                               "distance-4 modular colouring (41 probes), N=20 shifts, log det + d/dkappa2",
                   "n": 512 * 512, "probes": last["ncolours"], "nshifts": 20, "tol": 1e-5, "grad_tol": 1e-6,
                   "storage": "f32 vectors, f64 arithmetic", "iters_max": last["iters_max"],
                   "parallelism": "one GPU"},
        "roofline": roofline,
    }

    if not args.no_forms:
        # accuracy: the timed result against a tight FP64 run of the same library
        tight = ldq.ldq_options_default(k=4, nshifts=20, tol=1e-10, grad_tol=1e-10, precision=ldq.LDQ_FP64)
        ref_val, ref_grad, _ = ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], tight)
        # plain FP64 form at the same tolerances as the timed mixed form
        fp64 = ldq.ldq_options_default(k=4, nshifts=20, tol=1e-5, grad_tol=1e-6, precision=ldq.LDQ_FP64)
        ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], fp64)
        torch.cuda.synchronize()
        nf = max(2, args.steps // 3)
        t1 = time.perf_counter()
        for _ in range(nf):
            fv, fg, finfo = ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], fp64)
        torch.cuda.synchronize()
        fdt = (time.perf_counter() - t1) / nf
        out["rel_err_vs_fp64"] = {"logdet": abs(val - ref_val) / abs(ref_val),
                                  "grad": abs(grad[0] - ref_grad[0]) / abs(ref_grad[0])}
        out["forms"] = {
            "mixed": {"evals_per_s": round(value, 3), "ms": round(dt / args.steps * 1e3, 3),
                      "gbs": round(achieved, 1), "iters_max": last["iters_max"]},
            "fp64": {"evals_per_s": round(1.0 / fdt, 3), "ms": round(fdt * 1e3, 3),
                     "gbs": round(finfo["bytes_model"] / finfo["loop_seconds"] / 1e9, 1),
                     "iters_max": finfo["iters_max"],
                     "rel_err_vs_tight_fp64": {"logdet": abs(fv - ref_val) / abs(ref_val),
                                               "grad": abs(fg[0] - ref_grad[0]) / abs(ref_grad[0])}},
        }
        out["forms"].update(csr_forms(ctx, wl, nf, ref_val, ref_grad[0]))
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")    # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * a.numel() * 4

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, last["iters_total"])

    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
