#!/usr/bin/env python
"""Throughput of D = (R (x) K(x,y)) - I on one MI355X.

A step is one difference image of the 2048 x 4096 chip workload (21 x 21
kernel, 49 Gaussian bases, spatial degree 2): per-pixel coefficients, the
basis contraction on the matrix cores and the subtraction, inputs resident in
HBM.  Each arithmetic form (FP32 and the bf16/fp16 split forms) is timed with
HIP events on the stream the library launches on; the headline value is the
fastest matrix-core form whose error against the FP64 oracle (measured in the
CPU-baseline leg on sampled pixels) stays within 1e-2 sigma_sky.

Prints one JSON line (rank 0, N = 1).
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Mpix/s of D=(R⊗K(x,y))−I, FP32 vs MFMA form at ≤1e-2 "
          "σ_sky error; % roofline")
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "bf16x3": 2500.0,
               "fp16x2": 2500.0, "fp16x3": 2500.0}
PASSES = {"fp32": 1, "bf16": 1, "fp16": 1, "bf16x3": 3, "fp16x2": 2, "fp16x3": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_form(plan, args, R, I, a, D, precision, form):
    import torch
    from paper_1209_5823_amd._lib import SvconvError
    try:
        plan.set_precision(precision)
        plan.set_form(form)
        for _ in range(args.warmup):
            plan.difference(R, I, a, out=D)
    except SvconvError as e:
        log("  %s/%s: %s" % (form, precision, e))
        return None
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        plan.difference(R, I, a, out=D)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    return ms


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=["c1", "c3", "c4"])
    ap.add_argument("--precisions", default="fp32,bf16x3,fp16x3,fp16x2")
    ap.add_argument("--forms", default="basis,regrouped")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward + adjoint timing on the 4096 x 4096 workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (steps times), the "
                         "reference for scaling HBM byte counters")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration, "steps": args.steps}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the method shards into independent row slabs; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1209_5823_amd import svconv, flops

    wl = synth.WORKLOADS[args.workload]
    log("inputs: %s %dx%d" % (wl.name, wl.height, wl.width))
    R_h, a_h = synth.workload_inputs(wl)
    I_h = synth.second_image(wl)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    results = {}
    with torch.cuda.stream(stream):
        R = torch.from_numpy(R_h).cuda()
        I = torch.from_numpy(I_h).cuda()
        a = torch.from_numpy(a_h).cuda()
        D = torch.empty_like(R)
        plan = svconv.plan_for(wl, precision="fp32", pedestal=synth.SKY_LEVEL)
        outputs = {}
        for form in args.forms.split(","):
            for prec in args.precisions.split(","):
                ms = time_form(plan, args, R, I, a, D, prec, form)
                if ms is None:
                    continue
                torch.cuda.synchronize()
                outputs[(form, prec)] = D.cpu().numpy()
                mpix = wl.height * wl.width / (ms * 1e-3) / 1e6
                results[(form, prec)] = dict(ms=ms, mpix=mpix)
                log("  %-9s %-7s %8.3f ms  %10.1f Mpix/s" % (form, prec, ms, mpix))
        plan.close()

    # forward + adjoint (dL/dR and dL/da) on the differentiation workload:
    # 4096 x 4096, 31 x 31 kernel, 49 bases, spatial degree 3
    adjoint = None
    if not args.no_adjoint:
        wl3 = synth.WORKLOADS["c3"]
        log("inputs: %s %dx%d (adjoint)" % (wl3.name, wl3.height, wl3.width))
        R3, a3 = synth.workload_inputs(wl3)
        I3 = synth.second_image(wl3)
        G3 = synth.uniform_image(wl3.height, wl3.width, seed=3, lo=-60.0, hi=60.0)
        with torch.cuda.stream(stream):
            R3d, I3d, a3d, G3d = (torch.from_numpy(x).cuda() for x in (R3, I3, a3, G3))
            D3 = torch.empty_like(R3d)
            plan3 = svconv.plan_for(wl3, precision="fp32", pedestal=synth.SKY_LEVEL)

            def timed(fn, n):
                for _ in range(args.warmup):
                    fn()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(n):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / n

            n3 = max(2, args.steps // 4)
            adjoint = {"workload": wl3.description}
            for prec in ("fp32", "bf16x3"):
                plan3.set_precision(prec)
                adjoint["forward_%s_ms" % prec] = round(
                    timed(lambda: plan3.difference(R3d, I3d, a3d, out=D3), n3), 4)
            adjoint["backward_ms"] = round(timed(lambda: plan3.backward(R3d, a3d, G3d), n3), 4)
            adjoint["backward_dR_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_ga=False), n3), 4)
            adjoint["backward_da_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_gR=False), n3), 4)
            px3 = wl3.height * wl3.width
            adjoint["forward_backward_mpix"] = round(
                px3 / ((adjoint["forward_bf16x3_ms"] + adjoint["backward_ms"]) * 1e-3) / 1e6, 2)
            plan3.close()
        log("  adjoint: %s" % adjoint)

    # CPU baseline: the FP64 oracle on a bounded random sample of pixels; its
    # values also give the error of every form on that sample.
    cpu = None
    if not args.no_cpu:
        from oracle import oracle
        B = oracle.basis(wl.half_width, wl.sigmas, wl.degrees)
        rng = np.random.default_rng(1234)
        n0 = 20000
        for _ in range(2):   # the first round also starts the OpenMP pool
            xs = rng.integers(0, wl.width, n0).astype(np.int32)
            ys = rng.integers(0, wl.height, n0).astype(np.int32)
            t0 = time.perf_counter()
            oracle.convolve_at(R_h, wl.half_width, B, wl.spatial_degree, a_h, xs, ys)
            dt0 = time.perf_counter() - t0
        n = int(min(wl.height * wl.width, max(n0, n0 * args.cpu_seconds / max(dt0, 1e-6))))
        xs = rng.integers(0, wl.width, n).astype(np.int32)
        ys = rng.integers(0, wl.height, n).astype(np.int32)
        flat = np.argsort(R_h.ravel())[-256:]
        xs = np.concatenate([xs, (flat % wl.width).astype(np.int32)])
        ys = np.concatenate([ys, (flat // wl.width).astype(np.int32)])
        log("cpu baseline: oracle on %d sampled pixels" % len(xs))
        t0 = time.perf_counter()
        C = oracle.convolve_at(R_h, wl.half_width, B, wl.spatial_degree, a_h, xs, ys)
        dt = time.perf_counter() - t0
        Dref = C - I_h[ys, xs].astype(np.float64)
        sig = synth.sky_sigma()
        for key, Dg in outputs.items():
            d = np.abs(Dg[ys, xs].astype(np.float64) - Dref) / sig
            results[key]["max_err_sigma"] = float(d.max())
            results[key]["rms_err_sigma"] = float(np.sqrt(np.mean(d * d)))
        cpu = {"value": len(xs) / dt / 1e6, "unit": "Mpix/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": "%d random pixels + 256 brightest of the %dx%d frame, per-pixel "
                         "kernel and direct convolution in float64 (%.1f s)"
                         % (len(xs) - 256, wl.height, wl.width, dt)}

    # headline: the basis form (per-pixel coefficients, N basis responses) in
    # its fastest matrix-core precision within 1e-2 sigma_sky; the FP32 basis
    # form and the regrouped form are reported beside it
    def ok(r, tol):
        return ("max_err_sigma" not in r) or r["max_err_sigma"] <= tol

    def best(form, want_fp32, tol):
        c = [(r["mpix"], k) for k, r in results.items()
             if k[0] == form and (k[1] == "fp32") == want_fp32 and ok(r, tol)]
        return max(c)[1] if c else None

    head = best("basis", False, 1e-2) or best("basis", True, 1e-4)
    if head is None:
        print("no valid form was measured", file=sys.stderr)
        sys.exit(1)
    hr = results[head]
    form, prec = head
    N, M, k = wl.n_basis, wl.n_spatial, wl.k
    px = wl.height * wl.width

    def roof(key):
        r = results[key]
        per_px = (flops.flops_per_pixel(N, M, k) if key[0] == "basis"
                  else flops.regrouped_flops_per_pixel(M, k))
        ach = per_px * px / (r["ms"] * 1e-3) / 1e12
        return per_px, ach

    per_px, achieved = roof(head)
    peak = PEAK_TFLOPS[prec]
    traffic = recorded_traffic(prec, form)
    out = {
        "metric": METRIC,
        "value": round(hr["mpix"], 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": wl.description, "height": wl.height, "width": wl.width,
                   "kernel": k, "n_basis": N, "n_spatial": M, "form": form, "precision": prec,
                   "pedestal": synth.SKY_LEVEL},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                     "flop_per_pixel": per_px, "pixels_per_launch": px},
        "cpu_baseline": cpu,
    }
    fp = best("basis", True, 1e-4)
    if fp is not None:
        pp, ach = roof(fp)
        out["fp32"] = {"mpix": round(results[fp]["mpix"], 2), "ms": round(results[fp]["ms"], 4),
                       "achieved_tflops": round(ach, 3), "peak_tflops": PEAK_TFLOPS["fp32"],
                       "frac": round(ach / PEAK_TFLOPS["fp32"], 4),
                       "max_err_sigma": results[fp].get("max_err_sigma")}
    rg = best("regrouped", False, 1e-2)
    if rg is not None:
        pp, ach = roof(rg)
        out["regrouped"] = {"precision": rg[1], "mpix": round(results[rg]["mpix"], 2),
                            "ms": round(results[rg]["ms"], 4), "flop_per_pixel": pp,
                            "achieved_tflops": round(ach, 3),
                            "max_err_sigma": results[rg].get("max_err_sigma")}
    if adjoint is not None:
        out["adjoint"] = adjoint
    out["forms"] = {"%s/%s" % k_: {kk: (round(v, 6) if isinstance(v, float) else v)
                                   for kk, v in r.items()} for k_, r in results.items()}
    print(json.dumps(out), flush=True)


def recorded_traffic(precision, form):
    """HBM bytes per launch of the contraction kernel from the committed
    rocprofv3 counter summary, or None if the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get("%s/%s" % (form, precision))
    if not ent:
        return None
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return ent.get("traffic_bytes")


if __name__ == "__main__":
    main()
