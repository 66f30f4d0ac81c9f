#!/usr/bin/env python
"""Throughput of D = (R (x) K(x,y)) - I on one MI355X.

A step is one difference image of the 2048 x 4096 chip workload (21 x 21
kernel, 49 Gaussian bases, spatial degree 2): per-pixel coefficients, the
basis contraction and the subtraction, inputs resident in HBM.  Each form is
timed with HIP events on the stream the library launches on: the basis and
regrouped forms on the matrix cores (FP32 and the bf16/fp16 split
precisions), the separable form (row and column passes of the Gaussian
factors, float64 on the vector units or Toeplitz products on the matrix
cores) and the regrouped separable form (the coefficients folded into
per-call column filters, all passes on the matrix cores).  The headline value is the fastest
form whose error against the FP64 oracle (measured in the CPU-baseline leg on
sampled pixels) stays within 1e-2 sigma_sky; the fastest form within the FP32
path's 1e-4 sigma and the fastest matrix-core form are reported beside it.

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
               "fp16x2": 2500.0, "fp16x3": 2500.0, "f64": 78.6}
PASSES = {"fp32": 1, "bf16": 1, "fp16": 1, "bf16x3": 3, "fp16x2": 2, "fp16x3": 3}
SEP_MMA_PRECISIONS = ("fp16x3", "bf16x3", "fp16x2")


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
    # the timed steps: one event on each side, none between the steps (an event
    # between two launches adds its own few microseconds to every step)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        plan.difference(R, I, a, out=D)
    t1.record()
    torch.cuda.synchronize()
    mean = t0.elapsed_time(t1) / args.steps
    # then the spread over as many steps again, each bracketed by events
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        plan.difference(R, I, a, out=D)
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps))
    time_form.last = {"median_ms": per[len(per) // 2], "min_ms": per[0]}
    return mean


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=["c1", "c3", "c4"])
    ap.add_argument("--precisions", default="fp32,bf16x3,fp16x3,fp16x2")
    ap.add_argument("--forms", default="basis,regrouped,separable,separable_regrouped")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward + adjoint timing on the 4096 x 4096 workload")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the size sweep of the chip workload's kernel and basis")
    ap.add_argument("--no-dfb", action="store_true",
                    help="skip the Dirac delta basis size sweep")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the streamed host-tile pipeline measurement")
    ap.add_argument("--dfb-only", action="store_true",
                    help="only time the Dirac delta basis forms on the 4846 x 4868 tile and "
                         "print that sweep (for profiling the paper's own case)")
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
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method shards into independent row slabs of the image)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1209_5823_amd import svconv, flops

    if args.dfb_only:
        torch.cuda.set_device(0)
        print(json.dumps({"dfb": dfb_sweep(args, torch.cuda.Stream(), sizes=DFB_SIZES[-1:])}), flush=True)
        return

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
            # the separable form: float64 vector passes ("f64", set through the
            # fp32 precision) and, for the split 16-bit precisions, matrix-core passes
            precs = args.precisions.split(",")
            if form == "separable":
                precs = ["f64"] + [p_ for p_ in precs if p_ in SEP_MMA_PRECISIONS]
            elif form == "separable_regrouped":
                precs = [p_ for p_ in precs if p_ in SEP_MMA_PRECISIONS]
            for prec in precs:
                ms = time_form(plan, args, R, I, a, D, "fp32" if prec == "f64" else prec, form)
                if ms is None:
                    continue
                torch.cuda.synchronize()
                outputs[(form, prec)] = D.cpu().numpy()
                mpix = wl.height * wl.width / (ms * 1e-3) / 1e6
                results[(form, prec)] = dict(ms=ms, mpix=mpix, **time_form.last)
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
            plan3.set_form("separable")
            plan3.set_precision("fp16x3")
            adjoint["forward_separable_fp16x3_ms"] = round(
                timed(lambda: plan3.difference(R3d, I3d, a3d, out=D3), n3), 4)
            plan3.set_precision("fp32")
            adjoint["forward_separable_ms"] = round(
                timed(lambda: plan3.difference(R3d, I3d, a3d, out=D3), n3), 4)
            adjoint["backward_da_separable_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_gR=False), n3), 4)
            adjoint["backward_dR_separable_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_ga=False), n3), 4)
            # the split precisions take both adjoints on the matrix cores
            plan3.set_precision("fp16x3")
            adjoint["backward_dR_separable_mma_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_ga=False), n3), 4)
            adjoint["backward_da_separable_mma_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_gR=False), n3), 4)
            plan3.set_form("basis")
            plan3.set_precision("fp32")
            adjoint["backward_ms"] = round(timed(lambda: plan3.backward(R3d, a3d, G3d), n3), 4)
            adjoint["backward_dR_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_ga=False), n3), 4)
            adjoint["backward_da_ms"] = round(
                timed(lambda: plan3.backward(R3d, a3d, G3d, want_gR=False), n3), 4)
            px3 = wl3.height * wl3.width
            best_da = min(adjoint["backward_da_ms"], adjoint["backward_da_separable_ms"],
                          adjoint["backward_da_separable_mma_ms"])
            best_dr = min(adjoint["backward_dR_ms"], adjoint["backward_dR_separable_ms"],
                          adjoint["backward_dR_separable_mma_ms"])
            best_fw = min(adjoint["forward_separable_ms"], adjoint["forward_separable_fp16x3_ms"])
            adjoint["forward_backward_mpix"] = round(px3 / ((best_fw + best_dr + best_da) * 1e-3) / 1e6, 2)
            plan3.close()
        log("  adjoint: %s" % adjoint)

    dfb = None if args.no_dfb else dfb_sweep(args, stream)
    sweep = None if args.no_sweep else gauss_sweep(args, stream, wl)
    pipeline = None if args.no_pipeline else pipeline_bench(args)

    # CPU baseline: the FP64 oracle on a bounded random sample of pixels; its
    # values also give the error of every form on that sample.
    cpu = cpu1 = None
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
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": "%d random pixels + 256 brightest of the %dx%d frame, per-pixel "
                         "kernel and direct convolution in float64 (%.1f s)"
                         % (len(xs) - 256, wl.height, wl.width, dt)}
        # one thread: the analogue of the paper's single-thread ANSI-C baseline
        n1 = max(2000, len(xs) // (4 * max(1, oracle.max_threads())))
        t0 = time.perf_counter()
        oracle.convolve_at(R_h, wl.half_width, B, wl.spatial_degree, a_h, xs[:n1], ys[:n1], nthreads=1)
        dt1 = time.perf_counter() - t0
        cpu1 = {"value": n1 / dt1 / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
                "sample": "%d of the same pixels, one thread (%.1f s)" % (n1, dt1)}
        log("cpu baseline: %.2f Mpix/s on %d threads, %.3f Mpix/s on one"
            % (cpu["value"], cpu["cores"], cpu1["value"]))

    # headline: the fastest form within 1e-2 sigma_sky (every form computes D
    # of Eq. 1 exactly up to rounding); the fastest form within the FP32
    # path's 1e-4 sigma, the fastest matrix-core form and the dense FP32
    # matrix-core basis form are reported beside it
    # without the oracle's sampled errors (--no-cpu) a form qualifies by the
    # bound its parity tests hold: 1e-4 sigma for the float32 / float64 paths,
    # 1e-2 sigma for those and the fp16x3 / bf16x3 splits
    def ok(key, r, tol):
        if "max_err_sigma" in r:
            return r["max_err_sigma"] <= tol
        return key[1] in (("fp32", "f64") if tol <= 1e-4 else ("fp32", "f64", "fp16x3", "bf16x3"))

    def best(tol, forms=None, precs=None):
        c = [(r["mpix"], k) for k, r in results.items()
             if ok(k, r, tol) and (forms is None or k[0] in forms) and (precs is None or k[1] in precs)]
        return max(c)[1] if c else None

    head = best(1e-2)
    if head is None:
        print("no valid form was measured", file=sys.stderr)
        sys.exit(1)
    hr = results[head]
    form, prec = head
    N, M, k = wl.n_basis, wl.n_spatial, wl.k
    px = wl.height * wl.width

    def roof(key):
        r = results[key]
        if key[0] == "basis":
            per_px = flops.flops_per_pixel(N, M, k)
        elif key[0] == "regrouped":
            per_px = flops.regrouped_flops_per_pixel(M, k)
        elif key[1] == "f64":
            per_px = flops.separable_flops_per_pixel(wl.degrees, M, k)
        else:
            # the matrix-core separable forms: the tap-by-tap separable count
            # (row pass per factor, column pass per basis), the least work
            # any of the separable forms does
            per_px = flops.separable_unfolded_flops_per_pixel(wl.degrees, M, k)
        ach = per_px * px / (r["ms"] * 1e-3) / 1e12
        return per_px, ach

    def bound_of(key):
        return "alu" if key == ("separable", "f64") else "mfma"

    def summary(key):
        pp, ach = roof(key)
        peak = PEAK_TFLOPS[key[1]]
        return {"form": key[0], "precision": key[1], "mpix": round(results[key]["mpix"], 2),
                "ms": round(results[key]["ms"], 4), "flop_per_pixel": pp,
                "achieved_tflops": round(ach, 3), "peak_tflops": peak,
                "bound": bound_of(key),
                "frac": round(ach / peak, 4),
                "max_err_sigma": results[key].get("max_err_sigma")}

    def executed(key):
        """Matrix-core FLOP per pixel the form's kernels issue (None off the matrix cores)."""
        if key[1] == "f64" or key[0] not in ("separable", "separable_regrouped"):
            return None
        if key[0] == "separable":
            return flops.separable_mma_executed_flops_per_pixel(wl.degrees, PASSES[key[1]])
        return flops.separable_regrouped_executed_flops_per_pixel(wl.degrees, M, PASSES[key[1]])

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
        "roofline": {"bound": bound_of(head),
                     "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                     "flop_per_pixel": per_px, "pixels_per_launch": px,
                     "traffic_gbs": (round(traffic / (hr["ms"] * 1e-3) / 1e9, 1)
                                     if traffic else None),
                     "hbm_peak_gbs": 8000.0,
                     "form_flop_per_pixel": (flops.separable_regrouped_flops_per_pixel(wl.degrees, M, k)
                                             if form == "separable_regrouped" else per_px),
                     "mfma_executed_flop_per_pixel": executed(head),
                     "mfma_executed_frac": (round(executed(head) * px / (hr["ms"] * 1e-3) / 1e12 / peak, 4)
                                            if executed(head) else None)},
        "paper_model": {"flop_per_pixel": flops.paper_flops_gfb(N, k),
                        "note": "the paper's Gaussian-basis cost model (Sec. 3): every basis a full "
                                "k x k convolution; a dense-equivalent rate, not executed work",
                        "tflops_equivalent": round(flops.paper_flops_gfb(N, k) * px / (hr["ms"] * 1e-3) / 1e12, 3)},
        "cpu_baseline": cpu,
        "timing": {"mean_ms": round(hr["ms"], 4), "median_ms": round(hr["median_ms"], 4),
                   "min_ms": round(hr["min_ms"], 4)},
    }
    if cpu is not None:
        out["cpu_single_core"] = cpu1
        out["speedup"] = {"vs_oracle_all_threads": round(hr["mpix"] / cpu["value"], 1),
                          "vs_oracle_one_thread": round(hr["mpix"] / cpu1["value"], 1),
                          "paper": "about 50x over single-thread ANSI-C (GTX465 against "
                                   "Athlon II X3, delta basis; context only)"}
    fp = best(1e-4)
    if fp is not None:
        # the fastest form within the FP32 path's 1e-4 sigma; "precision" names
        # its arithmetic (f64: float64 FMAs on the vector units)
        out["fp32_path"] = summary(fp)
        out["fp32_path"]["tolerance_sigma"] = 1e-4
    mf = best(1e-2, forms=("basis", "regrouped", "separable", "separable_regrouped"),
              precs=("bf16", "fp16", "bf16x3", "fp16x2", "fp16x3"))
    if mf is not None:
        out["mfma"] = summary(mf)
    if ("basis", "fp32") in results:
        out["fp32"] = summary(("basis", "fp32"))
    if ("separable", "f64") in results:
        # the float64 separable form on the vector units, with its own (ALU) roofline
        out["separable_f64"] = summary(("separable", "f64"))
    rg = best(1e-2, forms=("regrouped",))
    if rg is not None:
        out["regrouped"] = summary(rg)
    if adjoint is not None:
        out["adjoint"] = adjoint
    if sweep is not None:
        out["size_sweep"] = sweep
    if dfb is not None:
        out["dfb"] = dfb
    if pipeline is not None:
        out["pipeline"] = pipeline
    out["forms"] = {"%s/%s" % k_: {kk: (round(v, 6) if isinstance(v, float) else v)
                                   for kk, v in r.items()} for k_, r in results.items()}
    print(json.dumps(out), flush=True)


SWEEP_FORMS = (("separable", "fp32"), ("separable", "fp16x3"), ("separable_regrouped", "fp16x3"),
               ("basis", "fp16x3"), ("regrouped", "fp16x3"))


def gauss_sweep(args, stream, wl):
    """Mpix/s against image size with the chip workload's kernel and basis
    (21 x 21, 49 Gaussian bases, spatial degree 2), sizes from 256 x 256 to
    one 4846 x 4868 camera tile (the x-axis of the paper's size study,
    Sec. 5): top-left crops of one tile-sized star field with the chip's star
    density and FWHM ramp."""
    import numpy as np
    import torch

    import synth
    from paper_1209_5823_amd import svconv

    Ht, Wt = DFB_SIZES[-1]
    n_stars = int(round(wl.n_stars * Ht * Wt / (wl.height * wl.width)))
    log("inputs: size sweep %dx%d, %d stars" % (Ht, Wt, n_stars))
    tile = synth.star_field(Ht, Wt, n_stars, wl.fwhm, seed=12)
    _, a_h = synth.workload_inputs(wl)
    rows = []
    with torch.cuda.stream(stream):
        a = torch.from_numpy(a_h).cuda()
        for (H, W) in DFB_SIZES:
            R = torch.from_numpy(np.ascontiguousarray(tile[:H, :W])).cuda()
            I = R.clone()
            D = torch.empty_like(R)
            row = {"height": H, "width": W}
            with svconv.Plan(H, W, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                             pedestal=synth.SKY_LEVEL) as plan:
                for form, prec in SWEEP_FORMS:
                    ms = time_form(plan, args, R, I, a, D, prec, form)
                    if ms is None:
                        continue
                    label = "%s/%s" % (form, "f64" if (form, prec) == ("separable", "fp32") else prec)
                    row[label] = {"ms": round(ms, 4), "mpix": round(H * W / (ms * 1e-3) / 1e6, 1)}
            log("  sweep %5dx%-5d %s" % (H, W, "  ".join("%s %.0f" % (k, v["mpix"]) for k, v in row.items()
                                                      if isinstance(v, dict))))
            rows.append(row)
    return {"kernel": wl.k, "n_basis": wl.n_basis, "spatial_degree": wl.spatial_degree, "sizes": rows}


DFB_SIZES = ((256, 256), (512, 512), (1024, 1024), (2048, 2048), (4096, 4096), (4846, 4868))
DFB_FORMS = (("regrouped", "fp32"), ("regrouped", "bf16x3"), ("regrouped", "fp16x3"),
             ("basis", "fp16x3"))


def dfb_sweep(args, stream, sizes=DFB_SIZES):
    """The paper's own benchmark case (Sec. 3): 7 x 7 Dirac delta basis
    (49 bases, one per kernel pixel), second-order spatial polynomial, image
    sizes from 256 x 256 up to one 4846 x 4868 camera tile.  Smaller sizes are
    top-left crops of the tile.  Reports, per size, each form's time and
    Mpix/s, the rate in the paper's DFB FLOP model (20 L^2 + 1 per pixel) and
    the error of each form on sampled pixels of the full tile."""
    import numpy as np
    import torch

    import synth
    from oracle import oracle
    from paper_1209_5823_amd import svconv, flops

    h, d_s = 3, 2
    k = 2 * h + 1
    Ht, Wt = DFB_SIZES[-1]
    log("inputs: dfb %dx%d tile, %dx%d kernel" % (Ht, Wt, k, k))
    tile = synth.star_field(Ht, Wt, 20000, seed=11)
    a_h = synth.coefficients(k * k, synth.n_spatial(d_s), (k * k) // 2, seed=11)
    sweep = []
    errs = {}
    with torch.cuda.stream(stream):
        a = torch.from_numpy(a_h).cuda()
        for (H, W) in sizes:
            R = torch.from_numpy(np.ascontiguousarray(tile[:H, :W])).cuda()
            I = R.clone()
            D = torch.empty_like(R)
            row = {"height": H, "width": W}
            best = None
            with svconv.Plan.dfb(H, W, h, d_s, pedestal=synth.SKY_LEVEL) as plan:
                for form, prec in DFB_FORMS:
                    ms = time_form(plan, args, R, I, a, D, prec, form)
                    if ms is None:
                        continue
                    mpix = H * W / (ms * 1e-3) / 1e6
                    row["%s/%s" % (form, prec)] = {"ms": round(ms, 4), "mpix": round(mpix, 1)}
                    if best is None or mpix > best[0]:
                        best = (mpix, form, prec)
                    if (H, W) == (Ht, Wt):
                        torch.cuda.synchronize()
                        errs[(form, prec)] = D.cpu().numpy()
            row["best"] = "%s/%s" % best[1:]
            row["best_mpix"] = round(best[0], 1)
            row["paper_model_gflops"] = round(flops.paper_flops_dfb(k) * best[0] * 1e6 / 1e9, 1)
            log("  dfb %5dx%-5d best %-16s %9.1f Mpix/s" % (H, W, row["best"], best[0]))
            sweep.append(row)
    # error of every form on 4000 random pixels + the 64 brightest of the tile
    rng = np.random.default_rng(99)
    xs = rng.integers(0, Wt, 4000).astype(np.int32)
    ys = rng.integers(0, Ht, 4000).astype(np.int32)
    flat = np.argsort(tile.ravel())[-64:]
    xs = np.concatenate([xs, (flat % Wt).astype(np.int32)])
    ys = np.concatenate([ys, (flat // Wt).astype(np.int32)])
    ref = oracle.convolve_at(tile, h, oracle.basis_dfb(h), d_s, a_h, xs, ys) - tile[ys, xs]
    sig = synth.sky_sigma()
    err = {"%s/%s" % key: round(float(np.max(np.abs(Dg[ys, xs] - ref)) / sig), 6)
           for key, Dg in errs.items()}
    return {"kernel": k, "n_basis": k * k, "spatial_degree": d_s,
            "paper_flop_per_pixel": flops.paper_flops_dfb(k),
            "max_err_sigma_tile": err, "sizes": sweep}


def pipeline_bench(args):
    """End-to-end rate with the images in host memory (Sec. 3: a 60-tile
    mosaic camera of 4846 x 4868 tiles; Sec. 4: asynchronous copies between
    page-locked host memory and the device).  Each tile's R and I are copied
    in and D copied back while other tiles are differenced.  The mosaic cycles
    through 4 distinct page-locked tiles.  Reported beside the HBM-resident
    headline, never instead of it: the host link, not the kernel, bounds it."""
    import numpy as np

    import synth
    from paper_1209_5823_amd import svconv

    H, W, n_tiles, n_distinct = 4846, 4868, 60, 4
    res = {"tiles": n_tiles, "tile": [H, W], "distinct_tiles": n_distinct, "depth": 3}
    host = []
    for t in range(n_distinct):
        R = svconv.pinned_empty((H, W))
        R.numpy()[:] = synth.star_field(H, W, 20000, seed=200 + t)
        I = svconv.pinned_empty((H, W))
        I.numpy()[:] = R.numpy()
        host.append((R, I, svconv.pinned_empty((H, W))))
    cases = [("dfb7_regrouped_fp16x3", dict(half_width=3, sigmas=None, degrees=None,
                                            spatial_degree=2, precision="fp16x3",
                                            form="regrouped")),
             ("gauss21_separable", dict(half_width=10, sigmas=(0.7, 1.5, 2.0),
                                        degrees=(6, 4, 2), spatial_degree=2,
                                        precision="fp32", form="separable"))]
    for name, kw in cases:
        with svconv.Plan(H, W, pedestal=synth.SKY_LEVEL, **kw) as plan:
            a = synth.coefficients(plan.n_basis, plan.n_spatial, 0, seed=5)
            Rs = [host[t % n_distinct][0] for t in range(n_tiles)]
            Is = [host[t % n_distinct][1] for t in range(n_tiles)]
            Ds = [host[t % n_distinct][2] for t in range(n_tiles)]
            As = [a] * n_tiles
            with svconv.Pipeline(plan, depth=res["depth"]) as pipe:
                pipe.run(Rs[:n_distinct], Is[:n_distinct], As[:n_distinct], Ds[:n_distinct])
                t0 = time.perf_counter()
                pipe.run(Rs, Is, As, Ds)
                dt = time.perf_counter() - t0
        mpix = n_tiles * H * W / dt / 1e6
        gbs = n_tiles * 3 * H * W * 4 / dt / 1e9
        res[name] = {"s": round(dt, 4), "mpix": round(mpix, 1), "host_link_gbs": round(gbs, 2)}
        log("  pipeline %-24s %8.1f Mpix/s  %6.2f GB/s over the host link" % (name, mpix, gbs))
    return res


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def recorded_traffic(precision, form):
    """HBM bytes per launch of the form's dominant kernel from the committed
    rocprofv3 counter summary, or None if the kernel's sources changed since."""
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
    for src in ent.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != ent.get("sources_sha256"):
        return None
    return ent.get("traffic_bytes")


if __name__ == "__main__":
    main()
