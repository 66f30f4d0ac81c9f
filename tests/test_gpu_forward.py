"""GPU parity of the forward path (D = (R (x) K(x,y)) - I, Eq. 1 - Eq. 3)
against the FP64 oracle, through the C ABI.

Tolerances (from the workload definition): max |dD| <= 1e-4 sigma_sky for
the FP32 path and <= 1e-2 sigma_sky for the bf16/fp16 matrix-core forms,
sigma_sky = sqrt(1000) ADU.  Full-size frames are compared on sampled pixels
(random pixels, every edge band, the brightest stars) that the oracle
evaluates one by one.
"""

import numpy as np
import pytest

import synth
from tests.helpers import (TOL_FP32, TOL_MFMA, say, to_dev, to_host, err_stats, sample_pixels,
                           workload_images)

pytestmark = pytest.mark.gpu

C0 = synth.WORKLOADS["c0"]
C1 = synth.WORKLOADS["c1"]
C3 = synth.WORKLOADS["c3"]
C4 = synth.WORKLOADS["c4"]


def run_difference(svc, R, I, a, h, sigmas, degrees, d_s, precision="fp32", form="basis",
                   frame=None, pedestal=0.0):
    H, W = R.shape
    with svc.Plan(H, W, h, sigmas, degrees, d_s, precision=precision, form=form, frame=frame,
                  pedestal=pedestal) as plan:
        D = plan.difference(to_dev(R), to_dev(I), to_dev(a))
        return to_host(D)


@pytest.fixture(scope="module")
def c0_case(orc):
    R, a = synth.workload_inputs(C0)
    B = orc.basis(C0.half_width, C0.sigmas, C0.degrees)
    C = orc.convolve(R, C0.half_width, B, C0.spatial_degree, a)
    I = (C + 10.0).astype(np.float32)
    D = C - I.astype(np.float64)
    return R, I, a, D


@pytest.mark.parametrize("form", ["basis", "regrouped"])
@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_c0_full_frame_fp32(svc, c0_case, form, pedestal):
    R, I, a, Dref = c0_case
    say("c0 full frame fp32", form, pedestal)
    D = run_difference(svc, R, I, a, C0.half_width, C0.sigmas, C0.degrees, C0.spatial_degree,
                       form=form, pedestal=pedestal)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e (tol %.3e)" % (mx, rms, TOL_FP32))
    assert mx <= TOL_FP32
    # D is the constant -10 where I = R (x) K + 10 (up to I's float32 rounding)
    assert np.max(np.abs(D + 10.0)) <= TOL_FP32 + np.max(np.abs(Dref + 10.0))


def test_basis_table_matches_oracle(svc, orc):
    with svc.Plan(64, 64, C1.half_width, C1.sigmas, C1.degrees, 2) as plan:
        B = plan.basis().numpy()
    Bo = orc.basis(C1.half_width, C1.sigmas, C1.degrees)
    assert np.max(np.abs(B - Bo)) <= 4 * np.finfo(np.float64).eps * np.max(np.abs(Bo))


EDGE_CASES = {
    # name: (H, W, h, sigmas, degrees, d_s, frame)
    "one_pixel": (1, 1, 0, (1.5,), (0,), 0, None),
    "kernel_larger_than_image": (5, 7, 10, C1.sigmas, C1.degrees, 2, None),
    "all_border_8x8": (8, 8, 4, (0.7, 1.5), (2, 1), 2, None),
    "h1_ragged": (37, 70, 1, (1.0,), (2,), 1, None),
    "nb3_degree3": (64, 96, 7, (0.7, 1.5, 2.0), (6, 2, 0), 3, None),
    "c1_kernel_ragged_crop": (200, 301, 10, C1.sigmas, C1.degrees, 2, (1000, 500, 4096, 2048)),
    "c3_kernel_degree4": (90, 133, 15, C3.sigmas, C3.degrees, 4, (17, 2000, 4096, 4096)),
    "max_filters_64": (48, 80, 6, (0.7, 1.2, 1.5, 2.0, 2.5), (6, 6, 2, 0, 0), 2, None),
    "max_spatial_degree_6": (50, 66, 5, (1.5,), (2,), 6, None),
    "max_half_width_31": (70, 90, 31, (2.0, 4.0), (2, 0), 1, None),
    "single_row": (1, 257, 3, (1.5,), (1,), 2, None),
    "single_column": (190, 1, 3, (1.5,), (1,), 2, None),
}


def _edge_inputs(name, case):
    H, W, h, sig, deg, d_s, frame = case
    seed = sum(map(ord, name))
    R = synth.star_field(H, W, max(1, H * W // 400), seed=seed)
    I = synth.star_field(H, W, max(1, H * W // 400), seed=seed + 1)
    N = synth.n_basis(deg)
    a = synth.coefficients(N, synth.n_spatial(d_s), 0, seed=seed)
    return R, I, a


@pytest.mark.parametrize("form", ["basis", "regrouped"])
@pytest.mark.parametrize("name", list(EDGE_CASES))
def test_edge_cases_fp32(svc, orc, name, form):
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("edge", name, form, (H, W, h, len(B), d_s))
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, form=form, frame=frame)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_FP32


def test_delta_kernel_identity(svc):
    # sigma = 0 basis with coefficient 1: D = R - I exactly (rounded once)
    R = synth.star_field(100, 130, 30, seed=11)
    I = synth.star_field(100, 130, 30, seed=12)
    a = np.zeros((1, 6), np.float32)
    a[0, 0] = 1.0
    say("delta identity")
    D = run_difference(svc, R, I, a, 4, (0.0,), (0,), 2)
    assert np.array_equal(D, (R.astype(np.float64) - I).astype(np.float32))


@pytest.mark.parametrize("form", ["basis", "regrouped"])
@pytest.mark.parametrize("wl_name", ["c1", "c3", "c4"])
def test_full_size_sampled_fp32(svc, orc, wl_name, form):
    wl = synth.WORKLOADS[wl_name]
    R, a, I = workload_images(wl_name)
    say("full size sampled", wl_name, form, R.shape)
    D = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       form=form)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    xs, ys = sample_pixels(wl.height, wl.width, 1500, seed=3, R=R, h=wl.half_width)
    Dref = orc.convolve_at(R, wl.half_width, B, wl.spatial_degree, a, xs, ys) - I[ys, xs]
    mx, rms = err_stats(D[ys, xs], Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_FP32
    assert np.all(np.isfinite(D))


# ------------------------------------------------ bf16 / fp16 matrix cores ----

# the split precisions that meet the matrix-core bound of 1e-2 sigma_sky
LOWP = ["bf16x3", "fp16x3"]


def c2_crops(orc):
    """The 512 x 512 crops of the 2048 x 4096 chip at its centre and at its
    brightest star, with the oracle's D on each (frame coordinates of the chip)."""
    wl = synth.WORKLOADS["c2"]
    R, a = synth.workload_inputs(wl)
    I = synth.second_image(wl)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    yb, xb = np.unravel_index(np.argmax(R), R.shape)
    out = []
    for (y0, x0) in [(768, 1792), (int(np.clip(yb - 256, 0, wl.height - 512)),
                                   int(np.clip(xb - 256, 0, wl.width - 512)))]:
        Rc = np.ascontiguousarray(R[y0:y0 + 512, x0:x0 + 512])
        Ic = np.ascontiguousarray(I[y0:y0 + 512, x0:x0 + 512])
        frame = (x0, y0, wl.width, wl.height)
        out.append((Rc, Ic, a, frame, orc.difference(Rc, Ic, wl.half_width, B, wl.spatial_degree, a,
                                                     frame=frame)))
    return wl, out


@pytest.mark.parametrize("precision", LOWP)
def test_c2_crops_lowp(svc, orc, precision):
    # 512 x 512 crops of the 2048 x 4096 chip (centre and brightest star),
    # frame coordinates of the chip, pedestal at the sky level
    wl, crops = c2_crops(orc)
    for Rc, Ic, a, frame, Dref in crops:
        say("c2 crop", precision, frame)
        D = run_difference(svc, Rc, Ic, a, wl.half_width, wl.sigmas, wl.degrees,
                           wl.spatial_degree, precision=precision, frame=frame,
                           pedestal=synth.SKY_LEVEL)
        mx, rms = err_stats(D, Dref)
        say("  max %.3e rms %.3e (%.2e sigma)" % (mx, rms, mx / np.sqrt(1000)))
        assert mx <= TOL_MFMA


@pytest.mark.parametrize("form", ["basis", "regrouped"])
@pytest.mark.parametrize("precision", LOWP)
@pytest.mark.parametrize("name", ["one_pixel", "kernel_larger_than_image", "all_border_8x8",
                                  "h1_ragged", "nb3_degree3", "c1_kernel_ragged_crop",
                                  "c3_kernel_degree4", "max_filters_64", "single_column"])
def test_edge_cases_lowp(svc, orc, name, precision, form):
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("edge lowp", name, precision, form)
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, precision=precision, form=form,
                       frame=frame, pedestal=synth.SKY_LEVEL)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_MFMA


@pytest.mark.parametrize("precision", LOWP)
def test_c0_full_frame_lowp(svc, c0_case, precision):
    R, I, a, Dref = c0_case
    say("c0 full frame", precision)
    D = run_difference(svc, R, I, a, C0.half_width, C0.sigmas, C0.degrees, C0.spatial_degree,
                       precision=precision, pedestal=synth.SKY_LEVEL)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_MFMA


def test_lowp_rejects_half_width_above_15(svc):
    import torch
    from paper_1209_5823_amd._lib import SvconvError, EUNSUPPORTED
    with svc.Plan(64, 64, 16, (2.0,), (0,), 1, precision="bf16x3") as plan:
        R = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
        a = torch.ones((1, 3), dtype=torch.float32, device="cuda")
        with pytest.raises(SvconvError) as ei:
            plan.forward(R, a)
        assert ei.value.status == EUNSUPPORTED


@pytest.mark.parametrize("form", ["basis", "regrouped"])
@pytest.mark.parametrize("precision", LOWP)
def test_full_size_sampled_lowp(svc, orc, precision, form):
    wl = synth.WORKLOADS["c1"]
    R, a, I = workload_images("c1")
    say("full size sampled", precision, form)
    D = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       precision=precision, form=form, pedestal=synth.SKY_LEVEL)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    xs, ys = sample_pixels(wl.height, wl.width, 1500, seed=4, R=R, h=wl.half_width)
    Dref = orc.convolve_at(R, wl.half_width, B, wl.spatial_degree, a, xs, ys) - I[ys, xs]
    mx, rms = err_stats(D[ys, xs], Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_MFMA


# ------------------------------- precisions that miss the 1e-2 sigma bound ----
# fp16x2 keeps the taps in one fp16 part (11-bit taps) and bf16 / fp16 keep
# both operands in one part: at the chip's brightest star their error exceeds
# the matrix-core bound (measured 1.1e-2 to 3.5e-2 sigma for fp16x2, 4e-2 to
# 0.5 sigma for the single-part forms).  They stay available with that error
# stated; each case is held to the bound and is an expected failure.
def _miss(form, precision, measured):
    return pytest.param(form, precision, id="%s-%s" % (form, precision),
                        marks=pytest.mark.xfail(strict=True, reason="%s/%s misses 1e-2 sigma at the "
                                                "brightest star (measured %s sigma)"
                                                % (form, precision, measured)))


OUTSIDE_BOUND = [_miss("basis", "fp16x2", "1.1e-2"), _miss("regrouped", "fp16x2", "1.2e-2"),
                 _miss("separable", "fp16x2", "3.5e-2"), _miss("basis", "bf16", "0.29"),
                 _miss("basis", "fp16", "4.4e-2"), _miss("regrouped", "bf16", "0.49"),
                 _miss("regrouped", "fp16", "4.3e-2")]


@pytest.mark.parametrize("form,precision", OUTSIDE_BOUND)
def test_precisions_outside_bound(svc, orc, form, precision):
    wl, crops = c2_crops(orc)
    Rc, Ic, a, frame, Dref = crops[1]   # the brightest star
    say("outside-bound precision at the brightest star", form, precision)
    D = run_difference(svc, Rc, Ic, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       precision=precision, form=form, frame=frame, pedestal=synth.SKY_LEVEL)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e (%.2e sigma)" % (mx, rms, mx / np.sqrt(1000)))
    assert np.all(np.isfinite(D))
    assert mx <= TOL_MFMA
