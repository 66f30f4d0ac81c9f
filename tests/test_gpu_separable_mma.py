"""GPU parity of the separable form on the matrix cores (the split 16-bit
precisions): the row and column passes of the Gaussian factors as banded
Toeplitz products, against the FP64 oracle's direct two-dimensional
convolution, at the matrix-core forms' bound of 1e-2 sigma_sky."""

import numpy as np
import pytest

import synth
from tests.helpers import TOL_MFMA, say, err_stats, sample_pixels, to_dev, to_host, workload_images
from tests.test_gpu_forward import EDGE_CASES, _edge_inputs, run_difference, LOWP
from tests.test_gpu_separable import FOLD_CASES

pytestmark = pytest.mark.gpu

C0 = synth.WORKLOADS["c0"]


@pytest.mark.parametrize("precision", LOWP)
@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_c0_full_frame(svc, orc, precision, pedestal):
    R, a = synth.workload_inputs(C0)
    B = orc.basis(C0.half_width, C0.sigmas, C0.degrees)
    C = orc.convolve(R, C0.half_width, B, C0.spatial_degree, a)
    I = (C + 10.0).astype(np.float32)
    Dref = C - I.astype(np.float64)
    say("separable mma c0", precision, pedestal)
    D = run_difference(svc, R, I, a, C0.half_width, C0.sigmas, C0.degrees, C0.spatial_degree,
                       precision=precision, form="separable", pedestal=pedestal)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e (%.2e sigma)" % (mx, rms, mx / np.sqrt(1000)))
    assert mx <= TOL_MFMA


@pytest.mark.parametrize("precision", LOWP)
def test_c2_crops(svc, orc, precision):
    # 512 x 512 crops of the 2048 x 4096 chip: the centre and the brightest star
    wl = synth.WORKLOADS["c2"]
    R, a = synth.workload_inputs(wl)
    I = synth.second_image(wl)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    yb, xb = np.unravel_index(np.argmax(R), R.shape)
    crops = [(768, 1792), (int(np.clip(yb - 256, 0, wl.height - 512)),
                           int(np.clip(xb - 256, 0, wl.width - 512)))]
    for (y0, x0) in crops:
        Rc = np.ascontiguousarray(R[y0:y0 + 512, x0:x0 + 512])
        Ic = np.ascontiguousarray(I[y0:y0 + 512, x0:x0 + 512])
        frame = (x0, y0, wl.width, wl.height)
        Dref = orc.difference(Rc, Ic, wl.half_width, B, wl.spatial_degree, a, frame=frame)
        say("separable mma c2 crop", precision, (y0, x0))
        D = run_difference(svc, Rc, Ic, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                           precision=precision, form="separable", frame=frame, pedestal=synth.SKY_LEVEL)
        mx, rms = err_stats(D, Dref)
        say("  max %.3e rms %.3e (%.2e sigma)" % (mx, rms, mx / np.sqrt(1000)))
        assert mx <= TOL_MFMA


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("name", ["h1_ragged", "nb3_degree3", "c1_kernel_ragged_crop", "c3_kernel_degree4",
                                  "max_filters_64", "max_spatial_degree_6", "single_row", "single_column",
                                  "all_border_8x8", "kernel_larger_than_image"])
def test_edge_cases(svc, orc, name, precision):
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("separable mma edge", name, precision)
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, precision=precision, form="separable",
                       frame=frame, pedestal=synth.SKY_LEVEL)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_MFMA


@pytest.mark.parametrize("name", list(FOLD_CASES))
def test_high_degree_families(svc, orc, name):
    case = FOLD_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("separable mma family", name)
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, precision="fp16x3", form="separable",
                       frame=frame, pedestal=synth.SKY_LEVEL)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_MFMA


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("wl_name", ["c1", "c3", "c4"])
def test_full_size_sampled(svc, orc, precision, wl_name):
    # full-size frames in the launch configurations the bench and the fit time
    # (the 2048 x 4096 chip; 4096^2 with a 31 x 31 kernel and spatial degree 3;
    # 8192^2 with spatial degree 4), checked on sampled pixels (and the brightest
    # ones) against the oracle
    wl = synth.WORKLOADS[wl_name]
    R, a, I = workload_images(wl_name)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    say("separable mma full size", wl_name, precision)
    D = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       precision=precision, form="separable", pedestal=synth.SKY_LEVEL)
    n = 20000 if wl_name == "c1" else 6000
    xs, ys = sample_pixels(wl.height, wl.width, n, seed=5, R=R, h=wl.half_width)
    Dref = orc.convolve_at(R, wl.half_width, B, wl.spatial_degree, a, xs, ys) - I[ys, xs]
    e = np.abs(D[ys, xs] - Dref)
    say("  max %.3e (%.2e sigma) over %d pixels" % (e.max(), e.max() / np.sqrt(1000), len(ys)))
    assert e.max() <= TOL_MFMA
    assert np.all(np.isfinite(D))


# ------------------------------------ adjoint in R on the matrix cores ----
# The split precisions route the separable adjoint in R through the Toeplitz
# fragments (bf16x3 for both); its error is bounded by a multiple of the
# magnitude sums, like the float32 adjoints, with the bf16x3 products' 2^-16.
MMA_ADJ_REL = 2e-4


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
def test_adjoint_R_mma_vs_oracle_c3_crop(svc, orc, precision):
    from tests.test_gpu_backward import crop_case, C3
    R, I, a, B, frame = crop_case(orc, C3)
    h, d_s = C3.half_width, C3.spatial_degree
    D = orc.difference(R, I, h, B, d_s, a, frame=frame)
    G = (2.0 * D * orc.interior_mask(*R.shape, h)).astype(np.float32)
    gR_ref = orc.grad_R(R.shape, h, B, d_s, a, G, frame=frame)
    sR = orc.grad_R(R.shape, h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True), np.abs(G),
                    frame=frame)
    say("matrix-core separable adjoint in R, c3 crop,", precision)
    with svc.Plan(R.shape[0], R.shape[1], h, C3.sigmas, C3.degrees, d_s, precision=precision,
                  form="separable", frame=frame) as plan:
        gR, _ = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_ga=False)
        gR = to_host(gR)
    e = np.abs(gR - gR_ref)
    say("  max err %.3e (scale %.3e), max err / scale %.3e" % (e.max(), sR.max(), (e / (sR + 1e-30)).max()))
    assert np.all(e <= MMA_ADJ_REL * sR + 1e-5)


@pytest.mark.parametrize("name", ["h1_ragged", "nb3_degree3", "max_filters_64",
                                  "max_spatial_degree_6", "single_column", "single_row",
                                  "all_border_8x8", "c1_kernel_ragged_crop", "one_pixel_h1"])
def test_adjoint_R_mma_edge_cases(svc, orc, name):
    if name == "one_pixel_h1":
        case = (1, 1, 1, (1.5,), (1,), 1, None)
    else:
        case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    G = synth.uniform_image(H, W, seed=19, lo=-40.0, hi=40.0)
    B = orc.basis(h, sig, deg)
    gR_ref = orc.grad_R((H, W), h, B, d_s, a, G, frame=frame)
    sR = orc.grad_R((H, W), h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True), np.abs(G),
                    frame=frame)
    say("matrix-core separable adjoint in R, edge", name)
    with svc.Plan(H, W, h, sig, deg, d_s, precision="fp16x3", form="separable", frame=frame) as plan:
        gR, _ = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_ga=False)
        gR = to_host(gR)
    e = np.abs(gR - gR_ref)
    say("  max err %.3e (scale %.3e)" % (e.max(), sR.max()))
    assert np.all(e <= MMA_ADJ_REL * sR + 1e-5)


# ------------------------------------ adjoint in a on the matrix cores ----
# The split precisions take the adjoint in a through the forward's Toeplitz
# passes, with the moment sums sum_p G P_m T_n in place of the epilogue; bound:
# a multiple of the magnitude sums sum_p |G| |T_n|, ten times the float32
# adjoints' (the products of the split precision and float32 tile sums).
MMA_ADJ_A_REL = 2e-4


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_adjoint_a_mma_vs_oracle_c3_crop(svc, orc, precision, pedestal):
    from tests.test_gpu_backward import crop_case, C3
    R, I, a, B, frame = crop_case(orc, C3)
    h, d_s = C3.half_width, C3.spatial_degree
    D = orc.difference(R, I, h, B, d_s, a, frame=frame)
    G = (2.0 * D * orc.interior_mask(*R.shape, h)).astype(np.float32)
    ga_ref = orc.grad_a(R, h, B, d_s, G, frame=frame)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G), frame=frame)[:, :1]
    say("matrix-core separable adjoint in a, c3 crop,", precision, "pedestal", pedestal)
    with svc.Plan(R.shape[0], R.shape[1], h, C3.sigmas, C3.degrees, d_s, precision=precision,
                  form="separable", frame=frame, pedestal=pedestal) as plan:
        _, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_gR=False)
        ga = to_host(ga)
    e = np.abs(ga - ga_ref)
    say("  max err %.3e (scale %.3e), max err / scale %.3e" % (e.max(), sa.max(), (e / sa).max()))
    assert np.all(e <= MMA_ADJ_A_REL * sa + 1e-9)


@pytest.mark.parametrize("name", ["h1_ragged", "nb3_degree3", "max_filters_64",
                                  "max_spatial_degree_6", "single_column", "single_row",
                                  "all_border_8x8", "c1_kernel_ragged_crop"])
def test_adjoint_a_mma_edge_cases(svc, orc, name):
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    G = synth.uniform_image(H, W, seed=17, lo=-40.0, hi=40.0)
    B = orc.basis(h, sig, deg)
    ga_ref = orc.grad_a(R, h, B, d_s, G, frame=frame)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G), frame=frame)[:, :1]
    say("matrix-core separable adjoint in a, edge", name)
    with svc.Plan(H, W, h, sig, deg, d_s, precision="fp16x3", form="separable", frame=frame,
                  pedestal=synth.SKY_LEVEL) as plan:
        _, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_gR=False)
        ga = to_host(ga)
    e = np.abs(ga - ga_ref)
    say("  max err %.3e (scale %.3e)" % (e.max(), sa.max()))
    assert np.all(e <= MMA_ADJ_A_REL * sa + 1e-9)
