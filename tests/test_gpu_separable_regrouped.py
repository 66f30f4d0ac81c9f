"""GPU parity of the regrouped separable form (the coefficients folded into
per-call column filters g_{r,m} = sum_j a[n(r,j)][m] f_j, so that
sum_n c_n T_n = sum_m P_m sum_r g_{r,m} (x)_y (f_r (x)_x R); row and column
passes as Toeplitz products of hi/lo parts on the matrix cores) against the
FP64 oracle's direct two-dimensional convolution, at the matrix-core forms'
bound of 1e-2 sigma_sky."""

import numpy as np
import pytest

import synth
from tests.helpers import TOL_MFMA, say, err_stats, sample_pixels, to_dev, to_host
from tests.test_gpu_forward import EDGE_CASES, _edge_inputs, run_difference

pytestmark = pytest.mark.gpu

FORM = "separable_regrouped"
PRECISIONS = ["fp16x3", "bf16x3"]
C0 = synth.WORKLOADS["c0"]

# cases of the form's range (1 <= h <= 12, spatial degree <= 2): the shared
# edge cases plus the largest half-width, spatial degrees 0 and 1, and odd
# numbers of row factors
CASES = {name: EDGE_CASES[name] for name in
         ("kernel_larger_than_image", "all_border_8x8", "h1_ragged", "c1_kernel_ragged_crop",
          "max_filters_64", "single_row", "single_column")}
CASES.update({
    "max_half_width_12": (100, 150, 12, (0.7, 1.5, 2.0), (6, 4, 2), 2, (700, 300, 4096, 2048)),
    "spatial_degree_0": (70, 130, 5, (1.0, 2.0), (3, 1), 0, None),
    "spatial_degree_1": (66, 200, 8, (0.9, 1.6), (4, 2), 1, (10, 20, 500, 400)),
    "one_family_odd_rows": (130, 65, 3, (1.2,), (4,), 2, None),
    "one_row_factor": (64, 64, 2, (1.5,), (0,), 2, None),
})


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_c0_full_frame(svc, orc, precision, pedestal):
    R, a = synth.workload_inputs(C0)
    B = orc.basis(C0.half_width, C0.sigmas, C0.degrees)
    C = orc.convolve(R, C0.half_width, B, C0.spatial_degree, a)
    I = (C + 10.0).astype(np.float32)
    Dref = C - I.astype(np.float64)
    say("regrouped separable c0", precision, pedestal)
    D = run_difference(svc, R, I, a, C0.half_width, C0.sigmas, C0.degrees, C0.spatial_degree,
                       precision=precision, form=FORM, pedestal=pedestal)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e (%.2e sigma)" % (mx, rms, mx / np.sqrt(1000)))
    assert mx <= TOL_MFMA


@pytest.mark.parametrize("precision", PRECISIONS)
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
        say("regrouped separable c2 crop", precision, (y0, x0))
        D = run_difference(svc, Rc, Ic, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                           precision=precision, form=FORM, frame=frame, pedestal=synth.SKY_LEVEL)
        mx, rms = err_stats(D, Dref)
        say("  max %.3e rms %.3e (%.2e sigma)" % (mx, rms, mx / np.sqrt(1000)))
        assert mx <= TOL_MFMA


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name", list(CASES))
def test_edge_cases(svc, orc, name, precision):
    case = CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("regrouped separable edge", name, precision, (H, W, h, len(B), d_s))
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, precision=precision, form=FORM,
                       frame=frame, pedestal=synth.SKY_LEVEL)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_MFMA
    assert np.all(np.isfinite(D))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_chip_sampled(svc, orc, precision):
    # the 2048 x 4096 chip at full size in the launch configuration the bench
    # times, on sampled pixels (and the brightest ones) against the oracle
    wl = synth.WORKLOADS["c1"]
    R, a = synth.workload_inputs(wl)
    I = synth.second_image(wl)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    say("regrouped separable c1 full size", precision)
    D = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       precision=precision, form=FORM, pedestal=synth.SKY_LEVEL)
    xs, ys = sample_pixels(wl.height, wl.width, 20000, seed=6, R=R, h=wl.half_width)
    Dref = orc.convolve_at(R, wl.half_width, B, wl.spatial_degree, a, xs, ys) - I[ys, xs]
    e = np.abs(D[ys, xs] - Dref)
    say("  max %.3e (%.2e sigma) over %d pixels" % (e.max(), e.max() / np.sqrt(1000), len(ys)))
    assert e.max() <= TOL_MFMA
    assert np.all(np.isfinite(D))


def test_repeated_calls_identical(svc):
    # no atomics and no state carried between calls: the same inputs give the
    # same bits, also after a call with other coefficients
    wl = synth.WORKLOADS["c0"]
    R, a = synth.workload_inputs(wl)
    a2 = synth.coefficients(wl.n_basis, wl.n_spatial, wl.const_basis, seed=9)
    I = synth.star_field(wl.height, wl.width, 50, seed=4)
    with svc.Plan(wl.height, wl.width, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                  precision="fp16x3", form=FORM, pedestal=synth.SKY_LEVEL) as plan:
        Rd, Id, ad, a2d = to_dev(R), to_dev(I), to_dev(a), to_dev(a2)
        say("regrouped separable repeated calls")
        D1 = to_host(plan.difference(Rd, Id, ad))
        plan.difference(Rd, Id, a2d)
        D2 = to_host(plan.difference(Rd, Id, ad))
    assert np.array_equal(D1, D2)


def test_matches_separable_form(svc):
    # both matrix-core separable forms compute D of Eq. 1; on the chip's
    # kernel and basis they agree far inside the bound
    wl = synth.WORKLOADS["c1"]
    H, W = 300, 520
    R = synth.star_field(H, W, 400, wl.fwhm, seed=21)
    I = synth.star_field(H, W, 400, wl.fwhm, seed=22)
    _, a = synth.workload_inputs(wl)
    frame = (1500, 900, wl.width, wl.height)
    say("regrouped separable against separable")
    D0 = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                        precision="fp16x3", form="separable", frame=frame, pedestal=synth.SKY_LEVEL)
    D1 = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                        precision="fp16x3", form=FORM, frame=frame, pedestal=synth.SKY_LEVEL)
    mx, _ = err_stats(D1, D0)
    say("  max |dD| %.3e" % mx)
    assert mx <= 0.1 * TOL_MFMA


@pytest.mark.parametrize("what", ["spatial_degree_3", "half_width_13", "fp32", "delta_basis"])
def test_rejects_outside_range(svc, what):
    import torch
    from paper_1209_5823_amd._lib import SvconvError, EUNSUPPORTED
    say("regrouped separable rejects", what)
    if what == "delta_basis":
        with svc.Plan.dfb(32, 32, 2, 1, precision="fp16x3") as plan:
            with pytest.raises(SvconvError) as ei:
                plan.set_form(FORM)
        assert ei.value.status == EUNSUPPORTED
        return
    d_s = 3 if what == "spatial_degree_3" else 2
    h = 13 if what == "half_width_13" else 4
    with svc.Plan(40, 40, h, (1.5,), (1,), d_s, precision="fp16x3") as plan:
        if what in ("spatial_degree_3", "half_width_13"):
            with pytest.raises(SvconvError) as ei:
                plan.set_form(FORM)
            assert ei.value.status == EUNSUPPORTED
            return
        plan.set_form(FORM)
        plan.set_precision("fp32")
        R = torch.zeros((40, 40), dtype=torch.float32, device="cuda")
        a = torch.zeros((3, 6), dtype=torch.float32, device="cuda")
        with pytest.raises(SvconvError) as ei:
            plan.forward(R, a)
        assert ei.value.status == EUNSUPPORTED
