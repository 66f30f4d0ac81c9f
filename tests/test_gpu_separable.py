"""GPU parity of the separable form (each Gaussian basis is a product of two
one-dimensional factors, so T_n is a row pass then a column pass) against
the FP64 oracle's direct two-dimensional convolution, at the FP32 path's
tolerance of 1e-4 sigma_sky."""

import numpy as np
import pytest

import synth
from tests.helpers import TOL_FP32, say, to_dev, to_host, err_stats, sample_pixels
from tests.test_gpu_forward import EDGE_CASES, _edge_inputs, run_difference

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(EDGE_CASES))
def test_edge_cases_separable(svc, orc, name):
    from paper_1209_5823_amd._lib import SvconvError, EUNSUPPORTED
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    if h < 1 or h > 15:
        with pytest.raises(SvconvError) as ei:
            run_difference(svc, R, I, a, h, sig, deg, d_s, form="separable", frame=frame)
        assert ei.value.status == EUNSUPPORTED
        return
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("separable edge", name, (H, W, h, len(B), d_s))
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, form="separable", frame=frame)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_FP32


@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_c0_full_frame_separable(svc, orc, pedestal):
    wl = synth.WORKLOADS["c0"]
    R, a = synth.workload_inputs(wl)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    C = orc.convolve(R, wl.half_width, B, wl.spatial_degree, a)
    I = (C + 10.0).astype(np.float32)
    say("separable c0", pedestal)
    D = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       form="separable", pedestal=pedestal)
    mx, rms = err_stats(D, C - I.astype(np.float64))
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_FP32


@pytest.mark.parametrize("wl_name", ["c1", "c3", "c4"])
def test_full_size_sampled_separable(svc, orc, wl_name):
    wl = synth.WORKLOADS[wl_name]
    R, a = synth.workload_inputs(wl)
    I = synth.second_image(wl)
    say("separable full size sampled", wl_name, R.shape)
    D = run_difference(svc, R, I, a, wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                       form="separable", pedestal=synth.SKY_LEVEL)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    xs, ys = sample_pixels(wl.height, wl.width, 1500, seed=5, R=R, h=wl.half_width)
    Dref = orc.convolve_at(R, wl.half_width, B, wl.spatial_degree, a, xs, ys) - I[ys, xs]
    mx, rms = err_stats(D[ys, xs], Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_FP32
    assert np.all(np.isfinite(D))


def test_separable_rejects_delta_basis_plans(svc):
    from paper_1209_5823_amd._lib import SvconvError, EUNSUPPORTED
    with svc.Plan.dfb(32, 32, 3, 1) as plan:
        with pytest.raises(SvconvError) as ei:
            plan.set_form("separable")
        assert ei.value.status == EUNSUPPORTED


# ----------------------------------------------- adjoint in a, separable ----

@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_separable_adjoint_a_vs_oracle_c3_crop(svc, orc, pedestal):
    # the c3 crop of the adjoint tests (256 x 256 at frame offset (2100,
    # 1900), 31 x 31 kernel, 49 bases, spatial degree 3) with the same
    # rounding bound: 2e-5 of the magnitude sums sum_p |G| |P_m| |T_n|
    from tests.test_gpu_backward import crop_case, REL, C3
    R, I, a, B, frame = crop_case(orc, C3)
    h, d_s = C3.half_width, C3.spatial_degree
    D = orc.difference(R, I, h, B, d_s, a, frame=frame)
    G = (2.0 * D * orc.interior_mask(*R.shape, h)).astype(np.float32)
    ga_ref = orc.grad_a(R, h, B, d_s, G, frame=frame)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G), frame=frame)[:, :1]
    say("separable adjoint in a, c3 crop, pedestal", pedestal)
    with svc.Plan(R.shape[0], R.shape[1], h, C3.sigmas, C3.degrees, d_s, form="separable",
                  frame=frame, pedestal=pedestal) as plan:
        _, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_gR=False)
        ga = to_host(ga)
    e = np.abs(ga - ga_ref)
    say("  max err %.3e (scale %.3e)" % (e.max(), sa.max()))
    assert np.all(e <= REL * sa + 1e-9)


@pytest.mark.parametrize("name", ["h1_ragged", "nb3_degree3", "max_filters_64",
                                  "max_spatial_degree_6", "single_column", "single_row",
                                  "all_border_8x8"])
def test_separable_adjoint_a_edge_cases(svc, orc, name):
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    G = synth.uniform_image(H, W, seed=17, lo=-40.0, hi=40.0)
    B = orc.basis(h, sig, deg)
    ga_ref = orc.grad_a(R, h, B, d_s, G, frame=frame)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G), frame=frame)[:, :1]
    say("separable adjoint edge", name)
    with svc.Plan(H, W, h, sig, deg, d_s, form="separable", frame=frame,
                  pedestal=synth.SKY_LEVEL) as plan:
        _, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_gR=False)
        ga = to_host(ga)
    e = np.abs(ga - ga_ref)
    say("  max err %.3e" % e.max())
    assert np.all(e <= 2e-5 * sa + 1e-9)


def test_separable_gauss_newton_recovers_noiseless_coefficients(svc, orc):
    import torch
    from tests.test_gpu_fit import small_case
    R, C, a_star, B, (H, W, h, sig, deg, d_s) = small_case(orc, H=96, W=112)
    I = C.astype(np.float32)
    r = np.random.default_rng(1)
    a0 = a_star.astype(np.float64) + r.uniform(-0.02, 0.02, a_star.shape)
    say("gauss-newton, separable form")
    with svc.Plan(H, W, h, sig, deg, d_s, form="separable", pedestal=1000.0) as plan:
        Rd, Id = to_dev(R), to_dev(I)
        JtJ = plan.cholesky_factor(plan.normal_matrix(Rd))
        a64 = torch.from_numpy(a0).cuda()
        a32 = torch.empty(a_star.shape, dtype=torch.float32, device="cuda")
        D = torch.empty_like(Rd)
        hist = [plan.gn_step(Rd, Id, JtJ, a64, a32, D) for _ in range(4)]
        a_fit = to_host(a64)
    err = np.abs(a_fit - a_star).max()
    say("  max |a - a*| = %.3e" % err)
    assert err <= 2e-5
    assert hist[-1][0] < 1e-3 * hist[0][0]


@pytest.mark.parametrize("with_mask,background", [(False, False), (True, False), (False, True)])
def test_separable_normal_matrix_vs_oracle(svc, orc, with_mask, background):
    # basis responses from the separable row and column passes (T-only mode)
    from tests.test_gpu_fit import small_case
    R, C, a_star, B, (H, W, h, sig, deg, d_s) = small_case(orc)
    mask = (synth.uniform_image(H, W, seed=11) > -0.5).astype(np.uint8) if with_mask else None
    if background:
        JtJ_ref, _ = orc.normal_equations_bg(R, C, h, B, d_s, mask=mask)
    else:
        JtJ_ref, _ = orc.normal_equations(R, None, h, B, d_s, mask=mask)
    say("separable normal matrix", with_mask, background)
    with svc.Plan(H, W, h, sig, deg, d_s, form="separable", pedestal=1000.0) as plan:
        plan.set_background(background)
        JtJ = to_host(plan.normal_matrix(to_dev(R), None if mask is None else to_dev(mask)))
    err = np.abs(JtJ - JtJ_ref).max() / np.abs(JtJ_ref).max()
    say("  rel err %.3e" % err)
    assert err <= 2e-6


def test_separable_pcg_with_stamp_preconditioner(svc, orc):
    # the stamp-preconditioned conjugate gradients of the OIS fit, every
    # forward and adjoint in the separable form
    import torch
    from paper_1209_5823_amd.fit import stamp_preconditioned_fit
    wl = synth.WORKLOADS["c0"]
    R, a_star = synth.workload_inputs(wl)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    H, W, h, d_s = wl.height, wl.width, wl.half_width, wl.spatial_degree
    I = synth.poisson_noise(orc.convolve(R, h, B, d_s, a_star), seed=4)
    x_ref = orc.fit_least_squares(R, I, h, B, d_s)
    say("separable pcg")
    with svc.plan_for(wl, form="separable", pedestal=synth.SKY_LEVEL) as plan:
        a0 = torch.zeros(plan._fit_coef, dtype=torch.float64).cuda()
        a0[wl.const_basis, 0] = 1.0
        a64, D, info = stamp_preconditioned_fit(plan, to_dev(R), to_dev(I), a0, synth.SKY_LEVEL,
                                                500.0, iters=12, rounds=2)
        x = to_host(a64)
    res = info["residuals"]
    say("  residuals " + " ".join("%.2e" % v for v in res))
    err = np.abs(x - x_ref).max() / np.abs(x_ref).max()
    say("  max |x - x_ref| / max |x_ref| = %.3e" % err)
    assert err <= 1e-3


# ----------------------------------------------- adjoint in R, separable ----

@pytest.mark.parametrize("pedestal", [0.0, 1000.0])
def test_separable_adjoint_R_vs_oracle_c3_crop(svc, orc, pedestal):
    from tests.test_gpu_backward import crop_case, REL, C3
    R, I, a, B, frame = crop_case(orc, C3)
    h, d_s = C3.half_width, C3.spatial_degree
    D = orc.difference(R, I, h, B, d_s, a, frame=frame)
    G = (2.0 * D * orc.interior_mask(*R.shape, h)).astype(np.float32)
    gR_ref = orc.grad_R(R.shape, h, B, d_s, a, G, frame=frame)
    sR = orc.grad_R(R.shape, h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True), np.abs(G),
                    frame=frame)
    say("separable adjoint in R, c3 crop, pedestal", pedestal)
    with svc.Plan(R.shape[0], R.shape[1], h, C3.sigmas, C3.degrees, d_s, form="separable",
                  frame=frame, pedestal=pedestal) as plan:
        gR, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G))
        gR = to_host(gR)
    e = np.abs(gR - gR_ref)
    say("  max err %.3e (scale %.3e)" % (e.max(), sR.max()))
    assert np.all(e <= REL * sR + 1e-6)


@pytest.mark.parametrize("name", ["h1_ragged", "nb3_degree3", "max_filters_64",
                                  "max_spatial_degree_6", "single_column", "single_row",
                                  "all_border_8x8", "c1_kernel_ragged_crop"])
def test_separable_adjoint_R_edge_cases(svc, orc, name):
    case = EDGE_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    G = synth.uniform_image(H, W, seed=19, lo=-40.0, hi=40.0)
    B = orc.basis(h, sig, deg)
    gR_ref = orc.grad_R((H, W), h, B, d_s, a, G, frame=frame)
    sR = orc.grad_R((H, W), h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True), np.abs(G),
                    frame=frame)
    say("separable adjoint in R, edge", name)
    with svc.Plan(H, W, h, sig, deg, d_s, form="separable", frame=frame) as plan:
        gR, _ = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_ga=False)
        gR = to_host(gR)
    e = np.abs(gR - gR_ref)
    say("  max err %.3e" % e.max())
    assert np.all(e <= 2e-5 * sR + 1e-6)


def test_separable_autograd_matches_dense_form(svc, orc):
    # the torch.autograd.Function on a separable plan gives the same
    # gradients as on the dense matrix-core plan, to float32 rounding
    import torch
    from tests.test_gpu_backward import crop_case, C3
    R, I, a, B, frame = crop_case(orc, C3, size=128)
    grads = {}
    for form in ("basis", "separable"):
        with svc.Plan(128, 128, C3.half_width, C3.sigmas, C3.degrees, C3.spatial_degree,
                      form=form, frame=frame) as plan:
            Rt = to_dev(R).requires_grad_(True)
            at = to_dev(a).requires_grad_(True)
            D = svc.difference(plan, Rt, to_dev(I), at)
            (D.double() ** 2).sum().backward()
            grads[form] = (to_host(Rt.grad), to_host(at.grad))
    for k in range(2):
        g0, g1 = grads["basis"][k], grads["separable"][k]
        assert np.abs(g1 - g0).max() <= 1e-4 * np.abs(g0).max()


# ------------------------------------------- the symmetric fold's variants ----
# Families of degree 1..9: the column pass folds 1, 2, 3 or 4 factors of one
# parity together and applies f_8 / f_9 tap by tap (degrees 8 and 9); spatial
# degrees above 2 take the kernel instance with the long polynomial in yh.
FOLD_CASES = {
    # name: (H, W, h, sigmas, degrees, d_s, frame)
    "degree9": (70, 100, 8, (2.0,), (9,), 2, None),
    "degree8_and_1": (61, 90, 5, (1.5, 3.0), (8, 1), 1, None),
    "degree7_ds4": (64, 70, 6, (1.8,), (7,), 4, None),
    "degree5_3_ds3_h15": (80, 75, 15, (2.5, 5.0), (5, 3), 3, (9, 40, 400, 300)),
    "degree1_ds0": (33, 47, 2, (1.0,), (1,), 0, None),
}


@pytest.mark.parametrize("name", list(FOLD_CASES))
def test_separable_fold_variants(svc, orc, name):
    case = FOLD_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    Dref = orc.difference(R, I, h, B, d_s, a, frame=frame)
    say("separable fold", name, (H, W, h, len(B), d_s))
    D = run_difference(svc, R, I, a, h, sig, deg, d_s, form="separable", frame=frame)
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= TOL_FP32


@pytest.mark.parametrize("name", list(FOLD_CASES))
def test_separable_fold_variants_adjoint_a(svc, orc, name):
    case = FOLD_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    G = synth.uniform_image(H, W, seed=23, lo=-40.0, hi=40.0)
    B = orc.basis(h, sig, deg)
    ga_ref = orc.grad_a(R, h, B, d_s, G, frame=frame)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G), frame=frame)[:, :1]
    say("separable fold, adjoint in a", name)
    with svc.Plan(H, W, h, sig, deg, d_s, form="separable", frame=frame,
                  pedestal=synth.SKY_LEVEL) as plan:
        _, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G), want_gR=False)
        ga = to_host(ga)
    e = np.abs(ga - ga_ref)
    say("  max err %.3e" % e.max())
    assert np.all(e <= 2e-5 * sa + 1e-9)


@pytest.mark.parametrize("name", ["degree9", "degree8_and_1", "degree5_3_ds3_h15"])
def test_separable_fold_variants_normal_matrix(svc, orc, name):
    # the T-only instance of the contraction writes the basis responses
    case = FOLD_CASES[name]
    H, W, h, sig, deg, d_s, frame = case
    R, I, a = _edge_inputs(name, case)
    B = orc.basis(h, sig, deg)
    JtJ_ref, _ = orc.normal_equations(R, None, h, B, d_s, frame=frame)
    say("separable fold, normal matrix", name)
    with svc.Plan(H, W, h, sig, deg, d_s, form="separable", frame=frame,
                  pedestal=synth.SKY_LEVEL) as plan:
        JtJ = to_host(plan.normal_matrix(to_dev(R)))
    err = np.abs(JtJ - JtJ_ref).max() / np.abs(JtJ_ref).max()
    say("  rel err %.3e" % err)
    assert err <= 2e-6
