"""The fit at survey scale: 8192 x 8192 star field, 31 x 31 kernel, 49
bases, spatial degree 4 (735 coefficients).  I = float32(Poisson(C(R;
a_hidden))) with C from the oracle's FFT regrouping; the coefficients are
fitted by Gauss-Newton with the bf16x3 and FP32 matrix-core forwards and with
the separable form (forward and adjoint through the Gaussian factors; the
forward in float64 or on the matrix cores in fp16x3), and by Newton steps on
the normal equations (matrix and right-hand side from one pass over the
image; per iteration the forward, the loss, J^T D = JtJ a - J^T I in float64
and the two triangular solves).  Reports the recovered-coefficient error, the
final D RMS in sigma_sky and the Mpix/s of one iteration."""

import numpy as np
import pytest

import synth
from tests.helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4_case(orc):
    wl = synth.WORKLOADS["c4"]
    R, a_hidden = synth.workload_inputs(wl)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    say("c4 synthesis (oracle FFT regrouping)")
    C = orc.convolve_fft(R, wl.half_width, B, wl.spatial_degree, a_hidden)
    I = synth.poisson_noise(C, seed=4)
    r = np.random.default_rng(44)
    a0 = (a_hidden + r.uniform(-0.01, 0.01, a_hidden.shape)).astype(np.float32)
    return wl, R, I, a_hidden, a0


@pytest.mark.parametrize("precision,form", [("bf16x3", "basis"), ("fp32", "basis"),
                                            ("fp32", "separable"), ("fp16x3", "separable")])
def test_fit_survey_scale(svc, c4_case, precision, form):
    import torch
    from paper_1209_5823_amd.fit import gauss_newton_fit
    wl, R, I, a_hidden, a0 = c4_case
    say("c4 fit", precision, form)
    with svc.plan_for(wl, precision=precision, form=form, pedestal=synth.SKY_LEVEL) as plan:
        Rd, Id = to_dev(R), to_dev(I)
        a64, D, hist, t_setup = gauss_newton_fit(plan, Rd, Id, to_dev(a0), iters=3, timings=True)
        a_fit = to_host(a64)
        Dh = to_host(D)
        L_fit, _ = plan.loss_grad(D)
        D_true = plan.difference(Rd, Id, to_dev(a_hidden))
        L_true, _ = plan.loss_grad(D_true)
        L_fit, L_true = float(to_host(L_fit)), float(to_host(L_true))
    h = wl.half_width
    interior = Dh[h:-h, h:-h].astype(np.float64)
    rms = float(np.sqrt(np.mean(interior ** 2)) / synth.sky_sigma())
    err = np.abs(a_fit - a_hidden)
    it_s = min(t for _, _, t in hist)
    say("  setup (normal matrix + Cholesky) %.3f s" % t_setup)
    for k, (L, step, t) in enumerate(hist):
        say("  it %d loss %.6e step %.3e  %.1f ms" % (k, L, step, 1e3 * t))
    say("  max |a - a_hidden| %.3e, rms %.3e; D rms %.4f sigma_sky; %.0f Mpix/s per iteration"
        % (err.max(), np.sqrt(np.mean(err ** 2)), rms, wl.height * wl.width / it_s / 1e6))
    say("  loss at the fit %.9e, at the hidden coefficients %.9e" % (L_fit, L_true))
    # the least-squares minimiser cannot have a larger loss than the hidden
    # coefficients (up to the forward pass's rounding)
    assert L_fit <= L_true * (1 + 1e-6)
    # Poisson noise of the sky and stars sets D's floor: rms just above 1 sigma
    assert 0.95 < rms < 1.6
    assert hist[-1][1] < 1e-2 * hist[0][1]


@pytest.mark.parametrize("precision,form", [("fp16x3", "separable"), ("fp32", "separable")])
def test_least_squares_fit_survey_scale(svc, c4_case, precision, form):
    from paper_1209_5823_amd.fit import least_squares_fit
    wl, R, I, a_hidden, a0 = c4_case
    say("c4 least-squares fit", precision, form)
    with svc.plan_for(wl, precision=precision, form=form, pedestal=synth.SKY_LEVEL) as plan:
        Rd, Id = to_dev(R), to_dev(I)
        a64, D, hist, t_setup = least_squares_fit(plan, Rd, Id, to_dev(a0), iters=4, timings=True)
        a_fit = to_host(a64)
        Dh = to_host(D)
        L_fit = float(to_host(plan.loss_grad(D)[0]))
        L_true = float(to_host(plan.loss_grad(plan.difference(Rd, Id, to_dev(a_hidden)))[0]))
        JtJ = to_host(plan.normal_matrix(Rd))
    h = wl.half_width
    rms = float(np.sqrt(np.mean(Dh[h:-h, h:-h].astype(np.float64) ** 2)) / synth.sky_sigma())
    it_s = sorted(t for _, _, t in hist)[len(hist) // 2]
    say("  setup (normal equations + Cholesky) %.3f s" % t_setup)
    for k, (L, step, t) in enumerate(hist):
        say("  it %d loss %.6e step %.3e  %.2f ms" % (k, L, step, 1e3 * t))
    say("  D rms %.4f sigma_sky; loss at the fit %.9e, at the hidden coefficients %.9e; "
        "median iteration %.2f ms (%.0f Mpix/s)" % (rms, L_fit, L_true, 1e3 * it_s,
                                                     wl.height * wl.width / it_s / 1e6))
    assert L_fit <= L_true * (1 + 1e-6)
    assert 0.95 < rms < 1.6
    # Recovery of the hidden coefficients.  The least-squares estimate has the
    # error covariance (JtJ)^-1 J^T V J (JtJ)^-1 for pixel noise variances V,
    # so its error is large along the eigenvectors of JtJ with small
    # eigenvalues (cond(JtJ) is reported) and bounded in the JtJ norm:
    # q = (a - a*)^T JtJ (a - a*) has expectation NM sigma^2 for white noise of
    # variance sigma^2 (estimated by L_fit / pixels).  Poisson noise weights
    # the bright stars more, so q is held to within a factor 10 of that.
    ev = np.linalg.eigvalsh(JtJ)
    da = (a_fit - a_hidden).ravel().astype(np.float64)
    q = float(da @ JtJ @ da)
    n_pix = (wl.height - 2 * h) * (wl.width - 2 * h)
    q_white = da.size * L_fit / n_pix
    say("  cond(JtJ) %.3e; max |a - a_hidden| %.3e, rms %.3e; (a - a*)^T JtJ (a - a*) = %.4e "
        "= %.3f x the white-noise expectation %.4e; L_true - L_fit = %.4e"
        % (ev[-1] / ev[0], np.abs(da).max(), np.sqrt(np.mean(da ** 2)), q, q / q_white, q_white,
           L_true - L_fit))
    assert 0.1 < q / q_white < 10
    # the loss is quadratic with its minimum at the fit: L_true - L_fit = q
    assert abs((L_true - L_fit) - q) <= 1e-2 * q + 1e-6 * L_true
    # float64 refinement on the normal equations: the last step is at most
    # 1e-4 of the first, at a median iteration of at most 8 ms
    assert hist[-1][1] <= 1e-4 * hist[0][1]
    assert it_s <= 8e-3
