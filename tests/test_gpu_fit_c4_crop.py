"""The fit with the survey-scale basis (49 bases, 31 x 31 kernel, spatial
degree 4: 735 coefficients) on a crop of the 8192 x 8192 frame, against the
FP64 oracle: the normal equations (matrix and right-hand side) element by
element, and the loss of the Gauss-Newton fit and of the Newton steps on the
normal equations against the loss at the oracle's least-squares solution (OIS
least squares, Sec. 2; D is linear in a, Eq. 2 - Eq. 3, so the loss is
quadratic and its minimiser unique)."""

import numpy as np
import pytest

import synth
from tests.helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu

C4 = synth.WORKLOADS["c4"]
CROP = (192, 192)                 # rows, columns
ORIGIN = (3000, 5000)             # x0, y0 of the crop in the 8192 x 8192 frame
N_STARS = 300                     # a dense crop, so that the stars, not the sky, shape the fit


def crop_inputs(orc, frame):
    H, W = CROP
    R = synth.star_field(H, W, N_STARS, C4.fwhm, seed=41)
    a_hidden = synth.coefficients(C4.n_basis, C4.n_spatial, C4.const_basis, C4.seed)
    B = orc.basis(C4.half_width, C4.sigmas, C4.degrees)
    C = orc.convolve(R, C4.half_width, B, C4.spatial_degree, a_hidden, frame=frame)
    I = synth.poisson_noise(C, seed=42)
    return R, I, a_hidden, B


def test_normal_matrix_c4_basis_vs_oracle(svc, orc):
    # the crop in the survey frame's coordinates: over 192 pixels of an 8192-pixel
    # frame the spatial terms are nearly collinear, the matrix is far from
    # invertible, and only its elements are compared
    H, W = CROP
    frame = (ORIGIN[0], ORIGIN[1], C4.width, C4.height)
    R, I, a_hidden, B = crop_inputs(orc, frame)
    say("c4 crop normal equations (oracle)")
    JtJ_ref, rhs_ref = orc.normal_equations(R, I, C4.half_width, B, C4.spatial_degree, frame=frame)
    scale = np.abs(JtJ_ref).max()
    for form in ("separable", "basis"):
        say("c4 crop normal equations", form, JtJ_ref.shape)
        with svc.Plan(H, W, C4.half_width, C4.sigmas, C4.degrees, C4.spatial_degree, form=form,
                      frame=frame) as plan:
            JtJ, rhs = plan.normal_equations(to_dev(R), to_dev(I))
            JtJ, rhs = to_host(JtJ), to_host(rhs)
        err = np.abs(JtJ - JtJ_ref).max() / scale
        err_r = np.abs(rhs - rhs_ref).max() / np.abs(rhs_ref).max()
        say("  max |dJtJ| / max |JtJ| = %.3e, max |drhs| / max |rhs| = %.3e" % (err, err_r))
        # float32 basis responses (float64 passes in the separable form), float64
        # sums: elementwise agreement to float32 rounding of the largest entry
        assert err <= 2e-6 and err_r <= 2e-6
        assert np.allclose(JtJ, JtJ.T, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("method", ["gauss_newton", "normal_equations"])
def test_fit_loss_reaches_oracle_least_squares(svc, orc, method):
    # the crop as its own frame (spatial terms over [-1, 1]): the normal matrix
    # is invertible in float64, though with a condition number near 1e14, so
    # the coefficients are poorly determined while the loss is not
    from paper_1209_5823_amd.fit import gauss_newton_fit, least_squares_fit
    fit = gauss_newton_fit if method == "gauss_newton" else least_squares_fit
    H, W = CROP
    R, I, a_hidden, B = crop_inputs(orc, None)
    say("c4 crop least squares (oracle)")
    JtJ_ref, rhs = orc.normal_equations(R, I, C4.half_width, B, C4.spatial_degree)
    a_ls = orc.cholesky_solve(JtJ_ref, rhs).reshape(a_hidden.shape)
    D_ls = orc.difference(R, I, C4.half_width, B, C4.spatial_degree, a_ls)
    inner = orc.interior_mask(H, W, C4.half_width)
    L_ls = float(np.sum(D_ls[inner] ** 2))
    ev = np.linalg.eigvalsh(JtJ_ref)
    r = np.random.default_rng(43)
    a0 = (a_hidden + r.uniform(-0.01, 0.01, a_hidden.shape)).astype(np.float32)
    say("c4 crop fit (%s); cond(JtJ) = %.3e" % (method, ev[-1] / ev[0]))
    with svc.Plan(H, W, C4.half_width, C4.sigmas, C4.degrees, C4.spatial_degree, form="separable",
                  pedestal=synth.SKY_LEVEL) as plan:
        a64, D, hist, _ = fit(plan, to_dev(R), to_dev(I), to_dev(a0), iters=6)
        a_fit = to_host(a64)
        L_fit = float(to_host(plan.loss_grad(D)[0]))
    for k, (L, step, _) in enumerate(hist):
        say("  it %d loss %.9e step %.3e" % (k, L, step))
    da = (a_fit - a_ls).ravel()
    say("  loss %.9e (oracle least squares %.9e), max |a - a_ls| %.3e, "
        "(a - a_ls)^T JtJ (a - a_ls) = %.3e" % (L_fit, L_ls, np.abs(da).max(), float(da @ JtJ_ref @ da)))
    # the loss is quadratic with its minimum L_ls at a_ls: the fit must reach it
    # to the rounding of the forward pass and of D (float32)
    assert abs(L_fit - L_ls) <= 1e-6 * L_ls
