"""GPU parity of the least-squares fit pieces: loss and gradient, normal
matrix and normal equations, Cholesky factor and solve, Gauss-Newton recovery
of noiseless coefficients, and the Newton steps on the normal equations
reaching the oracle's least-squares solution; all against the FP64 oracle or
numpy's FP64 linear algebra."""

import numpy as np
import pytest

import synth
from tests.helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu


def small_case(orc, H=48, W=56, h=4, sig=(0.7, 1.5), deg=(2, 1), d_s=2, seed=9):
    r = np.random.default_rng(seed)
    R = synth.star_field(H, W, 12, seed=seed)
    N, M = synth.n_basis(deg), synth.n_spatial(d_s)
    a_star = (r.normal(size=(N, M)) * 0.05).astype(np.float32)
    a_star[0, 0] = 1.0
    B = orc.basis(h, sig, deg)
    C = orc.convolve(R, h, B, d_s, a_star)
    return R, C, a_star, B, (H, W, h, sig, deg, d_s)


def test_loss_grad(svc, orc):
    H, W, h = 40, 52, 5
    D = synth.uniform_image(H, W, seed=4, lo=-30, hi=30)
    mask = (synth.uniform_image(H, W, seed=5) > 0).astype(np.uint8)
    with svc.Plan(H, W, h, (1.5,), (0,), 1) as plan:
        for m in (None, mask):
            L, G = plan.loss_grad(to_dev(D), None if m is None else to_dev(m))
            L, G = float(to_host(L)), to_host(G)
            sel = orc.interior_mask(H, W, h) if m is None else m.astype(bool)
            assert abs(L - np.sum(D.astype(np.float64)[sel] ** 2)) <= 1e-12 * L
            assert np.array_equal(G, np.where(sel, 2 * D, 0).astype(np.float32))


# 9 bases take one 16-filter block of the contraction; 6 bases (at most 8)
# take its two-row packed form, whose basis responses come out of both halves
# of the matrix-core accumulator.  Width 56 runs the Gram sums on whole
# 16-pixel steps plus a ragged one; width 61 (not a multiple of 4) runs them
# all on the element-wise path.
@pytest.mark.parametrize("width", [56, 61])
@pytest.mark.parametrize("basis", [((0.7, 1.5), (2, 1)), ((1.5,), (2,))], ids=["n9", "n6"])
@pytest.mark.parametrize("with_mask", [False, True])
def test_normal_matrix_vs_oracle(svc, orc, with_mask, basis, width):
    sig, deg = basis
    R, C, a_star, B, (H, W, h, sig, deg, d_s) = small_case(orc, H=53, W=width, sig=sig, deg=deg)
    mask = None
    if with_mask:
        mask = (synth.uniform_image(H, W, seed=11) > -0.5).astype(np.uint8)
    JtJ_ref, _ = orc.normal_equations(R, None, h, B, d_s, mask=mask)
    say("normal matrix", with_mask, len(B))
    with svc.Plan(H, W, h, sig, deg, d_s) as plan:
        JtJ = to_host(plan.normal_matrix(to_dev(R), None if mask is None else to_dev(mask)))
    err = np.abs(JtJ - JtJ_ref).max() / np.abs(JtJ_ref).max()
    say("  rel err %.3e" % err)
    assert err <= 2e-6          # float32 basis responses, float64 sums
    assert np.allclose(JtJ, JtJ.T, rtol=0, atol=1e-12 * np.abs(JtJ).max())


def test_cholesky_factor_and_solve(svc):
    import torch
    from paper_1209_5823_amd._lib import SvconvError, ENOTSPD
    r = np.random.default_rng(2)
    for n in (1, 7, 130, 735):
        X = r.normal(size=(n + 5, n))
        A = X.T @ X + 0.5 * np.eye(n)
        b = r.normal(size=n)
        say("cholesky", n)
        with svc.Plan(8, 8, 1, (1.0,), (0,), 0) as plan:
            Ad = torch.from_numpy(A.copy()).cuda()
            plan.cholesky_factor(Ad)
            L = to_host(Ad)
            Lref = np.linalg.cholesky(A)
            assert np.max(np.abs(L - Lref)) <= 1e-10 * np.abs(Lref).max()
            x = to_host(plan.cholesky_solve(Ad, torch.from_numpy(b).cuda()))
            xref = np.linalg.solve(A, b)
            assert np.max(np.abs(x - xref)) <= 1e-9 * max(1.0, np.abs(xref).max())
    with svc.Plan(8, 8, 1, (1.0,), (0,), 0) as plan:
        bad = torch.from_numpy(np.diag([1.0, 2.0, -1.0, 3.0])).cuda()
        with pytest.raises(SvconvError) as ei:
            plan.cholesky_factor(bad)
        assert ei.value.status == ENOTSPD


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_gauss_newton_recovers_noiseless_coefficients(svc, orc, precision):
    import torch
    R, C, a_star, B, (H, W, h, sig, deg, d_s) = small_case(orc, H=96, W=112)
    I = C.astype(np.float32)
    r = np.random.default_rng(1)
    a0 = a_star.astype(np.float64) + r.uniform(-0.02, 0.02, a_star.shape)
    say("gauss-newton", precision)
    with svc.Plan(H, W, h, sig, deg, d_s, precision=precision, pedestal=1000.0) as plan:
        Rd, Id = to_dev(R), to_dev(I)
        JtJ = plan.normal_matrix(Rd)
        plan.cholesky_factor(JtJ)
        a64 = torch.from_numpy(a0).cuda()
        a32 = torch.empty(a_star.shape, dtype=torch.float32, device="cuda")
        D = torch.empty_like(Rd)
        hist = []
        for it in range(4):
            L, step = plan.gn_step(Rd, Id, JtJ, a64, a32, D)
            hist.append((L, step))
            say("  it %d loss %.6e step %.3e" % (it, L, step))
        a_fit = to_host(a64)
    err = np.abs(a_fit - a_star).max()
    say("  max |a - a*| = %.3e" % err)
    tol = 2e-5 if precision == "fp32" else 2e-3
    assert err <= tol
    assert hist[-1][0] < 1e-3 * hist[0][0]


@pytest.mark.parametrize("form,precision,with_mask", [("basis", "fp32", False),
                                                      ("separable", "fp32", True),
                                                      ("separable_regrouped", "fp16x3", False)])
def test_normal_equations_vs_oracle(svc, orc, form, precision, with_mask):
    R, C, a_star, B, (H, W, h, sig, deg, d_s) = small_case(orc)
    I = synth.poisson_noise(C, seed=12)
    mask = None
    if with_mask:
        mask = (synth.uniform_image(H, W, seed=11) > -0.5).astype(np.uint8)
    JtJ_ref, rhs_ref = orc.normal_equations(R, I, h, B, d_s, mask=mask)
    say("normal equations", form, precision, with_mask)
    with svc.Plan(H, W, h, sig, deg, d_s, precision=precision, form=form) as plan:
        JtJ, rhs = plan.normal_equations(to_dev(R), to_dev(I), None if mask is None else to_dev(mask))
        JtJ, rhs = to_host(JtJ), to_host(rhs)
        JtJ_only = to_host(plan.normal_matrix(to_dev(R), None if mask is None else to_dev(mask)))
    e_m = np.abs(JtJ - JtJ_ref).max() / np.abs(JtJ_ref).max()
    e_r = np.abs(rhs - rhs_ref).max() / np.abs(rhs_ref).max()
    say("  rel err JtJ %.3e rhs %.3e" % (e_m, e_r))
    # float32 basis responses, float64 sums
    assert e_m <= 2e-6 and e_r <= 2e-6
    # the extra plane of I changes no entry of the matrix
    assert np.array_equal(JtJ, JtJ_only)


@pytest.mark.parametrize("form,precision", [("separable", "fp32"), ("basis", "bf16x3"),
                                            ("separable_regrouped", "fp16x3")])
def test_least_squares_steps_reach_oracle_solution(svc, orc, form, precision):
    import torch
    from paper_1209_5823_amd.fit import least_squares_fit
    R, C, a_star, B, (H, W, h, sig, deg, d_s) = small_case(orc, H=96, W=112)
    I = synth.poisson_noise(C, seed=13)
    JtJ_ref, rhs_ref = orc.normal_equations(R, I, h, B, d_s)
    a_ls = orc.cholesky_solve(JtJ_ref, rhs_ref).reshape(a_star.shape)
    inner = orc.interior_mask(H, W, h)
    L_ls = float(np.sum(orc.difference(R, I, h, B, d_s, a_ls)[inner] ** 2))
    r = np.random.default_rng(3)
    a0 = (a_star + r.uniform(-0.02, 0.02, a_star.shape)).astype(np.float32)
    say("least-squares steps", form, precision)
    with svc.Plan(H, W, h, sig, deg, d_s, precision=precision, form=form, pedestal=1000.0) as plan:
        a64, D, hist, _ = least_squares_fit(plan, to_dev(R), to_dev(I), to_dev(a0), iters=4)
        a_fit = to_host(a64)
    for k, (L, step, _) in enumerate(hist):
        say("  it %d loss %.9e step %.3e" % (k, L, step))
    da = (a_fit - a_ls).ravel()
    q = float(da @ JtJ_ref @ da)
    L_fit = float(np.sum(orc.difference(R, I, h, B, d_s, a_fit)[inner] ** 2))
    say("  loss %.9e (oracle %.9e), (a - a_ls)^T JtJ (a - a_ls) = %.3e" % (L_fit, L_ls, q))
    # the loss is quadratic with minimum L_ls at a_ls: L(a) - L_ls = q, and the
    # float32 basis responses in JtJ and rhs move the solution by far less
    # than the noise
    assert q <= 1e-6 * L_ls
    assert abs(L_fit - L_ls) <= 1e-6 * L_ls
    # float64 refinement: the steps fall by orders of magnitude
    assert hist[-1][1] <= 1e-6 * hist[0][1]
