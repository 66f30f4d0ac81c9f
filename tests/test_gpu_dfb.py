"""GPU parity of the Dirac delta basis (the paper's own benchmark case:
one basis per kernel pixel, second-order spatial polynomial) against the
FP64 oracle, through svconv_plan_create_dfb."""

import numpy as np
import pytest

import synth
from tests.helpers import (TOL_FP32, TOL_MFMA, say, to_dev, to_host, err_stats, sample_pixels)

pytestmark = pytest.mark.gpu


def dfb_inputs(H, W, h, d_s, seed):
    k = 2 * h + 1
    R = synth.star_field(H, W, max(1, H * W // 500), synth.configs._fwhm_const(2.0), seed=seed)
    I = synth.star_field(H, W, max(1, H * W // 500), synth.configs._fwhm_const(2.0), seed=seed + 1)
    # centre pixel carries the constant 1, every other kernel pixel 5% terms
    a = synth.coefficients(k * k, synth.n_spatial(d_s), (k * k) // 2, seed=seed)
    return R, I, a


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("form", ["basis", "regrouped"])
def test_dfb_7x7_second_order(svc, orc, form, precision):
    H, W, h, d_s = 160, 230, 3, 2
    R, I, a = dfb_inputs(H, W, h, d_s, seed=21)
    Dref = orc.difference(R, I, h, orc.basis_dfb(h), d_s, a)
    say("dfb 7x7", form, precision)
    with svc.Plan.dfb(H, W, h, d_s, precision=precision, form=form,
                      pedestal=synth.SKY_LEVEL) as plan:
        D = to_host(plan.difference(to_dev(R), to_dev(I), to_dev(a)))
    mx, rms = err_stats(D, Dref)
    say("  max %.3e rms %.3e" % (mx, rms))
    assert mx <= (TOL_FP32 if precision == "fp32" else TOL_MFMA)


@pytest.mark.parametrize("h,d_s", [(6, 2), (4, 3)])
def test_dfb_more_bases_than_the_basis_form_holds(svc, orc, h, d_s):
    # 169 and 81 delta bases: regrouped form only
    from paper_1209_5823_amd._lib import SvconvError, EUNSUPPORTED
    H, W = 120, 150
    R, I, a = dfb_inputs(H, W, h, d_s, seed=h)
    Dref = orc.difference(R, I, h, orc.basis_dfb(h), d_s, a)
    say("dfb regrouped", h, d_s)
    with svc.Plan.dfb(H, W, h, d_s) as plan:
        D = to_host(plan.difference(to_dev(R), to_dev(I), to_dev(a)))
        with pytest.raises(SvconvError) as ei:
            plan.set_form("basis")
        assert ei.value.status == EUNSUPPORTED
        assert plan.form == "regrouped"
    mx, _ = err_stats(D, Dref)
    assert mx <= TOL_FP32


def test_dfb_adjoint(svc, orc):
    # rounding bound as for the Gaussian basis: a small multiple of 2^-24
    # times the magnitude sums sum_p |G| |T_n| and sum |G| |K|
    H, W, h, d_s = 64, 72, 2, 2
    R, _, a = dfb_inputs(H, W, h, d_s, seed=5)
    G = synth.uniform_image(H, W, seed=6, lo=-50, hi=50)
    B = orc.basis_dfb(h)
    ga_ref = orc.grad_a(R, h, B, d_s, G)
    gR_ref = orc.grad_R(R.shape, h, B, d_s, a, G)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G))[:, :1]
    sR = orc.grad_R(R.shape, h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True), np.abs(G))
    say("dfb adjoint 5x5")
    with svc.Plan.dfb(H, W, h, d_s) as plan:
        gR, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G))
        gR, ga = to_host(gR), to_host(ga)
    ea, eR = np.abs(ga - ga_ref), np.abs(gR - gR_ref)
    say("  ga max err %.3e  gR max err %.3e" % (ea.max(), eR.max()))
    assert np.all(ea <= 2e-5 * sa + 1e-9)
    assert np.all(eR <= 2e-5 * sR + 1e-6)


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_dfb_pan_starrs_tile_sampled(svc, orc, precision):
    # one 4846 x 4868 camera tile (the paper's cost-model tile), 7 x 7 DFB
    H, W, h, d_s = 4846, 4868, 3, 2
    R, I, a = dfb_inputs(H, W, h, d_s, seed=7)
    say("dfb tile", precision)
    with svc.Plan.dfb(H, W, h, d_s, precision=precision, pedestal=synth.SKY_LEVEL) as plan:
        D = to_host(plan.difference(to_dev(R), to_dev(I), to_dev(a)))
    xs, ys = sample_pixels(H, W, 1000, seed=8, R=R, h=h)
    Dref = orc.convolve_at(R, h, orc.basis_dfb(h), d_s, a, xs, ys) - I[ys, xs]
    mx, _ = err_stats(D[ys, xs], Dref)
    say("  max %.3e" % mx)
    assert mx <= (TOL_FP32 if precision == "fp32" else TOL_MFMA)
