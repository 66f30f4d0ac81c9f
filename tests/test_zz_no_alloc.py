"""svconv_difference_noalloc (no plan, no allocation: every table in the
library's static scratch array) against svconv_difference of a plan in the
regrouped separable form, through the C ABI, on two calls in a row, the
second with a smaller input.  Its rejection of sizes beyond the scratch array
is tested without a GPU (tests/test_abi.py)."""

import numpy as np
import pytest

import synth
from tests.helpers import TOL_MFMA, say, err_stats, to_dev, to_host

pytestmark = pytest.mark.gpu


def noalloc(svc, R, I, a, h, sigmas, degrees, d_s, precision, pedestal):
    return to_host(svc.difference_noalloc(R, I, a, h, sigmas, degrees, d_s, precision=precision,
                                          pedestal=pedestal))


def with_plan(svc, R, I, a, h, sigmas, degrees, d_s, precision, pedestal):
    H, W = R.shape
    with svc.Plan(H, W, h, sigmas, degrees, d_s, precision=precision, form="separable_regrouped",
                  pedestal=pedestal) as plan:
        return to_host(plan.difference(R, I, a))


CALLS = [
    # the chip's kernel and basis on a ragged frame, then a smaller input with
    # fewer families, a smaller kernel and spatial degree 1
    dict(H=300, W=520, h=10, sigmas=(0.7, 1.5, 2.0), degrees=(6, 4, 2), d_s=2, seed=31),
    dict(H=70, W=133, h=5, sigmas=(1.1, 2.2), degrees=(3, 1), d_s=1, seed=32),
]


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
def test_noalloc_matches_plan_entry_point(svc, precision):
    for c in CALLS:
        R = synth.star_field(c["H"], c["W"], max(1, c["H"] * c["W"] // 300), seed=c["seed"])
        I = synth.star_field(c["H"], c["W"], max(1, c["H"] * c["W"] // 300), seed=c["seed"] + 1)
        N = synth.n_basis(c["degrees"])
        a = synth.coefficients(N, synth.n_spatial(c["d_s"]), 0, seed=c["seed"])
        Rd, Id, ad = to_dev(R), to_dev(I), to_dev(a)
        say("noalloc", precision, (c["H"], c["W"], c["h"], N, c["d_s"]))
        D0 = noalloc(svc, Rd, Id, ad, c["h"], c["sigmas"], c["degrees"], c["d_s"], precision, synth.SKY_LEVEL)
        D1 = with_plan(svc, Rd, Id, ad, c["h"], c["sigmas"], c["degrees"], c["d_s"], precision, synth.SKY_LEVEL)
        mx, rms = err_stats(D0, D1)
        say("  max |dD| %.3e rms %.3e, identical %.4f" % (mx, rms, np.mean(D0 == D1)))
        assert np.all(np.isfinite(D0))
        assert mx <= 1e-2 * TOL_MFMA
