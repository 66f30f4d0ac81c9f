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
