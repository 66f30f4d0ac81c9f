"""GPU tests of the streamed tile pipeline (svconv_pipeline_*): host-resident
tiles copied in, differenced and copied back on three streams.  Each tile's
D must equal, bit for bit, what svconv_difference gives for the same inputs
on the device (the same kernels run), and one tile is checked against the
FP64 oracle."""

import numpy as np
import pytest

import synth
from tests.helpers import TOL_FP32, TOL_MFMA, say, to_dev, to_host, err_stats

pytestmark = pytest.mark.gpu

C0 = synth.WORKLOADS["c0"]


def tiles(n, H, W, n_basis, n_spatial, const, seed):
    R = [synth.star_field(H, W, 60, seed=seed + t) for t in range(n)]
    I = [synth.star_field(H, W, 60, seed=seed + 100 + t) for t in range(n)]
    a = [synth.coefficients(n_basis, n_spatial, const, seed=seed + t) for t in range(n)]
    return R, I, a


def device_differences(plan, R, I, a):
    return [to_host(plan.difference(to_dev(r), to_dev(i), to_dev(c))) for r, i, c in zip(R, I, a)]


@pytest.mark.parametrize("depth,pinned,form", [(2, True, "basis"), (3, False, "basis"),
                                              (1, True, "basis"), (2, True, "separable")])
def test_pipeline_gaussian_basis(svc, orc, depth, pinned, form):
    H, W = 200, 232
    n = 5
    R, I, a = tiles(n, H, W, C0.n_basis, C0.n_spatial, C0.const_basis, seed=40)
    say("pipeline gaussian depth", depth, "pinned", pinned, form)
    with svc.Plan(H, W, C0.half_width, C0.sigmas, C0.degrees, C0.spatial_degree,
                  pedestal=synth.SKY_LEVEL, form=form) as plan:
        want = device_differences(plan, R, I, a)
        if pinned:
            Rh = [svc.pinned_empty((H, W)) for _ in range(n)]
            Ih = [svc.pinned_empty((H, W)) for _ in range(n)]
            Dh = [svc.pinned_empty((H, W)) for _ in range(n)]
            for t in range(n):
                Rh[t].numpy()[:] = R[t]
                Ih[t].numpy()[:] = I[t]
        else:
            Rh, Ih = R, I
            Dh = [np.full((H, W), np.nan, np.float32) for _ in range(n)]
        with svc.Pipeline(plan, depth=depth) as pipe:
            pipe.run(Rh, Ih, a, Dh)
            got = [np.asarray(d.numpy() if hasattr(d, "numpy") else d) for d in Dh]
            for t in range(n):
                assert np.array_equal(got[t], want[t]), t
            # a second run on the same pipeline, tiles in reverse order
            Dh2 = [np.empty((H, W), np.float32) for _ in range(n)]
            pipe.run(R[::-1], I[::-1], a[::-1], Dh2)
            for t in range(n):
                assert np.array_equal(Dh2[t], want[n - 1 - t]), t
    Dref = orc.difference(R[2], I[2], C0.half_width,
                          orc.basis(C0.half_width, C0.sigmas, C0.degrees), C0.spatial_degree, a[2])
    mx, _ = err_stats(got[2], Dref)
    say("  tile 2 vs oracle max %.3e" % mx)
    assert mx <= TOL_FP32


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_pipeline_dfb_regrouped_per_tile_coefficients(svc, orc, precision):
    # the regrouped form rebuilds its filters from each tile's a on the
    # compute stream: every tile must see its own coefficients
    H, W, h, d_s = 150, 170, 3, 2
    k = 2 * h + 1
    n = 7
    R, I, a = tiles(n, H, W, k * k, synth.n_spatial(d_s), (k * k) // 2, seed=7)
    say("pipeline dfb", precision)
    with svc.Plan.dfb(H, W, h, d_s, precision=precision, pedestal=synth.SKY_LEVEL) as plan:
        want = device_differences(plan, R, I, a)
        D = [I[t].copy() for t in range(n)]     # D aliases I
        with svc.Pipeline(plan, depth=2) as pipe:
            pipe.run(R, D, a, D)
            pipe.run([], [], [], [])
    for t in range(n):
        assert np.array_equal(D[t], want[t]), t
    Dref = orc.difference(R[5], I[5], h, orc.basis_dfb(h), d_s, a[5])
    mx, _ = err_stats(D[5], Dref)
    assert mx <= (TOL_FP32 if precision == "fp32" else TOL_MFMA)


def test_pipeline_rejects_wrong_shapes(svc):
    with svc.Plan(64, 64, 2, (1.0,), (1,), 1) as plan:
        with svc.Pipeline(plan, depth=2) as pipe:
            good = np.zeros((64, 64), np.float32)
            a = np.zeros((plan.n_basis, plan.n_spatial), np.float32)
            with pytest.raises(ValueError):
                pipe.run([np.zeros((64, 63), np.float32)], [good], [a], [good])
            with pytest.raises(TypeError):
                pipe.run([good.astype(np.float64)], [good], [a], [good])
            with pytest.raises(ValueError):
                pipe.run([good, good], [good], [a], [good])


def test_host_alloc_roundtrip(svc):
    import ctypes
    from paper_1209_5823_amd import _lib
    lib = _lib.load()
    p = ctypes.c_void_p()
    assert lib.svconv_host_alloc(1 << 20, ctypes.byref(p)) == _lib.OK
    assert p.value
    buf = (ctypes.c_float * (1 << 18)).from_address(p.value)
    buf[0], buf[-1] = 1.5, -2.5
    assert buf[0] == 1.5 and buf[-1] == -2.5
    assert lib.svconv_host_free(p) == _lib.OK
