"""GPU parity of the hand-written adjoint (dL/da, dL/dR) against the FP64
oracle, central finite differences and adjoint identities, through the C ABI
and through the torch.autograd.Function.

Tolerances come from the float32 arithmetic of the GPU path: every
gradient entry is a sum of products G * P * T (or G * K); its rounding error
is bounded by a small multiple of 2^-24 times the sum of the magnitudes of
its terms, which the oracle evaluates with |G|, |R| and |B|.
"""

import numpy as np
import pytest

import synth
from tests.helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu

C3 = synth.WORKLOADS["c3"]
REL = 2e-5     # multiple of the magnitude sums allowed as rounding error


def crop_case(orc, wl, size=256, seed=0, y0=1900, x0=2100):
    """A size x size crop of the workload's star field, its frame, the
    coefficients a* + U(-0.005, 0.005) and I = float32(Poisson(C(a*)))."""
    R_full, a_star = synth.workload_inputs(wl)
    R = np.ascontiguousarray(R_full[y0:y0 + size, x0:x0 + size])
    frame = (x0, y0, wl.width, wl.height)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    C = orc.convolve(R, wl.half_width, B, wl.spatial_degree, a_star, frame=frame)
    I = synth.poisson_noise(C, seed=seed)
    r = np.random.default_rng(seed + 7)
    a = (a_star + r.uniform(-0.005, 0.005, a_star.shape)).astype(np.float32)
    return R, I, a, B, frame


@pytest.fixture(scope="module")
def c3_crop(orc):
    R, I, a, B, frame = crop_case(orc, C3)
    h, d_s = C3.half_width, C3.spatial_degree
    D = orc.difference(R, I, h, B, d_s, a, frame=frame)
    omega = orc.interior_mask(*R.shape, h)
    G = (2.0 * D * omega).astype(np.float32)
    ga = orc.grad_a(R, h, B, d_s, G, frame=frame)
    gR = orc.grad_R(R.shape, h, B, d_s, a, G, frame=frame)
    # magnitude sums: sum_p |G| |P_m| |T_n| <= sum_p |G| (|B_n| (x) |R|)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G), frame=frame)[:, :1]
    sR = orc.grad_R(R.shape, h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True),
                    np.abs(G), frame=frame)
    return dict(R=R, I=I, a=a, B=B, frame=frame, G=G, ga=ga, gR=gR, sa=sa, sR=sR)


def make_plan(svc, shape, wl, frame=None, precision="fp32"):
    return svc.Plan(shape[0], shape[1], wl.half_width, wl.sigmas, wl.degrees, wl.spatial_degree,
                    precision=precision, frame=frame)


def test_adjoint_vs_oracle_c3_crop(svc, c3_crop):
    c = c3_crop
    say("adjoint c3 crop 256x256")
    with make_plan(svc, c["R"].shape, C3, frame=c["frame"]) as plan:
        gR, ga = plan.backward(to_dev(c["R"]), to_dev(c["a"]), to_dev(c["G"]))
        gR, ga = to_host(gR), to_host(ga)
    ea = np.abs(ga - c["ga"])
    eR = np.abs(gR - c["gR"])
    say("  ga max err %.3e (scale %.3e)  gR max err %.3e (scale %.3e)"
        % (ea.max(), c["sa"].max(), eR.max(), c["sR"].max()))
    assert np.all(ea <= REL * c["sa"] + 1e-9)
    assert np.all(eR <= REL * c["sR"] + 1e-6)


def test_finite_differences_c3_crop(svc, c3_crop):
    # L = sum_Omega D^2 is quadratic: central differences with step 1e-3 are
    # exact up to the rounding of the two forward passes
    import torch
    c = c3_crop
    R, I, a = to_dev(c["R"]), to_dev(c["I"]), c["a"]
    say("finite differences c3 crop")
    with make_plan(svc, c["R"].shape, C3, frame=c["frame"]) as plan:
        def loss(av):
            D = plan.difference(R, I, to_dev(av))
            L, _ = plan.loss_grad(D)
            torch.cuda.synchronize()
            return float(L.item())
        D = plan.difference(R, I, to_dev(a))
        _, G = plan.loss_grad(D)
        _, ga = plan.backward(R, to_dev(a), G, want_gR=False)
        ga = to_host(ga)
        step = 1e-3
        r = np.random.default_rng(3)
        picks = [(28, 0), (0, 0), (48, 9), (10, 3)] + [tuple(x) for x in
                                                       zip(r.integers(0, 49, 4), r.integers(0, 10, 4))]
        for (n, m) in picks:
            ap, am = a.astype(np.float64).copy(), a.astype(np.float64).copy()
            ap[n, m] += step
            am[n, m] -= step
            fd = (loss(ap.astype(np.float32)) - loss(am.astype(np.float32))) / (
                float(np.float32(ap[n, m])) - float(np.float32(am[n, m])))
            say("  (%d,%d) fd %.6e adjoint %.6e" % (n, m, fd, ga[n, m]))
            assert abs(fd - ga[n, m]) <= 2e-3 * np.abs(ga).max()


def test_autograd_function_matches_direct(svc, c3_crop):
    import torch
    c = c3_crop
    say("autograd function")
    with make_plan(svc, c["R"].shape, C3, frame=c["frame"]) as plan:
        R = to_dev(c["R"]).requires_grad_(True)
        I = to_dev(c["I"]).requires_grad_(True)
        a = to_dev(c["a"]).requires_grad_(True)
        D = svc.difference(plan, R, I, a)
        omega = torch.from_numpy(np.ascontiguousarray(
            np.pad(np.ones((256 - 30, 256 - 30), np.float32), 15))).cuda()
        L = (D.double() ** 2 * omega).sum()
        L.backward()
        Dd = plan.difference(R.detach(), I.detach(), a.detach())
        _, G = plan.loss_grad(Dd)
        gR, ga = plan.backward(R.detach(), a.detach(), G)
        torch.cuda.synchronize()
        assert torch.allclose(I.grad, -G, rtol=0, atol=1e-3)
        assert torch.allclose(a.grad.double(), ga, rtol=1e-5, atol=1e-3 * ga.abs().max().item())
        assert torch.allclose(R.grad, gR, rtol=1e-5, atol=1e-5 * gR.abs().max().item())


@pytest.mark.parametrize("shape,h,sig,deg,d_s", [
    ((37, 70), 1, (1.0,), (2,), 1),
    ((8, 8), 4, (0.7, 1.5), (2, 1), 2),
    ((64, 96), 7, (0.7, 1.5, 2.0), (6, 2, 0), 6),
    ((5, 7), 10, (0.7, 1.5, 2.0), (6, 4, 2), 2),
])
def test_adjoint_edge_cases(svc, orc, shape, h, sig, deg, d_s):
    H, W = shape
    R = synth.star_field(H, W, max(1, H * W // 300), seed=H + W)
    G = synth.uniform_image(H, W, seed=H * W, lo=-50, hi=50)
    N = synth.n_basis(deg)
    a = synth.coefficients(N, synth.n_spatial(d_s), 0, seed=h)
    B = orc.basis(h, sig, deg)
    ga_ref = orc.grad_a(R, h, B, d_s, G)
    gR_ref = orc.grad_R(R.shape, h, B, d_s, a, G)
    sa = orc.grad_a(np.abs(R), h, np.abs(B), 0, np.abs(G))[:, :1]
    sR = orc.grad_R(R.shape, h, np.abs(B), 0, np.abs(a).sum(axis=1, keepdims=True), np.abs(G))
    say("adjoint edge", shape, h, N, d_s)
    with svc.Plan(H, W, h, sig, deg, d_s) as plan:
        gR, ga = plan.backward(to_dev(R), to_dev(a), to_dev(G))
        gR, ga = to_host(gR), to_host(ga)
    assert np.all(np.abs(ga - ga_ref) <= REL * sa + 1e-9)
    assert np.all(np.abs(gR - gR_ref) <= REL * sR + 1e-6)


def test_adjoint_identities_full_size_c3(svc):
    # <J_R v, w> = <v, J_R^T w> and <J_a b, w> = <b, J_a^T w> at 4096 x 4096,
    # 31 x 31 kernel, 49 bases, spatial degree 3, both sides on the GPU
    import torch
    wl = C3
    R, a = synth.workload_inputs(wl)
    v = synth.uniform_image(wl.height, wl.width, seed=1)
    w = synth.uniform_image(wl.height, wl.width, seed=2)
    b = synth.coefficients(wl.n_basis, wl.n_spatial, None, seed=3)
    say("adjoint identities 4096x4096")
    with make_plan(svc, R.shape, wl) as plan:
        Rd, ad, vd, wd, bd = map(to_dev, (R, a, v, w, b))
        Jv = plan.forward(vd, ad)
        gR, _ = plan.backward(Rd, ad, wd, want_ga=False)
        lhs = float((Jv.double() * wd.double()).sum())
        rhs = float((vd.double() * gR.double()).sum())
        say("  R: %.9e vs %.9e" % (lhs, rhs))
        assert abs(lhs - rhs) <= 1e-5 * (Jv.double().abs() * wd.double().abs()).sum().item()
        Jb = plan.forward(Rd, bd)
        _, ga = plan.backward(Rd, ad, wd, want_gR=False)
        lhs = float((Jb.double() * wd.double()).sum())
        rhs = float((bd.double() * ga).sum())
        say("  a: %.9e vs %.9e" % (lhs, rhs))
        torch.cuda.synchronize()
        assert abs(lhs - rhs) <= 1e-5 * (Jb.double().abs() * wd.double().abs()).sum().item()
