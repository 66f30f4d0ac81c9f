"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, never against the oracle's own formulas.

Each test names the passage or the mathematical fact it relies on:

* closed forms of the Gaussian basis (normalisation, parity, second moment);
* the impulse response of a convolution (orientation of the kernel and the
  pixel at which it is evaluated);
* a delta kernel gives the identity;
* a spatially constant kernel is an ordinary convolution (a library routine),
  as the paper's Sec. 2 remarks when it explains why FFTs do not apply to the
  varying case;
* an exact regrouping of Eq. 2 evaluated by FFT;
* linearity of Eq. 1 - Eq. 2 in R and in a;
* an explicit operator matrix on 8x8 images;
* adjoint identities and exact finite differences of a quadratic loss;
* the least-squares fit recovers noiseless coefficients.
"""

import math

import numpy as np
import pytest
from scipy.signal import convolve2d

import synth

C0 = synth.WORKLOADS["c0"]
C1 = synth.WORKLOADS["c1"]


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- basis ----

def test_counts_match_workloads(orc):
    # 3 Gaussians with degrees (4,2,0) -> 15+6+1 bases; (6,4,2) -> 28+15+6.
    assert orc.n_basis([4, 2, 0]) == 22
    assert orc.n_basis([6, 4, 2]) == 49
    # Eq. 3 has six terms for the second order; 10 and 15 for orders 3 and 4.
    assert [orc.n_spatial(d) for d in (0, 1, 2, 3, 4)] == [1, 3, 6, 10, 15]
    assert orc.basis(7, C0.sigmas, C0.degrees).shape == (22, 15, 15)


def test_basis_unit_l1_and_gaussian_profile(orc):
    h = 10
    B = orc.basis(h, (1.5,), (0,))[0]
    assert abs(np.abs(B).sum() - 1.0) < 1e-14
    # ratio to the centre is exp(-(u^2+v^2) / (2 sigma^2)), written with math.exp
    for (u, v) in [(1, 0), (0, 1), (3, -2), (-7, 5), (10, 10)]:
        want = math.exp(-(u * u + v * v) / (2 * 1.5 ** 2))
        got = B[v + h, u + h] / B[h, h]
        assert abs(got - want) < 1e-13 * max(1.0, want)


def test_basis_second_moment_is_sigma_squared(orc):
    # For a sampled Gaussian with sigma >= 1 the discrete variance equals
    # sigma^2 to ~1e-8 (Poisson summation); a wrong factor in the exponent
    # (sigma vs 2 sigma^2) would be off by a factor of 2 or 4.
    h = 15
    for s in (1.5, 2.0):
        B = orc.basis(h, (s,), (0,))[0]
        u = np.arange(-h, h + 1)
        var_x = (B.sum(axis=0) * u ** 2).sum() / B.sum()
        var_y = (B.sum(axis=1) * u ** 2).sum() / B.sum()
        assert abs(var_x - s * s) < 1e-6 and abs(var_y - s * s) < 1e-6


def test_basis_order_and_parity(orc):
    # Degree-2 Gaussian lists (i,j) = (0,0),(1,0),(0,1),(2,0),(1,1),(0,2) for
    # u^i v^j (u along columns, v along rows).  Parity under u -> -u is
    # (-1)^i and under v -> -v is (-1)^j.
    h = 7
    B = orc.basis(h, (2.0,), (2,))
    ij = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    for n, (i, j) in enumerate(ij):
        b = B[n]
        assert np.allclose(b[:, ::-1], (-1) ** i * b, atol=1e-16)   # u -> -u
        assert np.allclose(b[::-1, :], (-1) ** j * b, atol=1e-16)   # v -> -v
        # the monomial factor: b(u,v) / b00(u,v) is proportional to u^i v^j
        g = B[0]
        u = np.arange(-h, h + 1)[None, :]
        v = np.arange(-h, h + 1)[:, None]
        mono = (u ** i) * (v ** j) * g
        scale = np.abs(mono).sum()
        assert np.allclose(b, mono / scale, atol=1e-15)


def test_delta_basis(orc):
    B = orc.basis(3, (0.0,), (0,))
    assert B.shape == (1, 7, 7)
    assert B[0, 3, 3] == 1.0 and np.count_nonzero(B) == 1
    with pytest.raises(ValueError):
        orc.basis(3, (0.0,), (1,))


# ----------------------------------------------------- convolution pins ----

def test_delta_kernel_gives_identity(orc):
    # A delta basis with coefficient 1 makes K the identity: D + I = R exactly.
    R = synth.star_field(64, 80, 20, seed=3).astype(np.float64)
    I = synth.star_field(64, 80, 20, seed=4).astype(np.float64)
    B = orc.basis(5, (0.0,), (0,))
    a = np.zeros((1, 6)); a[0, 0] = 1.0
    D = orc.difference(R, I, 5, B, 2, a)
    assert np.array_equal(D + I, R)


def test_impulse_response_orientation_and_evaluation_pixel(orc):
    # R = unit impulse at (xc, yc): C(x, y) = K(x, y)[x - xc, y - yc].
    # With the odd basis u*G (n=1) and coefficient a[1] = (0, 1, 0) (the xh
    # term), C(x, y) = xh(x) * B1(x - xc, y - yc): the kernel is evaluated at
    # the output pixel, and true convolution puts the positive lobe at x > xc.
    H, W, h, s = 33, 41, 6, 1.5
    xc, yc = 17, 20
    R = np.zeros((H, W)); R[yc, xc] = 1.0
    B = orc.basis(h, (s,), (1,))
    a = np.zeros((3, 3)); a[1, 1] = 1.0        # basis u*G times xh
    C = orc.convolve(R, h, B, 1, a)
    uu = np.arange(-h, h + 1)
    norm = sum(abs(u) * math.exp(-(u * u + v * v) / (2 * s * s)) for u in uu for v in uu)
    for (x, y) in [(xc + 1, yc), (xc - 1, yc), (xc + 3, yc - 2), (xc - 5, yc + 4), (xc, yc)]:
        u, v = x - xc, y - yc
        xh = 2.0 * x / (W - 1) - 1.0
        want = xh * u * math.exp(-(u * u + v * v) / (2 * s * s)) / norm
        assert abs(C[y, x] - want) < 1e-15
    assert C[yc, xc + 1] * (2.0 * (xc + 1) / (W - 1) - 1.0) > 0
    # outside the kernel footprint nothing arrives
    assert C[yc, xc + h + 1] == 0.0 and C[yc + h + 1, xc] == 0.0


def test_linear_ramp_coordinates_and_frame(orc):
    # Delta basis, degree-1 spatial terms, R = 1: C = a0 + a1 xh + a2 yh with
    # xh = 2x/(Wf-1)-1 over the full frame; a crop uses frame coordinates.
    H, W = 9, 13
    B = orc.basis(2, (0.0,), (0,))
    a = np.array([[0.25, 1.5, -0.75]])
    R = np.ones((H, W))
    C = orc.convolve(R, 2, B, 1, a)
    assert abs(C[0, 0] - (0.25 - 1.5 + 0.75)) < 1e-15
    assert abs(C[H - 1, W - 1] - (0.25 + 1.5 - 0.75)) < 1e-15
    assert abs(C[0, W - 1] - (0.25 + 1.5 + 0.75)) < 1e-15
    # crop of a 100 x 200 frame at (x0, y0) = (50, 30)
    Cc = orc.convolve(R, 2, B, 1, a, frame=(50, 30, 200, 100))
    for (x, y) in [(0, 0), (12, 8), (5, 3)]:
        xh = 2.0 * (x + 50) / 199 - 1.0
        yh = 2.0 * (y + 30) / 99 - 1.0
        assert abs(Cc[y, x] - (0.25 + 1.5 * xh - 0.75 * yh)) < 1e-14


def test_constant_coefficients_equal_library_convolution(orc):
    # Spatial degree 0 (or only m = 0 nonzero) is an ordinary convolution:
    # scipy.signal.convolve2d 'same' with zero fill is the reference.
    R, _ = synth.workload_inputs(C0)
    R = R[:96, :112].astype(np.float64)
    B = orc.basis(7, C0.sigmas, C0.degrees)
    a = rng(1).uniform(-0.05, 0.05, size=(22, 1)); a[15, 0] = 1.0
    K = np.tensordot(a[:, 0], B, axes=(0, 0))
    want = convolve2d(R, K, mode="same", boundary="fill", fillvalue=0.0)
    got = orc.convolve(R, 7, B, 0, a)
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
    a6 = np.zeros((22, 6)); a6[:, 0] = a[:, 0]
    got6 = orc.convolve(R, 7, B, 2, a6)
    assert np.max(np.abs(got6 - want)) < 1e-10 * np.max(np.abs(want))


@pytest.mark.parametrize("case", ["c0_full", "c0_crop_frame", "c1_ragged"])
def test_regrouped_fft_identity(orc, case):
    # Eq. 2 regrouped as sum_m P_m (R (x) sum_n a_nm B_n), evaluated by FFT,
    # must equal the per-pixel direct form to rounding.
    if case == "c0_full":
        wl, R, a = C0, *synth.workload_inputs(C0)
        frame = None
    elif case == "c0_crop_frame":
        wl = C0
        R, a = synth.workload_inputs(C0)
        R = R[40:140, 30:190]
        frame = (30, 40, 256, 256)
    else:
        wl = C1
        R = synth.star_field(100, 141, 60, seed=7)
        a = synth.coefficients(49, 6, 28, seed=7)
        frame = (1000, 500, 4096, 2048)
    B = orc.basis(wl.half_width, wl.sigmas, wl.degrees)
    Cd = orc.convolve(R, wl.half_width, B, wl.spatial_degree, a, frame=frame)
    Cf = orc.convolve_fft(R, wl.half_width, B, wl.spatial_degree, a, frame=frame)
    assert np.max(np.abs(Cd - Cf)) < 1e-12 * np.max(np.abs(Cd))


def test_linearity(orc):
    h, d_s = 4, 2
    B = orc.basis(h, (0.7, 1.5), (2, 1))
    N = B.shape[0]
    r = rng(2)
    R1, R2 = r.normal(size=(30, 37)), r.normal(size=(30, 37))
    a1, a2 = r.normal(size=(N, 6)), r.normal(size=(N, 6))
    al, be = 0.7, -1.3
    lhs = orc.convolve(al * R1 + be * R2, h, B, d_s, a1)
    rhs = al * orc.convolve(R1, h, B, d_s, a1) + be * orc.convolve(R2, h, B, d_s, a1)
    assert np.max(np.abs(lhs - rhs)) < 1e-12
    lhs = orc.convolve(R1, h, B, d_s, al * a1 + be * a2)
    rhs = al * orc.convolve(R1, h, B, d_s, a1) + be * orc.convolve(R1, h, B, d_s, a2)
    assert np.max(np.abs(lhs - rhs)) < 1e-12


@pytest.mark.parametrize("h", [1, 4, 5])
def test_brute_force_operator_8x8(orc, h):
    # Explicit 64x64 operator A[p, q] = K(p)[p - q] (zero padding implied by
    # leaving out-of-array q absent); D = A vec(R) - vec(I).  With h >= 4
    # every pixel of an 8x8 image sees the border.
    H = W = 8
    B = orc.basis(h, (0.7, 1.5), (2, 1))
    N = B.shape[0]
    r = rng(10 + h)
    a = r.normal(size=(N, 6))
    R = r.normal(size=(H, W))
    I = r.normal(size=(H, W))
    A = np.zeros((H * W, H * W))
    for py in range(H):
        for px in range(W):
            K = orc.kernel_at(px, py, h, B, 2, a, (0, 0, W, H))
            for qy in range(H):
                for qx in range(W):
                    u, v = px - qx, py - qy
                    if abs(u) <= h and abs(v) <= h:
                        A[py * W + px, qy * W + qx] = K[v + h, u + h]
    want = (A @ R.ravel() - I.ravel()).reshape(H, W)
    got = orc.difference(R, I, h, B, 2, a)
    assert np.max(np.abs(got - want)) < 1e-13


def test_convolve_at_matches_full(orc):
    R, a = synth.workload_inputs(C0)
    B = orc.basis(7, C0.sigmas, C0.degrees)
    C = orc.convolve(R, 7, B, 2, a)
    xs = np.array([0, 1, 7, 128, 254, 255, 3])
    ys = np.array([0, 255, 7, 128, 3, 255, 200])
    assert np.array_equal(orc.convolve_at(R, 7, B, 2, a, xs, ys), C[ys, xs])


# ------------------------------------------------------------ adjoints ----

def _small_problem(seed=5, H=24, W=29, h=4, d_s=2):
    B_spec = ((0.7, 1.5), (2, 1))
    r = rng(seed)
    R = r.normal(size=(H, W)) * 10 + 100
    I = r.normal(size=(H, W)) * 10 + 100
    return R, I, h, B_spec, d_s, r


def test_adjoint_dot_products(orc):
    # <J_R v, w> = <v, J_R^T w> and <J_a b, w> = <b, J_a^T w>, with J the
    # Jacobians of C = R (x) K(a) (C is bilinear in R and a).
    R, I, h, spec, d_s, r = _small_problem()
    B = orc.basis(h, *spec)
    N, M = B.shape[0], 6
    a = r.normal(size=(N, M))
    v = r.normal(size=R.shape)
    w = r.normal(size=R.shape)
    lhs = np.sum(orc.convolve(v, h, B, d_s, a) * w)
    rhs = np.sum(v * orc.grad_R(R.shape, h, B, d_s, a, w))
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))
    b = r.normal(size=(N, M))
    lhs = np.sum(orc.convolve(R, h, B, d_s, b) * w)
    rhs = np.sum(b * orc.grad_a(R, h, B, d_s, w))
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


def test_finite_differences_are_exact_for_quadratic_loss(orc):
    # L = sum_Omega D^2 is quadratic in a and in R, so central differences
    # with step 1e-3 equal the gradient up to rounding.
    R, I, h, spec, d_s, r = _small_problem(seed=6)
    B = orc.basis(h, *spec)
    N, M = B.shape[0], 6
    a = r.normal(size=(N, M)) * 0.1
    omega = orc.interior_mask(*R.shape, h)

    def loss(R_, a_):
        D = orc.difference(R_, I, h, B, d_s, a_)
        return np.sum(D[omega] ** 2)

    D = orc.difference(R, I, h, B, d_s, a)
    G = 2.0 * D * omega
    ga = orc.grad_a(R, h, B, d_s, G)
    gR = orc.grad_R(R.shape, h, B, d_s, a, G)
    step = 1e-3
    for (n, m) in [(0, 0), (3, 2), (N - 1, M - 1), (5, 4)]:
        e = np.zeros_like(a); e[n, m] = step
        fd = (loss(R, a + e) - loss(R, a - e)) / (2 * step)
        assert abs(fd - ga[n, m]) < 1e-7 * max(1.0, abs(ga).max())
    for (y, x) in [(0, 0), (12, 14), (23, 28), (3, 20)]:
        e = np.zeros_like(R); e[y, x] = step
        fd = (loss(R + e, a) - loss(R - e, a)) / (2 * step)
        assert abs(fd - gR[y, x]) < 1e-7 * max(1.0, abs(gR).max())


# ----------------------------------------------------------------- fit ----

def test_cholesky_solve_matches_library(orc):
    r = rng(8)
    X = r.normal(size=(40, 30))
    A = X.T @ X + 0.1 * np.eye(30)
    b = r.normal(size=30)
    x = orc.cholesky_solve(A, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    bad = A.copy(); bad[3, 3] = -1.0
    with pytest.raises(np.linalg.LinAlgError):
        orc.cholesky_solve(bad, b)


def test_normal_equations_recover_noiseless_coefficients(orc):
    # I = R (x) K(a*) exactly -> the least-squares minimiser over the
    # interior is a* (Phi has full rank for a textured R).
    R, _, h, spec, d_s, r = _small_problem(seed=9, H=40, W=44)
    B = orc.basis(h, *spec)
    N, M = B.shape[0], 6
    a_star = r.normal(size=(N, M)) * 0.1
    I = orc.convolve(R, h, B, d_s, a_star)
    JtJ, rhs = orc.normal_equations(R, I, h, B, d_s)
    assert np.allclose(JtJ, JtJ.T, rtol=0, atol=1e-9 * np.abs(JtJ).max())
    assert np.linalg.eigvalsh(JtJ).min() > 0
    a_fit = orc.fit_least_squares(R, I, h, B, d_s)
    assert np.max(np.abs(a_fit - a_star)) < 1e-6
    # the gradient of the interior loss is 2 (JtJ a - rhs)
    omega = orc.interior_mask(*R.shape, h)
    a0 = r.normal(size=(N, M)) * 0.1
    G = 2.0 * orc.difference(R, I, h, B, d_s, a0) * omega
    ga = orc.grad_a(R, h, B, d_s, G)
    assert np.allclose(ga.ravel(), 2.0 * (JtJ @ a0.ravel() - rhs), rtol=1e-9,
                       atol=1e-9 * np.abs(ga).max())


# ------------------------------------------------ Dirac delta basis ----

def test_dfb_basis_is_one_impulse_per_kernel_pixel(orc):
    # the delta basis has one basis function per kernel pixel (Sec. 2)
    for h in (0, 1, 3):
        B = orc.basis_dfb(h)
        k = 2 * h + 1
        assert B.shape == (k * k, k, k)
        assert np.array_equal(B.reshape(k * k, k * k), np.eye(k * k))


def test_dfb_impulse_response_is_the_coefficient_polynomial(orc):
    # R = unit impulse at (xc, yc): C(x, y) = K(x,y)[x - xc, y - yc]
    #   = sum_m a[n][m] P_m(x, y) with n the kernel pixel (x - xc, y - yc);
    # degree-1 terms written out: a0 + a1 xh + a2 yh
    H, W, h = 21, 23, 3
    xc, yc = 11, 9
    k = 2 * h + 1
    r = np.random.default_rng(12)
    a = r.normal(size=(k * k, 3))
    R = np.zeros((H, W)); R[yc, xc] = 1.0
    C = orc.convolve(R, h, orc.basis_dfb(h), 1, a)
    for (x, y) in [(xc, yc), (xc + 3, yc - 2), (xc - 1, yc + 3), (xc - 3, yc - 3)]:
        u, v = x - xc, y - yc
        n = (v + h) * k + (u + h)
        xh, yh = 2.0 * x / (W - 1) - 1.0, 2.0 * y / (H - 1) - 1.0
        assert abs(C[y, x] - (a[n, 0] + a[n, 1] * xh + a[n, 2] * yh)) < 1e-14
    assert C[yc, xc + h + 1] == 0.0


def test_dfb_regrouped_fft_identity(orc):
    # the paper's own case: 7 x 7 delta basis, second-order polynomial
    r = np.random.default_rng(13)
    R = synth.star_field(90, 130, 40, seed=13)
    a = r.uniform(-0.05, 0.05, size=(49, 6)); a[24, 0] = 1.0
    B = orc.basis_dfb(3)
    Cd = orc.convolve(R, 3, B, 2, a, frame=(100, 200, 4868, 4846))
    Cf = orc.convolve_fft(R, 3, B, 2, a, frame=(100, 200, 4868, 4846))
    assert np.max(np.abs(Cd - Cf)) < 1e-12 * np.max(np.abs(Cd))
