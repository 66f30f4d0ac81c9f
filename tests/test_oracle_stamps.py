"""Pins of the oracle's star-stamp selection and of the least-squares fit
with a differential background polynomial (OIS on isolated stars, Sec. 2).

The stamp fixtures are built by hand, so the expected centres follow from
the definition by construction: an isolated bright star, a close pair of
comparable stars, a bright star with a faint companion, a star inside the
edge margin, a star below the threshold and a two-pixel plateau."""

import numpy as np
import pytest

import synth

SKY = 1000.0


def gauss_star(img, x, y, amp, sigma=1.1):
    H, W = img.shape
    yy, xx = np.mgrid[0:H, 0:W]
    img += amp * np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / (2 * sigma * sigma))


@pytest.fixture(scope="module")
def field():
    img = np.full((96, 140), SKY)
    gauss_star(img, 20, 20, 5000)      # A: isolated, bright -> centre
    gauss_star(img, 60, 20, 5000)      # B: 4.5 px from C, C is comparable
    gauss_star(img, 64, 22, 3000)      # C
    gauss_star(img, 100, 20, 5000)     # D: bright, faint companion E -> centre
    gauss_star(img, 100, 26, 200)      # E: below frac * (D - sky)
    gauss_star(img, 3, 50, 5000)       # F: inside the edge margin
    gauss_star(img, 40, 60, 500)       # G: below the threshold
    img[80, 80] = img[80, 81] = SKY + 4000   # plateau: no strict maximum
    gauss_star(img, 120, 70, 8000)     # J: isolated, bright -> centre
    return img.astype(np.float32)


def test_stamp_centres_hand_built_field(orc, field):
    c = orc.stamp_centres(field, SKY, threshold=1000.0, frac=0.1, r_iso=6, margin=8)
    assert c == [(20, 20), (100, 20), (120, 70)]


def test_stamp_centres_isolation_radius_and_fraction(orc, field):
    # with a 3-pixel isolation window the pair B, C no longer interferes
    # (C is at offset (4, 2) from B): both are centres
    c = orc.stamp_centres(field, SKY, threshold=1000.0, frac=0.1, r_iso=3, margin=8)
    assert (60, 20) in c and (64, 22) in c
    # with frac below E's relative brightness (200 / 5000) D is not isolated
    c = orc.stamp_centres(field, SKY, threshold=1000.0, frac=0.03, r_iso=6, margin=8)
    assert (100, 20) not in c and (20, 20) in c
    # margin 2 admits F
    c = orc.stamp_centres(field, SKY, threshold=1000.0, frac=0.1, r_iso=6, margin=2)
    assert (3, 50) in c


def test_stamp_mask_boxes(orc):
    m = orc.stamp_mask(30, 40, [(5, 5), (20, 10), (39, 29)], 3)
    assert m.dtype == np.uint8
    assert m.sum() == 49 + 49 + 16          # the corner box is clipped to 4 x 4
    assert m[2, 2] == 1 and m[1, 2] == 0 and m[8, 8] == 1 and m[9, 8] == 0
    assert m[26, 36] == 1 and m[25, 36] == 0


def test_design_matrix_kernel_block_matches_normal_equations(orc):
    # the Python spatial-term images and basis responses against the C
    # normal equations, on a cropped frame (the background block aside)
    R = synth.star_field(24, 30, 6, seed=3)
    I = synth.star_field(24, 30, 6, seed=4)
    h, d_s = 2, 2
    B = orc.basis(h, (1.0, 1.6), (2, 0))
    frame = (7, 3, 61, 45)
    Phi, sel = orc.design_matrix_bg(R, h, B, d_s, frame=frame)
    JtJ, rhs = orc.normal_equations(R, I, h, B, d_s, frame=frame)
    NM = JtJ.shape[0]
    G = Phi.T @ Phi
    assert np.allclose(G[:NM, :NM], JtJ, rtol=1e-12, atol=1e-9 * np.abs(JtJ).max())
    assert np.allclose((Phi.T @ I.astype(np.float64)[sel])[:NM], rhs, rtol=1e-12,
                       atol=1e-9 * np.abs(rhs).max())


def test_background_fit_recovers_an_exact_model(orc):
    # I = R (x) K(a*) + bg(b*) exactly: the least-squares solution is (a*, b*)
    H, W, h, d_s = 40, 44, 3, 2
    R = synth.star_field(H, W, 12, seed=9).astype(np.float64)
    B = orc.basis(h, (0.9, 1.7), (2, 1))
    N, M = B.shape[0], orc.n_spatial(d_s)
    r = np.random.default_rng(5)
    a = r.uniform(-0.05, 0.05, (N, M))
    a[0, 0] = 1.0
    b = np.array([12.0, -3.0, 2.5, 0.8, -1.1, 0.4])
    I = orc.convolve(R, h, B, d_s, a) + orc.background(H, W, d_s, b)
    a_fit, b_fit = orc.fit_least_squares_bg(R, I, h, B, d_s)
    assert np.allclose(a_fit, a, atol=1e-7)
    assert np.allclose(b_fit, b, atol=1e-5)


def test_background_absorbs_a_constant_offset(orc):
    # D = R (x) K + bg - I: adding c to I moves only b_0 (P_0 = 1), by c
    H, W, h, d_s = 32, 36, 2, 1
    R = synth.star_field(H, W, 8, seed=1)
    I = synth.poisson_noise(synth.star_field(H, W, 8, seed=1), seed=2)
    B = orc.basis(h, (1.2,), (2,))
    a1, b1 = orc.fit_least_squares_bg(R, I, h, B, d_s)
    a2, b2 = orc.fit_least_squares_bg(R, I + 37.0, h, B, d_s)
    assert np.allclose(a1, a2, atol=1e-8)
    assert np.allclose(b2 - b1, [37.0, 0.0, 0.0], atol=1e-6)


def test_background_is_the_spatial_polynomial(orc):
    # bg at the four corners of a 5 x 3 frame: xh, yh in {-1, 1}
    b = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    bg = orc.background(3, 5, 2, b)
    for (x, y, xh, yh) in [(0, 0, -1, -1), (4, 0, 1, -1), (0, 2, -1, 1), (4, 2, 1, 1), (2, 1, 0, 0)]:
        want = 1 + 2 * xh + 3 * yh + 4 * xh * xh + 5 * xh * yh + 6 * yh * yh
        assert bg[y, x] == pytest.approx(want, abs=1e-12)
