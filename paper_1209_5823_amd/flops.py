"""Operation and byte counts of the method, for roofline reporting.

Two counts are kept apart:

* the paper's own cost model (Sec. 3): 20 L^2 + 1 FLOP per pixel for the
  Dirac delta basis and N L^2 + 2 L^2 + 18 N + 1 for N Gaussian bases, with an
  L x L kernel;
* the algorithmic count of the per-pixel-coefficient form used here, with a
  fused multiply-add counted as 2 FLOP:
  2 N k^2 (basis responses) + 2 N M (coefficients c_n) + 2 N (dot with c)
  + 1 (subtraction of I).

The minimum HBM traffic of D = (R (x) K) - I is one read of R and I and one
write of D: 12 bytes per pixel in float32.
"""

PAN_STARRS_TILE = (4846, 4868)
PAN_STARRS_TILES = 60


def paper_flops_dfb(L):
    """Paper's Dirac-delta-basis count per pixel (Sec. 3)."""
    return 20 * L * L + 1


def paper_flops_gfb(N, L):
    """Paper's Gaussian-basis count per pixel (Sec. 3)."""
    return N * L * L + 2 * L * L + 18 * N + 1


def flops_per_pixel(N, M, k):
    """Algorithmic FLOP per pixel of the per-pixel-coefficient form."""
    return 2 * N * k * k + 2 * N * M + 2 * N + 1


def regrouped_flops_per_pixel(M, k):
    """FLOP per pixel of the regrouped form sum_m P_m (R (x) Kt_m) - I."""
    return 2 * M * k * k + 2 * M + 1


def executed_flops_per_pixel(n_filters_padded, taps_padded, passes=1):
    """MFMA FLOP actually issued per pixel by a padded contraction."""
    return 2 * n_filters_padded * taps_padded * passes


BYTES_PER_PIXEL = 12          # R in, I in, D out (float32)
BYTES_PER_PIXEL_FORWARD = 8   # R in, C out


def separable_unfolded_flops_per_pixel(degrees, M, k):
    """FLOP per pixel of the separable Gaussian-basis form taken tap by tap: a
    row pass with the (d_g + 1) one-dimensional factors of each family, a
    column pass per basis, then the coefficients, the dot with c and the
    subtraction."""
    n_factors = sum(d + 1 for d in degrees)
    N = sum((d + 1) * (d + 2) // 2 for d in degrees)
    return 2 * n_factors * k + 2 * N * k + 2 * N * M + 2 * N + 1


def separable_flops_per_pixel(degrees, M, k):
    """FLOP per pixel of the separable Gaussian-basis form with the symmetric
    fold.  A factor is even or odd, f_e(-w) = (-1)^e f_e(w), and f_e(0) = 0
    for e >= 1, so applying the factors e = 0..J-1 to one window costs h adds
    per parity present (the pair sums x[-w] + x[w], or differences) and, per
    factor, h FMAs, plus one FMA for the centre tap of f_0.  Windows: one per
    family in the row pass (J = d + 1), one per row factor i in the column
    pass (J = d - i + 1).  Then 2 N M + 2 N + 1 as in the other forms."""
    h = (k - 1) // 2

    def window(J):
        adds = h * min(J, 2)
        fmas = J * h + 1
        return adds + 2 * fmas

    row = sum(window(d + 1) for d in degrees)
    col = sum(window(d - i + 1) for d in degrees for i in range(d + 1))
    N = sum((d + 1) * (d + 2) // 2 for d in degrees)
    return row + col + 2 * N * M + 2 * N + 1


def separable_mma_executed_flops_per_pixel(degrees, passes, tile=64, row_pass_rows=96, window=64):
    """Matrix-core FLOP issued per output pixel by the Toeplitz form of the
    separable passes: every one-dimensional pass is a product with a
    `window`-long reduction (16 + 2h samples padded to two 32-long chunks), the
    row pass covers `row_pass_rows` staged rows per `tile` output rows, and
    each product is issued `passes` times (the hi/lo split terms)."""
    n_factors = sum(d + 1 for d in degrees)
    N = sum((d + 1) * (d + 2) // 2 for d in degrees)
    row = n_factors * window * 2 * passes * row_pass_rows / tile
    col = N * window * 2 * passes
    return int(round(row + col))


def separable_regrouped_flops_per_pixel(degrees, M, k):
    """FLOP per pixel of the regrouped separable form taken tap by tap: a row
    pass per row factor (sum_g (d_g + 1) of them), a column pass per row
    factor and spatial term with the per-call filters
    g_{r,m} = sum_j a[n(r,j)][m] f_j, then sum_m P_m Z_m and the subtraction."""
    n_factors = sum(d + 1 for d in degrees)
    return 2 * n_factors * k + 2 * n_factors * M * k + 2 * M + 1


def separable_regrouped_executed_flops_per_pixel(degrees, M, passes, tile_rows=64, row_blocks=6):
    """Matrix-core FLOP issued per output pixel by the regrouped separable
    kernel: per 16-column strip of `tile_rows` rows, the row pass takes
    `row_blocks` 16-row blocks x 2 eight-column groups per pair of row factors
    and the column pass 8 output blocks of 8 rows per row factor and pair of
    spatial terms, each product of 16 x 16 x 32 (16384 FLOP) issued `passes`
    times."""
    n_factors = sum(d + 1 for d in degrees)
    pairs = (n_factors + 1) // 2
    mpairs = (M + 1) // 2
    per_strip = (pairs * row_blocks * 2 + n_factors * mpairs * (tile_rows // 8)) * passes * 16384
    return int(round(per_strip / (16 * tile_rows)))
