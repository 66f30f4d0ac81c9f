"""The paper's worked cost-model numbers (Sec. 3), from tests/golden."""

import os

from paper_1209_5823_amd import flops

GOLD = os.path.join(os.path.dirname(__file__), "golden", "flop_model.txt")


def _rows():
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            kind, L, N, per_px, tile_g, image, unit = line.split()
            yield kind, int(L), int(N), int(per_px), float(tile_g), float(image), unit


def test_paper_cost_model_numbers():
    tile = flops.PAN_STARRS_TILE[0] * flops.PAN_STARRS_TILE[1]
    rows = list(_rows())
    assert len(rows) == 2
    for kind, L, N, per_px, tile_g, image, unit in rows:
        got = flops.paper_flops_dfb(L) if kind == "dfb" else flops.paper_flops_gfb(N, L)
        assert got == per_px
        assert round(got * tile / 1e9, 2 if tile_g < 10 else 1) == tile_g
        scale = 1e12 if unit == "TFLOP" else 1e9
        digits = 2 if image < 10 else 0
        assert round(got * tile * flops.PAN_STARRS_TILES / scale, digits) == image


def test_algorithmic_counts_at_workloads():
    # 2 N k^2 + 2 N M + 2 N + 1 with (N, M, k) of the chip and survey workloads
    assert flops.flops_per_pixel(49, 6, 21) == 43905
    assert flops.flops_per_pixel(49, 15, 31) == 95747
    assert flops.flops_per_pixel(22, 6, 15) == 10209


def test_separable_unfolded_count_at_the_chip_workload():
    # 15 row factors (degrees 6, 4, 2) and 49 column passes of 21 taps, then
    # 2 N M + 2 N + 1 for the coefficients, the dot and the subtraction
    assert flops.separable_unfolded_flops_per_pixel((6, 4, 2), 6, 21) == 2 * 15 * 21 + 2 * 49 * 21 + 2 * 49 * 6 + 2 * 49 + 1
    assert flops.separable_unfolded_flops_per_pixel((6, 4, 2), 6, 21) == 3375
    # a single delta family: one factor, one basis
    assert flops.separable_unfolded_flops_per_pixel((0,), 1, 3) == 2 * 3 + 2 * 3 + 2 + 2 + 1


def _folded_by_enumeration(degrees, M, k):
    # every factor application and every window of pair sums counted one by one
    h = (k - 1) // 2
    total = 0
    for d in degrees:
        windows = [list(range(d + 1))] + [list(range(d - i + 1)) for i in range(d + 1)]
        for factors in windows:
            total += h * len({e % 2 for e in factors})          # pair sums / differences
            for e in factors:
                total += 2 * h + (2 if e == 0 else 0)          # h FMAs (+ the centre of f_0)
    N = sum((d + 1) * (d + 2) // 2 for d in degrees)
    return total + 2 * N * M + 2 * N + 1


def test_separable_folded_count():
    for degrees, M, k in (((6, 4, 2), 6, 21), ((6, 4, 2), 10, 31), ((0,), 1, 3), ((9,), 3, 11), ((1, 3), 1, 5)):
        assert flops.separable_flops_per_pixel(degrees, M, k) == _folded_by_enumeration(degrees, M, k)
    # the chip workload: row 366, column 1280, coefficients and dot 687
    assert flops.separable_flops_per_pixel((6, 4, 2), 6, 21) == 2333
    # a fold never costs more than the tap-by-tap count
    for degrees, M, k in (((6, 4, 2), 6, 21), ((0,), 1, 3), ((2,), 1, 3)):
        assert flops.separable_flops_per_pixel(degrees, M, k) <= flops.separable_unfolded_flops_per_pixel(degrees, M, k)


def test_separable_mma_executed_count():
    # 15 factors x 1.5 staged rows per output row x 64-long windows x 2 FLOP x 3 terms,
    # plus 49 bases x 64 x 2 x 3
    assert flops.separable_mma_executed_flops_per_pixel((6, 4, 2), 3) == 15 * 96 * 6 + 49 * 64 * 6
    assert flops.separable_mma_executed_flops_per_pixel((6, 4, 2), 3) == 27456
    assert flops.separable_mma_executed_flops_per_pixel((0,), 1) == 64 * 2 * 96 // 64 + 64 * 2
