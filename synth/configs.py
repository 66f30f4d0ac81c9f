"""Workload descriptions: image sizes, kernel half-width, basis and spatial
specifications and the star-field recipe of each benchmark configuration.

Counting conventions (a reading; the paper cites the Gaussian basis without
giving its formula):

* each Gaussian g of width sigma_g carries the monomials u^i v^j of total
  degree t = 0..d_g, listed by t, then by descending i, so it contributes
  (d_g+1)(d_g+2)/2 basis functions;
* the spatial polynomial of degree d_s has (d_s+1)(d_s+2)/2 terms, listed the
  same way (the paper's second-order case, Eq. 3, has six terms).

Only counts and indices live here, never basis values.
"""

from dataclasses import dataclass, field
from typing import Callable, Tuple


def n_basis(degrees) -> int:
    """Number of basis functions for per-Gaussian polynomial degrees."""
    return int(sum((d + 1) * (d + 2) // 2 for d in degrees))


def n_spatial(d_s: int) -> int:
    """Number of spatial polynomial terms of total degree <= d_s."""
    return (d_s + 1) * (d_s + 2) // 2


def const_basis_index(degrees, g: int) -> int:
    """Index of the degree-0 (pure Gaussian) basis of Gaussian number g."""
    return int(sum((d + 1) * (d + 2) // 2 for d in degrees[:g]))


def _fwhm_const(v):
    return lambda x, y, W, H: v + 0.0 * x


def _fwhm_ramp_x(lo, hi):
    # linear in column index from lo at x=0 to hi at x=W-1
    return lambda x, y, W, H: lo + (hi - lo) * x / max(W - 1, 1)


def _fwhm_diag(lo, hi):
    # linear along the diagonal: lo at (0,0), hi at (W-1,H-1)
    return lambda x, y, W, H: lo + 0.5 * (hi - lo) * (x / max(W - 1, 1) + y / max(H - 1, 1))


@dataclass(frozen=True)
class Workload:
    name: str
    height: int
    width: int
    half_width: int
    sigmas: Tuple[float, ...]
    degrees: Tuple[int, ...]
    spatial_degree: int
    n_stars: int
    fwhm: Callable = field(compare=False, repr=False, default=None)
    seed: int = 0
    const_sigma_index: int = 1      # Gaussian whose constant term carries a = 1
    description: str = ""

    @property
    def k(self) -> int:
        return 2 * self.half_width + 1

    @property
    def n_basis(self) -> int:
        return n_basis(self.degrees)

    @property
    def n_spatial(self) -> int:
        return n_spatial(self.spatial_degree)

    @property
    def const_basis(self) -> int:
        return const_basis_index(self.degrees, self.const_sigma_index)


SIGMAS = (0.7, 1.5, 2.0)

WORKLOADS = {
    # plain method at the size the oracle finishes in well under a second
    "c0": Workload("c0", 256, 256, 7, SIGMAS, (4, 2, 0), 2, 200, _fwhm_const(2.5),
                   description="256x256, 15x15 kernel, 22 bases, spatial degree 2"),
    # one 2048x4096 CCD chip, 21x21 kernel, 49 bases (plain FP32 and MFMA forms)
    "c1": Workload("c1", 2048, 4096, 10, SIGMAS, (6, 4, 2), 2, 20000, _fwhm_ramp_x(2.0, 3.5),
                   description="2048x4096 chip, 21x21 kernel, 49 bases, spatial degree 2"),
    "c2": Workload("c2", 2048, 4096, 10, SIGMAS, (6, 4, 2), 2, 20000, _fwhm_ramp_x(2.0, 3.5),
                   description="2048x4096 chip, 21x21 kernel, 49 bases, spatial degree 2 (MFMA forms)"),
    # differentiation: 4096x4096, 31x31 kernel, spatial degree 3 (490 coefficients)
    "c3": Workload("c3", 4096, 4096, 15, SIGMAS, (6, 4, 2), 3, 40000, _fwhm_ramp_x(2.0, 3.5),
                   description="4096x4096, 31x31 kernel, 49 bases, spatial degree 3"),
    # fit at survey scale: 8192x8192, spatial degree 4 (735 coefficients)
    "c4": Workload("c4", 8192, 8192, 15, SIGMAS, (6, 4, 2), 4, 80000, _fwhm_diag(2.0, 3.5),
                   description="8192x8192, 31x31 kernel, 49 bases, spatial degree 4"),
}
