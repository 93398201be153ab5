"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the solver itself: it only describes the
problems (grid, wavenumber, decomposition) and draws the seeded media, sources
and receivers.  Both sides receive the same numpy arrays from here.

Every workload is a 2-D Helmholtz problem -Lap u - k^2 m u = f on the unit
square sampled at the nodes x = (ix+1) h, y = (iy+1) h, ix, iy in [0, N),
h = 1/(N+1), with m = 1/c^2 (squared slowness).  Arrays are indexed [iy, ix]
(row-major, x fastest), which is also the flat layout the C ABI expects.

The paper's own test case (a sound-soft cylinder meshed with P7 triangles,
Sec. 7) needs an unstructured mesh; these workloads stand in for it with the
same physics on a finite-difference grid: wavenumbers fixed by a number of
points per wavelength, smooth random or layered media, and Gaussian sources.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """A fully specified synthetic problem.

    nx, ny   interior grid size (h = 1/(nx+1) in both directions)
    n1, n2   checkerboard decomposition: n1 columns (x), n2 rows (y)
    ppw      points per wavelength at the reference speed c = 1
    medium   "homogeneous" | "grf" | "layered" | "grf_m"
    seed     medium seed
    sources  list of (x, y) source centres
    """

    name: str
    nx: int
    ny: int
    n1: int
    n2: int
    ppw: float
    medium: str
    seed: int
    sources: tuple
    tol: float = 1e-6
    restart: int = 50

    @property
    def h(self) -> float:
        return 1.0 / (self.nx + 1)

    @property
    def k(self) -> float:
        """Reference wavenumber: ppw grid points per wavelength at c = 1."""
        return 2.0 * math.pi / (self.ppw * self.h)

    @property
    def sub_nx(self) -> int:
        return self.nx // self.n1

    @property
    def sub_ny(self) -> int:
        return self.ny // self.n2


def _standardise(z: np.ndarray) -> np.ndarray:
    return (z - z.mean()) / z.std()


def gaussian_random_field(n: int, h: float, seed: int, corr: float = 0.1) -> np.ndarray:
    """Standardised smooth Gaussian random field on an n x n grid.

    White noise from ``default_rng(seed)`` filtered by a Gaussian kernel whose
    width is the correlation length ``corr`` in grid cells (corr / h).
    """
    from scipy.ndimage import gaussian_filter

    z = np.random.default_rng(seed).standard_normal((n, n))
    z = gaussian_filter(z, sigma=corr / h, mode="reflect")
    return _standardise(z)


def speed_grf(n: int, h: float, seed: int) -> np.ndarray:
    """c(x) = clip(1 + 0.1 z, 0.8, 1.2) for a correlation-0.1 random field z."""
    return np.clip(1.0 + 0.1 * gaussian_random_field(n, h, seed), 0.8, 1.2)


def speed_layered(nx: int, ny: int, seed: int, nlayers: int = 8, smooth_cells: float = 4.0) -> np.ndarray:
    """Horizontal layers: c in [1, 2] drawn per layer, smoothed over a few cells in y."""
    from scipy.ndimage import gaussian_filter1d

    vals = np.random.default_rng(seed).uniform(1.0, 2.0, nlayers)
    h = 1.0 / (nx + 1)
    y = (np.arange(ny) + 1) * h
    layer = np.minimum((y * nlayers).astype(np.int64), nlayers - 1)
    col = vals[layer]
    col = gaussian_filter1d(col, sigma=smooth_cells, mode="nearest")
    return np.repeat(col[:, None], nx, axis=1)


def slowness2(w: Workload) -> np.ndarray:
    """m = 1/c^2 on the [ny, nx] grid (float64)."""
    if w.medium == "homogeneous":
        c = np.ones((w.ny, w.nx))
    elif w.medium == "grf":
        assert w.nx == w.ny
        c = speed_grf(w.nx, w.h, w.seed)
    elif w.medium == "layered":
        c = speed_layered(w.nx, w.ny, w.seed)
    elif w.medium == "grf_m":
        assert w.nx == w.ny
        return np.clip(1.0 + 0.1 * gaussian_random_field(w.nx, w.h, w.seed), 0.8, 1.2)
    elif w.medium == "random_smooth":
        # small-grid test medium: any size, smooth, in [0.8, 1.2]
        rng = np.random.default_rng(w.seed)
        from scipy.ndimage import gaussian_filter

        z = gaussian_filter(rng.standard_normal((w.ny, w.nx)), sigma=max(1.0, w.nx / 10), mode="reflect")
        c = np.clip(1.0 + 0.1 * _standardise(z), 0.8, 1.2)
    else:
        raise ValueError(w.medium)
    return np.ascontiguousarray(1.0 / c**2)


def smoothed_model(m: np.ndarray, width_cells: float = 20.0) -> np.ndarray:
    """Initial model for the gradient workload: m smoothed by a Gaussian of the given width."""
    from scipy.ndimage import gaussian_filter

    return np.ascontiguousarray(gaussian_filter(m, sigma=width_cells, mode="nearest"))


def gaussian_source(nx: int, ny: int, h: float, x0: float, y0: float, width: float | None = None) -> np.ndarray:
    """Unit-mass Gaussian exp(-|x-x0|^2 / (2 s^2)) / (2 pi s^2), s = 2h by default (complex128)."""
    s = 2.0 * h if width is None else width
    x = (np.arange(nx) + 1) * h
    y = (np.arange(ny) + 1) * h
    gx = np.exp(-((x - x0) ** 2) / (2 * s * s))
    gy = np.exp(-((y - y0) ** 2) / (2 * s * s))
    f = np.outer(gy, gx) / (2 * math.pi * s * s)
    return f.astype(np.complex128)


def sources(w: Workload) -> np.ndarray:
    """All sources of a workload, shape [nsrc, ny, nx], complex128."""
    return np.stack([gaussian_source(w.nx, w.ny, w.h, x0, y0) for (x0, y0) in w.sources])


def sources_along_line(nsrc: int, y0: float) -> tuple:
    """nsrc sources evenly spaced along the line y = y0 at x_s = (s + 1/2)/nsrc."""
    return tuple(((s + 0.5) / nsrc, y0) for s in range(nsrc))


def receiver_row(w: Workload, y_rec: float = 0.95) -> np.ndarray:
    """Flat indices of every node on the grid row nearest to y = y_rec (int32)."""
    iy = int(round(y_rec / w.h)) - 1
    return (iy * w.nx + np.arange(w.nx)).astype(np.int32)


def gradient_direction(shape, j: int) -> np.ndarray:
    """Seeded perturbation direction j of a model m for finite-difference checks of dL/dm:
    ``default_rng(100 + j)`` normal draws scaled to max-norm 1 (float64)."""
    d = np.random.default_rng(100 + j).standard_normal(shape)
    return d / np.abs(d).max()


def random_interface_vector(nif: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Seeded complex128 test vector for operator-level parity checks."""
    rng = np.random.default_rng(seed)
    shape = (nif,) if nrhs is None else (nrhs, nif)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex128)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the problems the method is benchmarked on:
# 10 (or 15) points per wavelength, 128^2 or 64^2 subdomains, checkerboards up
# to 16 x 16.
# ---------------------------------------------------------------------------

SMALL = Workload("small_64_2x2_homog", 64, 64, 2, 2, 10.0, "homogeneous", 0, ((0.5, 0.5),), tol=1e-6)
FP64_1024 = Workload("fp64_1024_8x8_grf", 1024, 1024, 8, 8, 10.0, "grf", 0, ((0.5, 0.1),), tol=1e-8)
MIXED_1024 = Workload("mixed_1024_8x8_grf", 1024, 1024, 8, 8, 10.0, "grf", 0, ((0.5, 0.1),), tol=1e-6)
MULTI_2048 = Workload(
    "multi_2048_16x16_layered", 2048, 2048, 16, 16, 15.0, "layered", 1, sources_along_line(64, 0.05), tol=1e-6
)
GRAD_512 = Workload("grad_512_8x8_grf", 512, 512, 8, 8, 10.0, "grf_m", 2, sources_along_line(16, 0.05), tol=1e-12)

WORKLOADS = {w.name: w for w in (SMALL, FP64_1024, MIXED_1024, MULTI_2048, GRAD_512)}


def scaled(w: Workload, nx: int, ny: int | None = None, n1: int | None = None, n2: int | None = None,
           medium: str | None = None, **kw) -> Workload:
    """Same physics (points per wavelength, medium family, source layout) on another grid."""
    ny = nx if ny is None else ny
    return dataclasses.replace(w, name=f"{w.name}@{nx}x{ny}", nx=nx, ny=ny,
                               n1=w.n1 if n1 is None else n1, n2=w.n2 if n2 is None else n2,
                               medium=w.medium if medium is None else medium, **kw)
