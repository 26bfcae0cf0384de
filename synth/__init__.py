"""Seeded synthetic inputs: two-phase microstructures and macro strains.

This module is shared by the FP64 oracle, the tests and the benchmark.  It
holds no arithmetic of the solver method itself: it only draws geometry
(binary phase indicators g(x), 1 = inclusion, 0 = matrix, as defined for the
geometrically adapted pattern in Sec. 4.2 of the paper) and macro strains.

Conventions
-----------
* Grids are C-ordered numpy arrays of dtype uint8, shape (N0, N1) or
  (N0, N1, N2); array axis a is physical direction x_{a+1}.
* Voxelisation: a voxel with integer index i along an axis has its centre at
  (i + 1/2) h with h = 1; a voxel belongs to an inclusion if the periodic
  minimum-image distance from its centre to the inclusion centre is <= r.
* Every random draw goes through ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "disk", "ellipse", "square", "annulus", "laminate", "sphere",
    "rsa_fibres", "rsa_spheres", "RSAResult", "macro_strains",
    "phase_lame", "FIBRE_E", "FIBRE_NU", "MATRIX_E", "MATRIX_NU",
    "fibre_rve_256", "metric_rve",
]

# Phase constants of the synthetic workloads (GPa): a stiff fibre in a softer
# matrix, stiffness contrast about 6 in shear.
FIBRE_E, FIBRE_NU = 400.0, 0.2
MATRIX_E, MATRIX_NU = 70.0, 0.3


def phase_lame(E: float, nu: float) -> tuple[float, float]:
    """(lambda, mu) of an isotropic phase from Young's modulus and Poisson ratio.

    Plain unit conversion for building inputs, not part of the method.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def _centres(shape):
    """Cell-centre coordinates (i + 1/2) along every axis, broadcastable."""
    axes = []
    for a, n in enumerate(shape):
        c = np.arange(n, dtype=np.float64) + 0.5
        sh = [1] * len(shape)
        sh[a] = n
        axes.append(c.reshape(sh))
    return axes


def _min_image(d, n):
    """Periodic minimum-image difference of coordinates on a period-n axis."""
    return d - n * np.round(d / n)


def _dist2(shape, centre):
    axes = _centres(shape)
    d2 = 0.0
    for a, n in enumerate(shape):
        d = _min_image(axes[a] - centre[a], n)
        d2 = d2 + d * d
    return d2


def disk(n0: int, n1: int, radius: float, centre=None) -> np.ndarray:
    """One circular inclusion (periodic), default centre = cell centre of the box."""
    if centre is None:
        centre = (n0 / 2.0, n1 / 2.0)
    return (_dist2((n0, n1), centre) <= radius * radius).astype(np.uint8)


def sphere(n0: int, n1: int, n2: int, radius: float, centre=None) -> np.ndarray:
    """One spherical inclusion (periodic), default centre = centre of the box."""
    if centre is None:
        centre = (n0 / 2.0, n1 / 2.0, n2 / 2.0)
    return (_dist2((n0, n1, n2), centre) <= radius * radius).astype(np.uint8)


def ellipse(n0: int, n1: int, a: float, b: float, angle: float = 0.0, centre=None) -> np.ndarray:
    """Elliptical inclusion with semi-axes a (rotated by ``angle`` from axis 0) and b."""
    if centre is None:
        centre = (n0 / 2.0, n1 / 2.0)
    x0, x1 = _centres((n0, n1))
    d0 = _min_image(x0 - centre[0], n0)
    d1 = _min_image(x1 - centre[1], n1)
    c, s = math.cos(angle), math.sin(angle)
    u = c * d0 + s * d1
    v = -s * d0 + c * d1
    return ((u / a) ** 2 + (v / b) ** 2 <= 1.0).astype(np.uint8)


def square(n0: int, n1: int, side: float, centre=None) -> np.ndarray:
    """Axis-aligned square inclusion of edge length ``side``."""
    if centre is None:
        centre = (n0 / 2.0, n1 / 2.0)
    x0, x1 = _centres((n0, n1))
    d0 = np.abs(_min_image(x0 - centre[0], n0))
    d1 = np.abs(_min_image(x1 - centre[1], n1))
    return ((d0 <= side / 2.0) & (d1 <= side / 2.0)).astype(np.uint8)


def annulus(n0: int, n1: int, r_in: float, r_out: float, centre=None) -> np.ndarray:
    """Ring-shaped inclusion r_in < d <= r_out."""
    if centre is None:
        centre = (n0 / 2.0, n1 / 2.0)
    d2 = _dist2((n0, n1), centre)
    return ((d2 <= r_out * r_out) & (d2 > r_in * r_in)).astype(np.uint8)


def laminate(shape, thickness: int, offset: int = 0, axis: int = 0) -> np.ndarray:
    """Layered microstructure: g depends on the coordinate along ``axis`` only.

    Inclusion layer = indices offset .. offset+thickness-1 (periodic); the
    interfaces lie on voxel faces.
    """
    n = shape[axis]
    idx = (np.arange(n) - offset) % n
    prof = (idx < thickness).astype(np.uint8)
    sh = [1] * len(shape)
    sh[axis] = n
    return np.broadcast_to(prof.reshape(sh), tuple(shape)).copy()


@dataclass
class RSAResult:
    g: np.ndarray
    centres: list = field(default_factory=list)
    radii: list = field(default_factory=list)
    vf: float = 0.0
    attempts: int = 0

    @property
    def count(self) -> int:
        return len(self.radii)


def _stamp(g, centre, r):
    """Set g = 1 on the voxels of one periodic ball; only its bounding box is
    visited (voxels outside it are farther than r from the centre)."""
    shape = g.shape
    idx, ds = [], []
    for a, n in enumerate(shape):
        lo = int(np.floor(centre[a] - r - 1.0))
        hi = int(np.floor(centre[a] + r + 1.0))
        if hi - lo + 1 >= n:
            ii = np.arange(n)
        else:
            ii = np.arange(lo, hi + 1) % n
        x = ii.astype(np.float64) + 0.5
        d = _min_image(x - centre[a], n)
        sh = [1] * len(shape)
        sh[a] = ii.size
        idx.append(ii)
        ds.append(d.reshape(sh))
    d2 = 0.0
    for d in ds:
        d2 = d2 + d * d
    inside = d2 <= r * r
    sub = g[np.ix_(*idx)]
    sub |= inside.astype(np.uint8)
    g[np.ix_(*idx)] = sub


def _rsa(shape, r_lo, r_hi, target_vf, seed, max_count, max_attempts, gap):
    rng = np.random.default_rng(seed)
    dim = len(shape)
    ext = np.array(shape, dtype=np.float64)
    g = np.zeros(shape, dtype=np.uint8)
    centres = np.zeros((0, dim))
    radii = np.zeros(0)
    attempts = 0
    total = float(np.prod(shape))
    count = 0
    while attempts < max_attempts:
        if max_count is not None and radii.size >= max_count:
            break
        if target_vf is not None and count / total >= target_vf:
            break
        attempts += 1
        r = rng.uniform(r_lo, r_hi)
        c = rng.uniform(0.0, 1.0, size=dim) * ext
        if radii.size:
            d = _min_image(c[None, :] - centres, ext)
            dist2 = np.sum(d * d, axis=1)
            if np.any(dist2 < (r + radii + gap) ** 2):
                continue
        centres = np.vstack([centres, c[None, :]])
        radii = np.append(radii, r)
        _stamp(g, c, r)
        count = int(g.sum())
    return RSAResult(g=g, centres=[c for c in centres], radii=radii.tolist(), vf=float(g.sum()) / total,
                     attempts=attempts)


def rsa_fibres(n0: int, n1: int, r_lo: float, r_hi: float, seed: int, target_vf=None,
               max_count=None, max_attempts: int = 20000, gap: float = 1.0) -> RSAResult:
    """Random sequential addition of non-overlapping periodic disks.

    Radii ~ U[r_lo, r_hi]; centres ~ U over the box; a candidate is rejected if it
    comes closer than ``gap`` voxels to an accepted disk (minimum image).  Stops
    when the voxel volume fraction reaches ``target_vf``, when ``max_count``
    disks are placed, or after ``max_attempts`` draws.  The achieved count and
    volume fraction are recorded in the result.
    """
    return _rsa((n0, n1), r_lo, r_hi, target_vf, seed, max_count, max_attempts, gap)


def rsa_spheres(n0: int, n1: int, n2: int, r_lo: float, r_hi: float, seed: int, target_vf=None,
                max_count=None, max_attempts: int = 20000, gap: float = 1.0) -> RSAResult:
    """3D analogue of :func:`rsa_fibres` (non-overlapping periodic spheres)."""
    return _rsa((n0, n1, n2), r_lo, r_hi, target_vf, seed, max_count, max_attempts, gap)


def macro_strains(count: int, ncomp: int, amplitude: float, seed: int) -> np.ndarray:
    """``count`` macro strains, each component ~ U[-amplitude, amplitude].

    Component order: 2D [11, 22, 12], 3D [11, 22, 33, 23, 13, 12]; shear entries
    are tensor components (not engineering shear).
    """
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=(count, ncomp))


def fibre_rve_256(seed: int, n: int = 256) -> RSAResult:
    """Random-fibre RVE of the learned-warm-start workload.

    Volume fraction target ~ U[0.2, 0.5], fibre radius ~ U[8, 16] px (scaled by
    n/256 on other grids), RSA with at most 20000 draws.
    """
    rng = np.random.default_rng(seed)
    vf = rng.uniform(0.2, 0.5)
    s = n / 256.0
    return rsa_fibres(n, n, 8.0 * s, 16.0 * s, seed=seed + 7919, target_vf=vf, max_attempts=20000)


def metric_rve(index: int, n: int = 256):
    """Held-out RVE ``index`` of the headline workload: (g, macro strain [3]).

    Microstructure seed 1_000_000 + index; macro-strain seed = that + 10**7.
    """
    seed = 1_000_000 + index
    g = fibre_rve_256(seed, n).g
    eb = macro_strains(1, 3, 5e-3, seed + 10_000_000)[0]
    return g, eb
