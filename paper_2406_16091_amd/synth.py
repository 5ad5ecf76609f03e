"""Seeded synthetic particle systems.

The paper evaluates on synthetic particles only: i.i.d. uniform positions in
a grid of d^3 cells with 1, 10 or 100 particles per cell on average, in
single precision (Sec. 7.1 "Experimental Setup").  The systems here follow
the same recipe at the sizes of the workloads this library is measured on,
plus a clustered (Gaussian-blob) mix, a batch of many small systems and a
serving request stream.

Every coordinate is drawn as an integer lattice index m and scaled by a power
of two (x = m * 2^-p with m < 2^24), so it is exactly representable in
float32 and every difference of two coordinates is exact.  Weights are
w = 0.5 + m' * 2^-23, uniform on [0.5, 1.5).

This module holds no arithmetic of the method itself (no cell indices, no
sums, no kernel); it only draws inputs, and both the GPU path and the oracle
consume what it returns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class System:
    name: str
    x: np.ndarray            # float32 [n]
    y: np.ndarray
    z: np.ndarray
    w: np.ndarray            # float32 [n] weights
    origin: tuple            # (ox, oy, oz) float
    dims: tuple              # (nx, ny, nz) int
    cell_w: float            # cell width (>= rc)
    rc: float                # cutoff radius
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


def _weights(rng, n):
    m = rng.integers(0, 1 << 23, size=n, dtype=np.int64)
    return (0.5 + m.astype(np.float64) * 2.0 ** -23).astype(np.float32)


def _lattice_uniform(rng, n, extent_units, p):
    """n points uniform on {0, 2^-p, ..., extent - 2^-p} per axis."""
    hi = int(extent_units) << p
    assert hi <= (1 << 24)
    out = []
    for _ in range(3):
        m = rng.integers(0, hi, size=n, dtype=np.int64)
        out.append((m.astype(np.float64) * 2.0 ** -p).astype(np.float32))
    return out


def _lattice_quantize(v, extent_units, p):
    """Clip v to [0, extent - 2^-p] and round down to the 2^-p lattice."""
    hi = (int(extent_units) << p) - 1
    m = np.clip(np.floor(v * float(1 << p)), 0, hi).astype(np.int64)
    return (m.astype(np.float64) * 2.0 ** -p).astype(np.float32)


def uniform_unit_cube(n, rc_log2, seed, name="uniform"):
    """n particles uniform in [0,1)^3 on the 2^-24 lattice; r_c = cell width =
    2^rc_log2 (a power of two), non-periodic grid of (1/r_c)^3 cells."""
    rng = np.random.default_rng(seed)
    x, y, z = _lattice_uniform(rng, n, 1, 24)
    w = _weights(rng, n)
    rc = 2.0 ** rc_log2
    d = int(round(1.0 / rc))
    return System(name, x, y, z, w, (0.0, 0.0, 0.0), (d, d, d), rc, rc,
                  {"seed": seed, "lattice": 2.0 ** -24})


def tiny(seed=1):
    """32,768 uniform particles, r_c = 1/32, 32^3 cells (about 1 per cell)."""
    return uniform_unit_cube(32768, -5, seed, "tiny-32k-32^3")


def scale_1ppc(seed=2):
    """2^24 uniform particles, r_c = 1/256, 256^3 cells (1 per cell)."""
    return uniform_unit_cube(1 << 24, -8, seed, "uniform-16.8M-256^3-1ppc")


def scale_8ppc(seed=2):
    """2^24 uniform particles, r_c = 1/128, 128^3 cells (8 per cell)."""
    return uniform_unit_cube(1 << 24, -7, seed, "uniform-16.8M-128^3-8ppc")


def dense_64ppc(seed=4):
    """2^21 uniform particles, r_c = 1/32, 32^3 cells (64 per cell): the
    occupancy of the dense cores of the clustered inputs, everywhere."""
    return uniform_unit_cube(1 << 21, -5, seed, "uniform-2.1M-32^3-64ppc")


def _blob_sigmas(rng, n_blobs, n_blob_pts, g, lo, hi, peak_ppc):
    """Blob widths in cells: drawn from U(lo, hi) * g, raised where needed so
    that no blob's centre holds more than about peak_ppc particles per cell
    (density of an isotropic Gaussian at its centre: n / ((2 pi)^1.5 s^3))."""
    sig = rng.uniform(lo, hi, size=n_blobs) * g
    floor = (n_blob_pts / ((2.0 * math.pi) ** 1.5 * peak_ppc)) ** (1.0 / 3.0)
    return np.maximum(sig, floor)


def _blob_points(rng, centres, sig, which, extent):
    """Gaussian points around centres[which]; a point that falls outside
    [0, extent)^3 is drawn again (truncated Gaussians), so no mass piles up
    on the faces of the box."""
    pts = centres[which] + sig[which, None] * rng.standard_normal((which.size, 3))
    bad = np.nonzero(((pts < 0) | (pts >= extent)).any(axis=1))[0]
    while bad.size:
        w = which[bad]
        pts[bad] = centres[w] + sig[w, None] * rng.standard_normal((bad.size, 3))
        bad = bad[((pts[bad] < 0) | (pts[bad] >= extent)).any(axis=1)]
    return pts


def clustered(n=1 << 23, n_blobs=64, bg_frac=0.10, rc_log2=-7, seed=3, name=None,
              sigma=(0.04, 0.08), peak_ppc=60.0):
    """Gaussian blobs (centres uniform in [0,1)^3, blob chosen uniformly,
    width U(sigma) in box units, raised so that blob centres stay near
    peak_ppc particles per cell, truncated to the unit cube) plus a uniform
    background fraction, quantized to the 2^-24 lattice."""
    rng = np.random.default_rng(seed)
    rc = 2.0 ** rc_log2
    d = int(round(1.0 / rc))
    n_bg = int(round(bg_frac * n))
    n_bl = n - n_bg
    centres = rng.random((n_blobs, 3))
    sig = _blob_sigmas(rng, n_blobs, n_bl / n_blobs, d, sigma[0], sigma[1], peak_ppc) / d
    which = rng.integers(0, n_blobs, size=n_bl)
    pts = _blob_points(rng, centres, sig, which, 1.0)
    bg = rng.random((n_bg, 3))
    allp = np.concatenate([pts, bg], axis=0)
    order = rng.permutation(n)          # interleave blob and background points
    allp = allp[order]
    x = _lattice_quantize(allp[:, 0], 1, 24)
    y = _lattice_quantize(allp[:, 1], 1, 24)
    z = _lattice_quantize(allp[:, 2], 1, 24)
    w = _weights(rng, n)
    return System(name or f"clustered-{n}-{d}^3", x, y, z, w, (0.0, 0.0, 0.0),
                  (d, d, d), rc, rc, {"seed": seed, "blobs": n_blobs, "lattice": 2.0 ** -24})


def box_system(n, g, seed, lattice_log2, clustered_blobs=0, name=None,
               sigma=(0.04, 0.08), peak_ppc=60.0):
    """n particles in the box [0, g)^3 of unit cells (cell width = r_c = 1),
    on the 2^-lattice_log2 lattice; uniform, or `clustered_blobs` Gaussian
    blobs (width U(sigma) * g, raised so that blob centres stay near
    peak_ppc particles per cell) with a 10% uniform background."""
    rng = np.random.default_rng(seed)
    p = lattice_log2
    if clustered_blobs <= 0:
        x, y, z = _lattice_uniform(rng, n, g, p)
        kind = "uniform"
    else:
        n_bg = int(round(0.1 * n))
        centres = rng.random((clustered_blobs, 3)) * g
        sig = _blob_sigmas(rng, clustered_blobs, (n - n_bg) / clustered_blobs, g,
                           sigma[0], sigma[1], peak_ppc)
        which = rng.integers(0, clustered_blobs, size=n - n_bg)
        pts = _blob_points(rng, centres, sig, which, float(g))
        allp = np.concatenate([pts, rng.random((n_bg, 3)) * g], axis=0)[rng.permutation(n)]
        x = _lattice_quantize(allp[:, 0], g, p)
        y = _lattice_quantize(allp[:, 1], g, p)
        z = _lattice_quantize(allp[:, 2], g, p)
        kind = "clustered"
    w = _weights(rng, n)
    return System(name or f"{kind}-{n}-{g}^3", x, y, z, w, (0.0, 0.0, 0.0), (g, g, g),
                  1.0, 1.0, {"seed": seed, "lattice": 2.0 ** -p, "kind": kind})


def batch_systems(count=512, seed=4):
    """Independent systems for one batched launch: N_k log-uniform in
    [1e3, 2e5], target occupancy U[1, 4] per cell, g_k = clamp(round(cbrt(
    N_k / ppc)), 10, 58) unit cells per side, 2^-18 lattice; system k is drawn
    with seed 1000 * seed + k."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nk = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        ppc = float(rng.uniform(1.0, 4.0))
        g = int(min(58, max(10, round((nk / ppc) ** (1.0 / 3.0)))))
        out.append(box_system(nk, g, 1000 * seed + k, 18, name=f"batch{k}-{nk}-{g}^3"))
    return out


def serve_requests(count, seed=5, n_lo=1e4, n_hi=4e6):
    """Request systems for the serving loop: N log-uniform in [n_lo, n_hi],
    uniform or 8-blob clustered (50/50), mean occupancy in {1, 2, 4, 8},
    g = round(cbrt(N / ppc)) unit cells per side, 2^-16 lattice."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        ppc = int(rng.choice([1, 2, 4, 8]))
        g = int(max(1, round((n / ppc) ** (1.0 / 3.0))))
        blobs = 8 if rng.random() < 0.5 else 0
        out.append(box_system(n, g, 1000 * seed + k, 16, clustered_blobs=blobs,
                              name=f"req{k}-{n}-{g}^3-{'c' if blobs else 'u'}"))
    return out


def subsample(n, count, seed=20):
    """Sorted distinct target indices for sampled parity checks."""
    rng = np.random.default_rng(seed)
    if count >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)
