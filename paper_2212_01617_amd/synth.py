"""Seeded synthetic inputs for FRE LBM droplet runs.

This module builds initial fields and geometry only -- droplet order parameter
profiles, seeded noise, initial shear velocity and voxelised roller masks.  It
holds none of the lattice Boltzmann arithmetic and imports nothing else from
the package, so the GPU path and the CPU oracle can both consume its output.

Arrays are numpy, shaped (nz, ny, nx) (x fastest in memory), float64.
Mask codes: 0 fluid, 1 static solid, 2+k moving with roller k.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """SplitMix64 (Steele, Lea, Flood 2014) evaluated at counter `index`:
    state = seed + (index+1) * golden gamma, then the published finaliser."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n uniforms in [lo, hi) from the top 53 bits of SplitMix64(seed, i)."""
    u = (splitmix64(seed, np.arange(n, dtype=np.uint64)) >> np.uint64(11)).astype(np.float64)
    u *= 2.0 ** -53
    return lo + (hi - lo) * u


def grid(shape):
    """Cell-centre coordinates (x, y, z), each shaped (nz, ny, nx)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def droplet_phi(shape, radius, xi, center=None, noise=0.0, seed=0, dims=3):
    """phi0 = tanh((R - r)/(sqrt(2) xi)) (+ seeded uniform noise in
    [-noise, noise)), r the distance from `center` (default: domain centre).
    dims=2 measures r in the x-y plane only (2D drop or cylinder along z)."""
    nz, ny, nx = shape
    x, y, z = grid(shape)
    if center is None:
        center = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2
    if dims == 3:
        r2 = r2 + (z - center[2]) ** 2
    r = np.sqrt(r2)
    phi = np.tanh((radius - r) / (math.sqrt(2.0) * xi))
    if noise:
        phi = phi + uniform(seed, phi.size, -noise, noise).reshape(shape)
    return phi


def slab_phi(shape, width, xi, axis=0):
    """Flat interfaces: phi = +1 inside a centred slab of `width` along `axis`,
    -1 outside, joined by two tanh(d/(sqrt(2) xi)) profiles."""
    coords = grid(shape)[axis]
    n = shape[2 - axis]
    c = (n - 1) / 2.0
    d = width / 2.0 - np.abs(coords - c)
    return np.tanh(d / (math.sqrt(2.0) * xi))


def shear_velocity(shape, rate, axis_normal=1, axis_flow=0):
    """Linear shear u_flow = rate * (s - (N-1)/2) along the wall-normal axis;
    returns u0 shaped (3, nz, ny, nx)."""
    u = np.zeros((3,) + tuple(shape))
    s = grid(shape)[axis_normal]
    n = shape[2 - axis_normal]
    u[axis_flow] = rate * (s - (n - 1) / 2.0)
    return u


def smooth_random_field(shape, seed, amplitude=1.0, modes=3):
    """A smooth periodic field: a few low Fourier modes with seeded amplitudes
    and phases (for brute-force and parity cases)."""
    nz, ny, nx = shape
    x, y, z = grid(shape)
    coef = uniform(seed, 4 * modes, -1.0, 1.0)
    out = np.zeros(shape)
    for m in range(modes):
        a, px, py, pz = coef[4 * m: 4 * m + 4]
        kx = 2 * math.pi * (m + 1) / nx
        ky = 2 * math.pi * ((m % 2) + 1) / ny
        kz = 2 * math.pi * ((m % 3) + 1) / nz if nz > 1 else 0.0
        out += a * np.sin(kx * x + math.pi * px) * np.cos(ky * y + math.pi * py) \
            * np.cos(kz * z + math.pi * pz)
    return amplitude * out / modes


def roller_mask(shape, centers, radius, axis=2, base=None):
    """Staircase voxelisation of cylinders along `axis`: a cell is solid (code
    2+k for roller k) iff its centre lies within `radius` of roller k's axis."""
    mask = np.zeros(shape, dtype=np.uint8) if base is None else base.copy()
    x, y, z = grid(shape)
    pos = (x, y, z)
    others = [a for a in range(3) if a != axis]
    for k, c in enumerate(centers):
        d2 = (pos[others[0]] - c[others[0]]) ** 2 + (pos[others[1]] - c[others[1]]) ** 2
        mask[d2 <= radius * radius] = 2 + k
    return mask


def four_roller_geometry(nx, ny, radius, nz=1):
    """Four cylinders along z centred at (nx/4, ny/4), (3nx/4, ny/4),
    (nx/4, 3ny/4), (3nx/4, 3ny/4) with alternating spin signs
    s_k = sign((X_k - nx/2)(Y_k - ny/2)); returns (centers, signs)."""
    cs = []
    signs = []
    for (fx, fy) in ((0.25, 0.25), (0.75, 0.25), (0.25, 0.75), (0.75, 0.75)):
        cx, cy = fx * nx, fy * ny
        cs.append((cx, cy, (nz - 1) / 2.0))
        signs.append(1.0 if (cx - nx / 2.0) * (cy - ny / 2.0) > 0 else -1.0)
    return cs, signs
