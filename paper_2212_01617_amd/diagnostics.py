"""Host-side droplet diagnostics on read-back fields (FP64, NumPy).

These evaluate the quantities the paper reports for its droplet runs
(Sec. 3: Taylor deformation D and orientation angle, breakup, the Laplace
pressure jump, droplet volume) from fields read back from a lattice.  They
do not take part in the time step.

Fields are NumPy arrays indexed [z, y, x] (2D lattices have z-extent 1), as
returned by ``Lattice.read``.

Readings used where the paper leaves the measurement open:
  * Deformation: the second central moments of the phase indicator
    C = clamp((phi - phi_out) / (phi_in - phi_out), 0, 1) about its
    centroid, restricted to the shear plane, where phi_in and phi_out are
    the medians of phi over the cells with phi > 0 and phi <= 0 (+1 and -1
    for ideal bulk phases: then C = (1 + phi) / 2).  Referencing the bulk
    keeps a slightly supersaturated matrix (a drop giving up volume by
    diffusion) from adding a box-shaped background to the moments.  With
    eigenvalues l1 >= l2 of that 2x2 tensor, D = (sqrt(l1) - sqrt(l2)) /
    (sqrt(l1) + sqrt(l2)) and theta is the angle of the leading eigenvector
    to the flow axis.  Exact for ellipses and for
    ellipsoids with a principal axis normal to the plane.
  * Breakup: connected components of {phi > 0} with face connectivity,
    periodic axes wrapped; components smaller than ``min_cells`` are ignored.
  * Steady state: D sampled every ``dt`` strain units is steady once
    max - min over the last ``window`` strain units is below ``tol``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import ndimage

AXES = {"x": 2, "y": 1, "z": 0}  # array axis of each spatial direction


def indicator(phi: np.ndarray, solid: np.ndarray | None = None) -> np.ndarray:
    """Phase indicator, 1 in the droplet's bulk and 0 in the matrix's:
    C = clamp((phi - phi_out) / (phi_in - phi_out), 0, 1) with phi_in,
    phi_out the medians of phi over the fluid cells with phi > 0 and
    phi <= 0.  Cells flagged in ``solid`` (obstacles, whose phi reads 0) get
    C = 0: they belong to neither phase."""
    phi = np.asarray(phi, dtype=np.float64)
    fluid = np.ones(phi.shape, dtype=bool) if solid is None else ~np.asarray(solid, dtype=bool)
    inside = (phi > 0.0) & fluid
    outside = (phi <= 0.0) & fluid
    if not inside.any() or not outside.any():
        C = np.clip(0.5 * (1.0 + phi), 0.0, 1.0)
    else:
        hi = float(np.median(phi[inside]))
        lo = float(np.median(phi[outside]))
        C = np.clip((phi - lo) / (hi - lo), 0.0, 1.0)
    if solid is not None:
        C[~fluid] = 0.0
    return C


def _periodic_centre(w: np.ndarray, axis: int) -> float:
    """Centroid of weights w along a periodic array axis (circular mean)."""
    n = w.shape[axis]
    prof = w.sum(axis=tuple(a for a in range(w.ndim) if a != axis))
    ang = 2.0 * math.pi * np.arange(n) / n
    s, c = float((prof * np.sin(ang)).sum()), float((prof * np.cos(ang)).sum())
    if s == 0.0 and c == 0.0:
        return (n - 1) / 2.0
    return (math.atan2(s, c) % (2.0 * math.pi)) * n / (2.0 * math.pi)


def centred(C: np.ndarray, periodic=(True, True, True)) -> tuple[np.ndarray, list[float]]:
    """Roll C along its periodic axes so that the droplet sits mid-domain.

    ``periodic`` is given for the spatial axes (x, y, z).  Returns the rolled
    array and the shift applied per array axis."""
    out = C
    shifts = [0.0, 0.0, 0.0]
    for name, ax in AXES.items():
        if not periodic["xyz".index(name)] or C.shape[ax] == 1:
            continue
        c = _periodic_centre(C, ax)
        k = int(round((C.shape[ax] - 1) / 2.0 - c))
        out = np.roll(out, k, axis=ax)
        shifts[ax] = k
    return out, shifts


def second_moments(C: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Centroid (x, y, z) and 3x3 second central moment tensor of weights C."""
    nz, ny, nx = C.shape
    m = C.sum()
    if m <= 0.0:
        raise ValueError("no droplet: the indicator is zero everywhere")
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = [x, y, z]
    cen = np.array([(C * p).sum() / m for p in pos])
    T = np.empty((3, 3))
    for a in range(3):
        for b in range(a, 3):
            T[a, b] = T[b, a] = (C * (pos[a] - cen[a]) * (pos[b] - cen[b])).sum() / m
    return cen, T


def centred_moments(C: np.ndarray, periodic=(True, True, True)) -> tuple[np.ndarray, np.ndarray]:
    """second_moments(centred(C, periodic)[0]), from the three plane sums of
    C: each moment involves at most two coordinates, so summing C over the
    third first gives it exactly, and the periodic centring rolls only those
    sums.  Equal to the direct form up to the order of the floating-point
    sums, for a fraction of its passes over C."""
    nz, ny, nx = C.shape
    m = C.sum()
    if m <= 0.0:
        raise ValueError("no droplet: the indicator is zero everywhere")
    P = {("x", "y"): C.sum(axis=0), ("x", "z"): C.sum(axis=1), ("y", "z"): C.sum(axis=2)}  # [ny,nx], [nz,nx], [nz,ny]
    prof = {"x": P[("x", "y")].sum(axis=0), "y": P[("x", "y")].sum(axis=1), "z": P[("x", "z")].sum(axis=1)}
    # the roll centred() applies per axis, from the same circular mean
    shift = {}
    for name in "xyz":
        n = prof[name].size
        if not periodic["xyz".index(name)] or n == 1:
            shift[name] = 0
            continue
        c = _periodic_centre(prof[name], 0)
        shift[name] = int(round((n - 1) / 2.0 - c))
    for name in "xyz":
        prof[name] = np.roll(prof[name], shift[name])
    for (u, v), Q in P.items():  # Q[v index, u index]
        P[(u, v)] = np.roll(np.roll(Q, shift[u], axis=1), shift[v], axis=0)
    pos = {name: np.arange(prof[name].size, dtype=np.float64) for name in "xyz"}
    cen = np.array([(prof[name] * pos[name]).sum() / m for name in "xyz"])
    d = {name: pos[name] - cen["xyz".index(name)] for name in "xyz"}
    T = np.empty((3, 3))
    for a, u in enumerate("xyz"):
        T[a, a] = (prof[u] * d[u] * d[u]).sum() / m
    for (u, v), Q in P.items():
        a, b = "xyz".index(u), "xyz".index(v)
        T[a, b] = T[b, a] = (Q * d[v][:, None] * d[u][None, :]).sum() / m
    return cen, T


@dataclass
class Deformation:
    D: float          # Taylor deformation (L - B)/(L + B)
    theta: float      # angle of the long axis to the flow axis, radians, in (-pi/2, pi/2]
    L: float          # relative long-axis length sqrt(l1)
    B: float          # relative short-axis length sqrt(l2)
    centre: tuple     # centroid (x, y, z) in the rolled frame


def deformation(phi: np.ndarray, plane: str = "xz", periodic=(True, True, True),
                solid: np.ndarray | None = None) -> Deformation:
    """Taylor deformation and orientation of the droplet in ``plane``.

    ``plane`` names the flow axis first and the second in-plane axis next,
    e.g. "xz" for shear along x with walls normal to z, "xy" for a 2D
    lattice or a four-roller cell.  theta > 0 means the long axis tilts
    from the flow axis towards the positive second axis.  ``solid`` flags
    obstacle cells, which are left out of the droplet."""
    cen, T = centred_moments(indicator(phi, solid), periodic)
    a, b = "xyz".index(plane[0]), "xyz".index(plane[1])
    S = np.array([[T[a, a], T[a, b]], [T[b, a], T[b, b]]])
    lam, vec = np.linalg.eigh(S)
    l2, l1 = max(lam[0], 0.0), max(lam[1], 0.0)
    v = vec[:, 1]
    theta = math.atan2(v[1], v[0])
    if theta > math.pi / 2:
        theta -= math.pi
    elif theta <= -math.pi / 2:
        theta += math.pi
    Lx, Bx = math.sqrt(l1), math.sqrt(l2)
    D = (Lx - Bx) / (Lx + Bx) if Lx + Bx > 0 else 0.0
    return Deformation(D=D, theta=theta, L=Lx, B=Bx, centre=tuple(cen))


def components(phi: np.ndarray, periodic=(True, True, True), min_cells: int = 8) -> list[int]:
    """Sizes (cells, descending) of the connected components of {phi > 0},
    face connectivity, periodic axes wrapped; components below ``min_cells``
    are dropped."""
    mask = np.asarray(phi) > 0.0
    lab, n = ndimage.label(mask)  # face connectivity by default
    if n == 0:
        return []
    parent = np.arange(n + 1)

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for name, ax in AXES.items():
        if not periodic["xyz".index(name)] or lab.shape[ax] < 2:
            continue
        lo = np.take(lab, 0, axis=ax)
        hi = np.take(lab, lab.shape[ax] - 1, axis=ax)
        both = (lo > 0) & (hi > 0)
        for a, b in zip(lo[both].ravel(), hi[both].ravel()):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n + 1)])
    # cells per label, then per merged component (label 0 is the matrix)
    per_label = np.bincount(lab.ravel(), minlength=n + 1)
    per_label[0] = 0
    sizes = np.bincount(roots, weights=per_label, minlength=n + 1).astype(np.int64)
    out = sorted((int(s) for s in sizes if s >= min_cells), reverse=True)
    return out


def broken_up(phi: np.ndarray, periodic=(True, True, True), min_cells: int = 8) -> bool:
    """True when {phi > 0} has split into two or more components."""
    return len(components(phi, periodic, min_cells)) >= 2


def laplace_jump(P: np.ndarray, phi: np.ndarray, bulk: float = 0.9) -> float:
    """Pressure jump across the interface: mean bulk pressure P over cells
    with phi > bulk minus the mean over cells with phi < -bulk (the bulk
    pressure formula holds away from interfaces only)."""
    phi = np.asarray(phi)
    inside, outside = phi > bulk, phi < -bulk
    if not inside.any() or not outside.any():
        raise ValueError("no bulk region on one side of the interface")
    return float(np.asarray(P)[inside].mean() - np.asarray(P)[outside].mean())


def droplet_volume(phi: np.ndarray) -> dict:
    """Droplet volume two ways: cells with phi > 0, and the sum of the
    bulk-referenced indicator."""
    phi = np.asarray(phi)
    return {"cells_phi_pos": int((phi > 0).sum()), "indicator_sum": float(indicator(phi).sum())}


def mass_drift(r0, r1) -> dict:
    """Relative drift of the totals reported by ``Lattice.reduce`` between two
    calls: sum rho relative to itself, sum phi relative to sum |phi|."""
    return {"rho": abs(r1[0] - r0[0]) / abs(r0[0]), "phi": abs(r1[1] - r0[1]) / max(abs(r0[2]), 1e-300)}


class SteadyTracker:
    """Steady-deformation test on D sampled every ``dt`` strain units: steady
    once the last ``window`` strain units of samples span less than ``tol``."""

    def __init__(self, dt: float = 0.1, window: float = 2.0, tol: float = 5e-4):
        self.dt, self.window, self.tol = dt, window, tol
        self.samples: list[tuple[float, float]] = []

    def add(self, strain: float, D: float) -> bool:
        self.samples.append((strain, D))
        return self.steady()

    def steady(self) -> bool:
        if not self.samples:
            return False
        s_end = self.samples[-1][0]
        if s_end < self.window:
            return False
        recent = [d for s, d in self.samples if s >= s_end - self.window - 1e-12]
        if len(recent) < 2:
            return False
        return max(recent) - min(recent) < self.tol
