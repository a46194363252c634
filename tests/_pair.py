"""Helpers that run the same seeded case through the CPU oracle and through
the GPU library (C ABI), for the parity tests."""
from __future__ import annotations

import os
import sys

import numpy as np

from oracle import oracle as O
from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth


def ensure_gpu_lib():
    if not os.path.exists(F.LIB_PATH):
        from paper_2212_01617_amd import build
        build.build()
    return F.lib()


def case_inputs(kind, shape, *, radius, xi, noise=1e-4, seed=0, rho_amp=0.0, u_amp=0.0,
                shear=None, center=None):
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    dims = 2 if kind == 0 else 3
    phi0 = synth.droplet_phi(sh, radius, xi, center=center, noise=noise, seed=seed, dims=dims)
    rho0 = None
    if rho_amp:
        rho0 = 1.0 + rho_amp * synth.smooth_random_field(sh, seed + 11)
    u0 = None
    if u_amp:
        u0 = u_amp * np.stack([synth.smooth_random_field(sh, seed + 20 + a) for a in range(3)])
    if shear is not None:
        rate, normal = shear
        u0 = (u0 if u0 is not None else 0.0) + synth.shear_velocity(sh, rate, axis_normal=normal)
    if u0 is not None and kind == 0:
        u0 = np.array(u0)
        u0[2] = 0.0
    return phi0, rho0, u0


def run_pair(kind, shape, steps, *, phi0, rho0=None, u0=None, mask=None, bc=(0, 0, 0),
             wall_u=None, rollers=(), storage=0, stream=None, **phys):
    """Returns (oracle Lattice, GPU Lattice) after `steps` steps."""
    po = O.make_params(kind, shape, bc=bc, wall_u=wall_u,
                       rollers=[(r[0], r[1], r[2]) for r in rollers], **phys)
    ref = O.Lattice(po, phi0, rho0, u0, mask)
    ref.step(steps)
    pg = F.make_params(kind, shape, storage=storage, bc=bc, wall_u=wall_u, rollers=rollers, **phys)
    gpu = F.Lattice(pg, phi0, rho0, u0, mask, stream=stream)
    gpu.step(steps)
    return ref, gpu


def field_errors(ref, gpu):
    a = ref.observe()
    b = gpu.read()
    fluid = a["solid"] == 0
    err = {}
    for k in ("rho", "phi", "mu_rho", "mu_phi", "P"):
        err[k] = float(np.abs((a[k] - b[k])[fluid]).max())
    uerr = 0.0
    for c, name in enumerate(("ux", "uy", "uz")):
        uerr = max(uerr, float(np.abs((a[name] - b["u"][c])[fluid]).max()))
    err["u"] = uerr
    return err


def pop_errors(ref, gpu):
    fa, ga = ref.populations()
    fb, gb = gpu.populations()
    return float(np.abs(fa - fb).max()), float(np.abs(ga - gb).max())


def log(*a):
    print(*a, file=sys.stderr, flush=True)
