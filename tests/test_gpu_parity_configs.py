"""Parity at the full sizes of the other benchmark configurations, stepped as
the benchmark steps (own stream, captured graphs), every cell against the
FP64 oracle on the same seeded inputs:

* the 100x100 D2Q9 static drop (R = 20, xi = 1.5, A = 0.04, kappa = 0.09,
  tau = 1, M = 0.1), its full 2000 steps;
* the 400x200 D2Q9 parallel-band shear (walls at -+u_w, R = 40, xi = 2,
  Re = 0.5, Ca = 0.1, linear-shear start): 300 steps at the bar, then 1000
  and 2000 of its 40k steps with the phi difference stated and the Taylor
  deformation D from both phi fields within 1%;
* the 256x256x64 D3Q19 four-roller cell (cylinders of radius 30 at the
  quarter points in alternating rotation, R = 24, xi = 2, Re = 0.5,
  Ca = 0.1), 20 steps on all 4.2 M cells.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2212_01617_amd import diagnostics as Dg
from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth
from paper_2212_01617_amd.params import derive_params

from _pair import ensure_gpu_lib, field_errors, log, pop_errors

pytestmark = pytest.mark.gpu

TOL = {"rho": 1e-5, "phi": 1e-5, "u": 1e-5, "mu_rho": 1e-6, "mu_phi": 1e-6, "P": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _run(kind, shape, steps, phi0, u0=None, mask=None, bc=(0, 0, 0), wall_u=None, rollers=(), **phys):
    ref = O.Lattice(O.make_params(kind, shape, bc=bc, wall_u=wall_u,
                                  rollers=[(r[0], r[1], r[2]) for r in rollers], **phys), phi0, None, u0, mask)
    ref.step(steps)
    gpu = F.Lattice(F.make_params(kind, shape, bc=bc, wall_u=wall_u, rollers=rollers, **phys), phi0, None, u0,
                    mask, stream=torch.cuda.Stream())
    gpu.step(steps)
    return ref, gpu


def _check(name, ref, gpu, extra=""):
    err = field_errors(ref, gpu)
    pf, pg = pop_errors(ref, gpu)
    log(f"[parity] {name}: " + " ".join(f"{k}={v:.2e}" for k, v in err.items()) + f" f={pf:.2e} g={pg:.2e}" + extra)
    for k, v in TOL.items():
        assert err[k] < v, (name, k, err[k])
    assert pf < 1e-5 and pg < 1e-5


def test_static_drop_100x100_full_run():
    sh = (1, 100, 100)
    phi0 = synth.droplet_phi(sh, 20.0, 1.5, center=(49.5, 49.5, 0), noise=1e-4, seed=0, dims=2)
    ref, gpu = _run(0, (100, 100, 1), 2000, phi0, A=0.04, kappa=0.09, tau_f=1.0, tau_g=1.0, M=0.1)
    _check("config_static_drop_100x100_2000", ref, gpu)


def test_parallel_band_shear_400x200():
    """300 steps at the 1e-5 bar; then to 2000 steps, where the max-abs phi
    difference has grown past it: the FP32 collision conserves momentum only
    to rounding, and in this low-Re, 200-cell channel the velocity
    difference grows linearly over the run (viscous time about 240k steps),
    moving the interface.  Stated, with u below 1e-5 and D within 1%."""
    nx, ny = 400, 200
    dp = derive_params(Re=0.5, Ca=0.1, radius=40.0, xi=2.0, H=ny, Pe=0.43)
    wu = np.zeros((3, 2, 3)); wu[1, 0, 0] = -dp.wall_u; wu[1, 1, 0] = dp.wall_u
    sh = (1, ny, nx)
    phi0 = synth.droplet_phi(sh, 40.0, 2.0, noise=1e-4, seed=0, dims=2)
    u0 = synth.shear_velocity(sh, dp.rate, axis_normal=1)
    ref, gpu = _run(0, (nx, ny, 1), 300, phi0, u0, bc=(0, 1, 0), wall_u=wu, **dp.phys())
    _check("config_shear_400x200_300", ref, gpu)
    per = (True, False, True)
    for upto in (1000, 2000):
        n = upto - ref.t
        ref.step(n)
        gpu.step(n)
        err = field_errors(ref, gpu)
        d_ref = Dg.deformation(ref.observe()["phi"], plane="xy", periodic=per).D
        d_gpu = Dg.deformation(gpu.read(("phi",))["phi"], plane="xy", periodic=per).D
        rel = abs(d_gpu - d_ref) / abs(d_ref)
        log(f"[parity] config_shear_400x200_{upto}: " + " ".join(f"{k}={v:.2e}" for k, v in err.items())
            + f" D_oracle={d_ref:.5f} D_gpu={d_gpu:.5f} rel={rel:.2e}")
        assert err["u"] < 1e-5 and err["phi"] < 5e-5 and rel < 0.01
    assert d_ref > 1e-3


def test_four_roller_256x256x64():
    nx, ny, nz = 256, 256, 64
    rr = 30.0
    dp = derive_params(Re=0.5, Ca=0.1, radius=24.0, xi=2.0, Pe=0.43)
    cs, signs = synth.four_roller_geometry(nx, ny, rr, nz=nz)
    om = dp.rate * (math.hypot(nx / 4.0, ny / 4.0) - rr) / rr
    sh = (nz, ny, nx)
    mask = synth.roller_mask(sh, cs, rr)
    rollers = [(c, s * om, 2, rr) for c, s in zip(cs, signs)]
    phi0 = synth.droplet_phi(sh, 24.0, 2.0, noise=1e-4, seed=0)
    solid = float((mask != 0).mean())
    ref, gpu = _run(1, (nx, ny, nz), 20, phi0, mask=mask, rollers=rollers, **dp.phys())
    _check("config_four_roller_256x256x64_20", ref, gpu, f" solid={solid:.3f}")
    assert 0.15 < solid < 0.2
