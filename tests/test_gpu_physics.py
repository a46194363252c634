"""Physics of the GPU path (not parity tests): the free-energy model's
surface tension, the capillary relaxation rate and drop deformation in
shear, against the closed forms they should approach.

* Laplace law in 3D: dp = 2 sigma / R for a static drop.
* Capillary relaxation of a slightly prolate drop at rest: small-deformation
  theory for viscosity ratio 1 gives a decay rate of D of
  (40 (l+1) / ((2l+3)(19l+16))) sigma / (mu R) = 0.457 sigma / (mu R).
* Drop in shear.  Taylor's small-deformation law D = 35/32 Ca is for an
  unbounded sharp-interface 3D drop; 2D drops (cylinders) deform more.  The
  2D runs must reach a steady D roughly proportional to Ca within a loose
  band of 35/32 Ca.  The 3D run at the 256x128x128 benchmark's resolution
  (R = 25, xi = 2) is reported: there D keeps growing slowly over ten
  strain units, a resolution effect of the diffuse interface recorded, not
  asserted.
Peclet numbers are 10-20 here: at Pe = 0.43 the mobility is large enough
that drops of this size give up a large share of their volume by diffusion
within the run (the uniform mixture has less free energy than a drop at a
few per cent volume fraction).
"""
import math

import numpy as np
import pytest
import torch

from paper_2212_01617_amd import diagnostics as Dg
from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth
from paper_2212_01617_amd.params import derive_params

from _pair import ensure_gpu_lib, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _params(R, H=96, Pe=20.0, Ca=0.1, Re=1.0, xi=2.0):
    return derive_params(Re=Re, Ca=Ca, radius=R, xi=xi, H=H, Pe=Pe)


def test_laplace_law_3d():
    dp = _params(18.75)
    n, R = 64, 16.0
    phi0 = synth.droplet_phi((n, n, n), R, 2.0)
    L = F.Lattice(F.make_params(1, (n, n, n), **dp.phys()), phi0, stream=torch.cuda.Stream())
    L.step(4000)
    f = L.read(("phi", "P"))
    jump = Dg.laplace_jump(f["P"], f["phi"])
    log(f"[physics] laplace 3D: dp={jump:.4e} 2 sigma/R={2 * dp.sigma / R:.4e} ratio={jump / (2 * dp.sigma / R):.4f}")
    assert abs(jump / (2 * dp.sigma / R) - 1.0) < 0.03


def test_capillary_relaxation_rate_3d():
    dp = _params(18.75)
    n, R, e = 96, 18.75, 0.35
    x, y, z = synth.grid((n, n, n))
    c = (n - 1) / 2.0
    a, b = R * (1 + e) ** (2 / 3), R / (1 + e) ** (1 / 3)
    r = np.sqrt(((x - c) / a) ** 2 + ((y - c) / b) ** 2 + ((z - c) / b) ** 2)
    phi0 = np.tanh((1 - r) * R / (math.sqrt(2) * 2.0))
    L = F.Lattice(F.make_params(1, (n, n, n), **dp.phys()), phi0, stream=torch.cuda.Stream())
    t, ds = [], []
    for k in range(1, 9):
        L.step(250)
        t.append(250 * k)
        ds.append(Dg.deformation(L.read(("phi",))["phi"], plane="xz").D)
    rate = -np.polyfit(t, np.log(ds), 1)[0]
    theory = 0.457 * dp.sigma / (dp.nu * R)
    log(f"[physics] relaxation 3D: rate={rate:.3e}/step theory={theory:.3e} ratio={rate / theory:.3f} D={['%.4f' % d for d in ds]}")
    assert 0.6 < rate / theory < 1.25


def _shear_2d(Ca, R=40.0, nx=400, ny=200, strain=12, Pe=10.0):
    dp = derive_params(Re=0.5, Ca=Ca, radius=R, xi=2.0, H=ny, Pe=Pe)
    wu = np.zeros((3, 2, 3)); wu[1, 0, 0] = -dp.wall_u; wu[1, 1, 0] = dp.wall_u
    sh = (1, ny, nx)
    phi0 = synth.droplet_phi(sh, R, 2.0, noise=1e-4, seed=0, dims=2)
    u0 = synth.shear_velocity(sh, dp.rate, axis_normal=1)
    p = F.make_params(0, (nx, ny, 1), bc=(0, 1, 0), wall_u=wu, **dp.phys())
    L = F.Lattice(p, phi0, None, u0, stream=torch.cuda.Stream())
    per = int(round(1.0 / dp.rate))
    hist = []
    for _ in range(strain):
        L.step(per)
        hist.append(Dg.deformation(L.read(("phi",))["phi"], plane="xy", periodic=(True, False, True)))
    return hist


def test_drop_in_shear_2d_steady_and_proportional_to_ca():
    out = {}
    for Ca in (0.05, 0.1, 0.2):
        h = _shear_2d(Ca)
        last = [d.D for d in h[-4:]]
        out[Ca] = float(np.mean(last))
        log(f"[physics] shear 2D Ca={Ca}: D(strain)={['%.3f' % d.D for d in h]} "
            f"theta={math.degrees(h[-1].theta):.1f} D/(35/32 Ca)={out[Ca] / (35 / 32 * Ca):.3f}")
        assert max(last) - min(last) < 0.01            # steady over the last 4 strain units
        assert 0.8 < out[Ca] / (35 / 32 * Ca) < 2.0
    assert 1.4 < out[0.1] / out[0.05] < 2.4
    assert 1.5 < out[0.2] / out[0.1] < 2.4


def test_drop_in_shear_3d_reported():
    Ca, R, xi = 0.1, 25.0, 2.0
    nx, ny, nz = 256, 128, 128
    dp = derive_params(Re=0.5, Ca=Ca, radius=R, xi=xi, H=nz, Pe=10.0)
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -dp.wall_u; wu[2, 1, 0] = dp.wall_u
    sh = (nz, ny, nx)
    phi0 = synth.droplet_phi(sh, R, xi, noise=1e-4, seed=0)
    u0 = synth.shear_velocity(sh, dp.rate, axis_normal=2)
    L = F.Lattice(F.make_params(1, (nx, ny, nz), bc=(0, 0, 1), wall_u=wu, **dp.phys()), phi0, None, u0,
                  stream=torch.cuda.Stream())
    per = int(round(1.0 / dp.rate))
    hist = []
    for _ in range(4):
        L.step(per)
        hist.append(Dg.deformation(L.read(("phi",))["phi"], plane="xz", periodic=(True, True, False)))
    phi = L.read(("phi",))["phi"]
    log(f"[physics] shear 3D Ca={Ca} R={R} xi={xi}: D(strain)={['%.3f' % d.D for d in hist]} "
        f"theta={['%.0f' % math.degrees(d.theta) for d in hist]} D/(35/32 Ca) at 1 strain="
        f"{hist[0].D / (35 / 32 * Ca):.2f}")
    assert len(Dg.components(phi, (True, True, False))) == 1
    assert L.reduce()[6] == 0
    # the first response is of Taylor's size; later growth is reported above
    assert 0.5 < hist[0].D / (35 / 32 * Ca) < 2.0


def test_drop_in_shear_3d_thin_interface_reaches_taylor():
    """P8 at the C3 box (256x128x128, R = 25, Ca = 0.1, Re = 0.5, Pe = 10):
    with R/xi = 25 the deformation after one strain unit is Taylor's
    35/32 Ca, and the slow later growth of D, which the diffuse interface
    causes, is much weaker than at R/xi = 12.5 (it falls with the Cahn number
    and does not depend on the wall distance or the force discretisation)."""
    from paper_2212_01617_amd import campaign
    thin = campaign.shear_history(radius=25.0, xi=1.0, strain=8.0, every=1.0)
    wide = campaign.shear_history(radius=25.0, xi=2.0, strain=8.0, every=1.0)
    taylor = thin["taylor_D"]
    D = {k: {h["strain"]: h["D"] for h in r["history"]} for k, r in (("thin", thin), ("wide", wide))}
    grow = {k: D[k][8.0] - D[k][4.0] for k in D}
    log(f"[physics] shear 3D R/xi=25: D={[D['thin'][s] for s in sorted(D['thin'])]}; "
        f"R/xi=12.5: D={[D['wide'][s] for s in sorted(D['wide'])]}; Taylor {taylor:.4f}; "
        f"growth 4->8 strain: {grow['thin']:.4f} vs {grow['wide']:.4f}")
    assert 0.8 < D["thin"][1.0] / taylor < 1.2
    assert 0 < grow["thin"] < 0.5 * grow["wide"]
