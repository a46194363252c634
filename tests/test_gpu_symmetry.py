"""Symmetries of the step on the HIP path (no oracle needed): a rounding
bias that breaks them shows up as a systematic difference that grows with
time, where unbiased rounding stays at the level of its noise.

* Point reflection (x -> -x about the centre, velocities reversed): the
  parallel-band shear with a centred drop, run from its initial state and
  from the reflected one, gives reflected fields.
* Phase inversion (phi -> -phi with kappa1 = kappa2): mu_rho is even and
  mu_phi odd in phi, so the run from -phi0 gives -phi and the same velocity.

Both run the 400x200 D2Q9 shear case (Re = 0.5, Ca = 0.1, R = 40, xi = 2)
for 2000 steps, stepped as the benchmark steps a lattice."""
import numpy as np
import pytest
import torch

from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth
from paper_2212_01617_amd.params import derive_params

from _pair import ensure_gpu_lib, log

pytestmark = pytest.mark.gpu

STEPS = 2000


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _case():
    nx, ny = 400, 200
    dp = derive_params(Re=0.5, Ca=0.1, radius=40.0, xi=2.0, H=ny, Pe=0.43)
    wu = np.zeros((3, 2, 3)); wu[1, 0, 0] = -dp.wall_u; wu[1, 1, 0] = dp.wall_u
    sh = (1, ny, nx)
    phi0 = synth.droplet_phi(sh, 40.0, 2.0, noise=1e-4, seed=0, dims=2)
    u0 = synth.shear_velocity(sh, dp.rate, axis_normal=1)
    p = F.make_params(0, (nx, ny, 1), bc=(0, 1, 0), wall_u=wu, **dp.phys())
    return p, phi0, u0


def _run(p, phi0, u0):
    L = F.Lattice(p, phi0, None, u0, stream=torch.cuda.Stream())
    L.step(STEPS)
    out = L.read(("phi", "u"))
    L.close()
    return out


def _reflect(a):
    # point reflection of a (nz, ny, nx) field about the centre of the x-y plane
    return a[:, ::-1, ::-1].copy()


def test_point_reflection():
    p, phi0, u0 = _case()
    a = _run(p, phi0, u0)
    b = _run(p, _reflect(phi0), -np.stack([_reflect(u0[k]) for k in range(3)]))
    e_phi = float(np.abs(_reflect(b["phi"]) - a["phi"]).max())
    e_u = max(float(np.abs(-_reflect(b["u"][k]) - a["u"][k]).max()) for k in range(2))
    log(f"[symmetry] point reflection, shear_400x200_{STEPS}: phi={e_phi:.2e} u={e_u:.2e}")
    assert e_phi < 1e-5 and e_u < 1e-7


def test_phase_inversion():
    p, phi0, u0 = _case()
    a = _run(p, phi0, u0)
    b = _run(p, -phi0, u0)
    e_phi = float(np.abs(b["phi"] + a["phi"]).max())
    e_u = max(float(np.abs(b["u"][k] - a["u"][k]).max()) for k in range(2))
    log(f"[symmetry] phase inversion, shear_400x200_{STEPS}: phi={e_phi:.2e} u={e_u:.2e}")
    assert e_phi < 1e-5 and e_u < 1e-7
