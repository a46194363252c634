"""Pins of the oracle's consistent initialisation (CPU).

Sec. 2.3 initialises the populations at equilibrium and then aligns their
kinetic moments by collisions, after Mei et al. (2006).  The oracle reads
this as pre-iterations of f with the velocity held at u0 and phi at phi0
(rho free), g reset to its equilibrium afterwards.  What fixes the result
independently of the oracle's own code:

* Plane Couette flow: the non-equilibrium part of f of a BGK lattice in a
  linear shear u_x = gamma y has the Chapman-Enskog second moment
  sum_i c_ix c_iy (f_i - f_i^eq) = -tau rho cs^2 gamma (exact for a linear
  profile).  Equilibrium initialisation has zero there; the pre-iterations
  must reach the closed form.
* Static drop: with u held at 0 the density relaxes to mechanical
  equilibrium, cs^2 grad rho = F, so the bulk pressure jump across the
  interface approaches the Laplace value sigma/R already at t = 0 (the
  equilibrium initialisation gives almost none of it), phi is untouched, and
  the observed velocity (which includes F/2) drops towards the prescribed
  u0 = 0.  g then satisfies the g^eq moment identity sum c_x^2 g = Gamma
  mu_phi with the mu_phi of the new density.
* A uniform bulk state at rest is a fixed point.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2212_01617_amd import synth

CS2 = 1.0 / 3.0


def _couette(kind, n_wall, tau, uw=5e-3):
    """Walls normal to y (D2Q9) or z (D3Q19) moving at -uw / +uw along x and
    the exact linear profile between the halfway walls as u0."""
    ax = 1 if kind == 0 else 2
    shape = (4, n_wall, 1) if kind == 0 else (2, 3, n_wall)
    bc = [0, 0, 0]
    bc[ax] = 1
    wu = np.zeros((3, 2, 3))
    wu[ax, 0, 0], wu[ax, 1, 0] = -uw, uw
    p = O.make_params(kind, shape, bc=tuple(bc), wall_u=wu, A=0.04, kappa=0.09, tau_f=tau, tau_g=1.0, M=0.1)
    nx, ny, nz = shape
    coord = np.arange(n_wall)
    prof = uw * (2.0 * (coord + 0.5) / n_wall - 1.0)
    u0 = np.zeros((3, nz, ny, nx))
    if ax == 1:
        u0[0] = prof[None, :, None]
    else:
        u0[0] = prof[:, None, None]
    phi0 = -np.ones((nz, ny, nx))
    return p, phi0, u0, 2.0 * uw / n_wall, ax


def _shear_moment(L, kind, u0, ax):
    c, _ = O.tables(kind)
    f, _ = L.populations()
    rho = L.observe()["rho"]
    q = f.shape[0]
    fl = f.reshape(q, -1)
    r = rho.reshape(-1)
    uu = u0.reshape(3, -1)
    out = np.empty(r.size)
    for k in range(r.size):
        fneq = fl[:, k] - O.feq(kind, r[k], uu[:, k])
        out[k] = (c[:, 0] * c[:, ax] * fneq).sum()
    return out, r


@pytest.mark.parametrize("kind,n_wall,tau", [(0, 16, 0.8), (1, 12, 1.3)])
def test_couette_nonequilibrium_reaches_chapman_enskog(kind, n_wall, tau):
    p, phi0, u0, gam, ax = _couette(kind, n_wall, tau)
    L0 = O.Lattice(p, phi0, None, u0)
    m0, _ = _shear_moment(L0, kind, u0, ax)
    assert np.abs(m0).max() < 1e-15          # equilibrium initialisation: no stress
    L = O.Lattice(p, phi0, None, u0).consistent_init(phi0, u0, 80)
    m, rho = _shear_moment(L, kind, u0, ax)
    theory = -tau * rho * CS2 * gam
    assert np.abs(m / theory - 1.0).max() < 1e-6
    assert np.abs(rho - 1.0).max() < 1e-12   # Couette flow has uniform pressure
    assert L.t == 0


@pytest.fixture(scope="module")
def drop():
    n, R, xi, A, kap = 64, 16.0, 1.5, 0.04, 0.09
    p = O.make_params(0, (n, n, 1), A=A, kappa=kap, tau_f=1.0, tau_g=1.0, M=0.1)
    phi0 = synth.droplet_phi((1, n, n), R, xi, dims=2)
    sigma = math.sqrt(8.0 * kap * A / 9.0)
    return p, phi0, sigma / R


def _jump(o):
    return o["P"][o["phi"] > 0.9].mean() - o["P"][o["phi"] < -0.9].mean()


def test_static_drop_pressure_jump_at_t0(drop):
    p, phi0, laplace = drop
    o_eq = O.Lattice(p, phi0).observe()
    o = O.Lattice(p, phi0).consistent_init(phi0, None, 2000).observe()
    assert _jump(o_eq) / laplace < 0.1                 # equilibrium start: no Laplace jump yet
    assert 0.85 < _jump(o) / laplace < 1.05            # aligned start: close to sigma/R
    assert np.abs(o["phi"] - phi0).max() < 1e-14       # phi is the prescribed field
    # the observed velocity (j + F/2)/rho approaches the prescribed u0 = 0
    u_eq = np.abs(np.stack([o_eq["ux"], o_eq["uy"]])).max()
    u = np.abs(np.stack([o["ux"], o["uy"]])).max()
    assert u < 0.1 * u_eq and u < 5e-5


def test_g_is_the_equilibrium_of_the_aligned_state(drop):
    """g is reset to g^eq(phi0, mu_phi, u0 = 0) with the mu_phi of the new rho:
    its second moment is Gamma mu_phi (the g^eq moment identity) with the
    mu_phi the lattice reports, which differs from the mu_phi of rho0 = 1."""
    p, phi0, _ = drop
    L = O.Lattice(p, phi0).consistent_init(phi0, None, 500)
    o = L.observe()
    _, g = L.populations()
    c, _ = O.tables(0)
    gamma = p.M / (p.tau_g - 0.5)
    m2 = np.tensordot(c[:, 0] ** 2, g, axes=1)
    assert np.abs(m2 - gamma * o["mu_phi"]).max() < 1e-12
    mu_start = O.Lattice(p, phi0).observe()["mu_phi"]
    assert np.abs(o["mu_phi"] - mu_start).max() > 1e-6


@pytest.mark.parametrize("phase", [1.0, -1.0])
def test_uniform_bulk_is_a_fixed_point(phase):
    p = O.make_params(1, (4, 4, 4), A=0.04, kappa=0.09, tau_f=0.9, tau_g=1.0, M=0.1)
    phi0 = phase * np.ones((4, 4, 4))
    L0 = O.Lattice(p, phi0)
    f0, g0 = L0.populations()
    L = O.Lattice(p, phi0).consistent_init(phi0, None, 20)
    f, g = L.populations()
    assert np.abs(f - f0).max() < 1e-15 and np.abs(g - g0).max() < 1e-15


def test_only_before_the_first_step():
    p, phi0, u0, _, _ = _couette(0, 8, 1.0)
    L = O.Lattice(p, phi0, None, u0).step(1)
    with pytest.raises(ValueError):
        L.consistent_init(phi0, u0, 2)
