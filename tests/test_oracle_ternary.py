"""Pins of the oracle's ternary extension (Sec. 2.2, Remark after the
mobility relation: one more coupled Cahn-Hilliard equation and one more
population for a third order parameter psi, with the free energy of the
ternary model the Remark cites, in concentrations C1 = (rho + phi - psi)/2,
C2 = (rho - phi - psi)/2, C3 = psi).

* brute force: the C oracle against the independently structured NumPy
  step (written in the concentrations) on tiny lattices with moving walls, a
  box and a roller, 100 steps, to 1e-13;
* with psi = 0 and no mobility for it the ternary step is the binary step
  (to rounding) and psi and h stay exactly zero;
* the potentials are the derivatives of the bulk free-energy density, and of
  the discrete functional with its gradient terms written with the lattice
  Laplacian (a numerical derivative of an energy assembled here);
* the three order parameters are conserved to 1e-12 with moving walls;
* a flat interface between any two components, the third absent, relaxes
  to the profile that solves the discrete equilibrium of the pair
  (C(1 - C)(1 - 2C) - alpha^2 lap_h C uniform, by Newton), the same for all
  three pairs whatever the kappas, with the third component back at zero
  and the continuum tanh((x - x0) / 2 alpha) profile within the lattice
  error;
* a drop of component 1 in component 3 obeys the Laplace law with the pair
  tension alpha (kappa1 + kappa3) / 6, which is not the (1, 2) tension."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle.brute import Brute3
from paper_2212_01617_amd import synth

KW = dict(kappa1=0.16, kappa2=0.12, alpha=1.0, tau_f=0.8, tau_g=1.1, M=0.1)
K3 = dict(kappa3=0.2, M3=0.07, tau_h=0.9)


def _fields(kind, shape, seed=0):
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    c1 = 0.5 * (1 + synth.droplet_phi(sh, 2.5, 1.2, dims=3 if kind else 2))
    c3 = 0.3 * (1 - c1) + 0.02 * synth.smooth_random_field(sh, 4 + seed)
    c2 = 1 - c1 - c3
    rho0 = 1 + 0.01 * synth.smooth_random_field(sh, 3 + seed)
    u0 = 0.01 * np.stack([synth.smooth_random_field(sh, 5 + a + seed) for a in range(3)])
    if kind == 0:
        u0[2] = 0
    return c1 - c2, c3, rho0, u0


CASES = {
    "d2q9_walls": (0, (8, 8, 1), (0, 1, 0), [[[0] * 3] * 2, [[-0.01, 0, 0], [0.01, 0, 0]], [[0] * 3] * 2]),
    "d3q19_walls": (1, (8, 8, 8), (0, 0, 1), [[[0] * 3] * 2, [[0] * 3] * 2, [[-0.01, 0, 0], [0.02, 0.005, 0]]]),
    "d3q19_box": (1, (8, 6, 7), (1, 0, 1), np.random.default_rng(0).uniform(-0.01, 0.01, (3, 2, 3))),
}


def _pair(kind, shape, bc, wu, mask=None, rollers=()):
    phi0, psi0, rho0, u0 = _fields(kind, shape)
    L = O.Lattice3(O.make_params(kind, shape, bc=bc, wall_u=wu, rollers=rollers, **KW), K3["kappa3"], K3["M3"],
                   K3["tau_h"], phi0, psi0, rho0, u0, mask)
    B = Brute3(kind, shape, phi0, psi0, rho0, u0, mask, bc=bc, wall_u=wu, rollers=rollers, **K3, **KW)
    return L, B


@pytest.mark.parametrize("name", sorted(CASES))
def test_ternary_matches_brute(name):
    kind, shape, bc, wu = CASES[name]
    L, B = _pair(kind, shape, bc, np.asarray(wu, float))
    L.step(100)
    B.step(100)
    for a, b in zip(L.populations(), B.populations()):
        assert np.abs(a - b).max() < 1e-13
    a, b = L.observe(), B.observe()
    for k in b:
        assert np.abs(a[k] - b[k]).max() < 1e-13, k


def test_ternary_matches_brute_roller():
    mask = np.zeros((1, 10, 10), np.uint8)
    mask[0, 2:4, 2:4] = 2
    mask[0, 6, 6] = 1
    L, B = _pair(0, (10, 10, 1), (0, 0, 0), None, mask=mask, rollers=[((2.5, 2.5, 0.0), 0.01, 2)])
    L.step(100)
    B.step(100)
    for a, b in zip(L.populations(), B.populations()):
        assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("kind,shape,bc", [(0, (12, 10, 1), (0, 1, 0)), (1, (10, 8, 6), (0, 0, 1))])
def test_reduces_to_binary_without_third_component(kind, shape, bc):
    wu = np.zeros((3, 2, 3)); wu[bc.index(1), 0, 0] = -0.01; wu[bc.index(1), 1, 0] = 0.01
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    phi0 = synth.droplet_phi(sh, 3.0, 1.2, noise=1e-3, dims=3 if kind else 2)
    rho0 = 1 + 0.01 * synth.smooth_random_field(sh, 2)
    u0 = 0.005 * np.stack([synth.smooth_random_field(sh, 7 + a) for a in range(3)])
    if kind == 0:
        u0[2] = 0
    p = O.make_params(kind, shape, bc=bc, wall_u=wu, **KW)
    b = O.Lattice(p, phi0, rho0, u0).step(200)
    t = O.Lattice3(p, 0.3, 0.0, 1.0, phi0, np.zeros(sh), rho0, u0).step(200)
    fb, gb = b.populations()
    ft, gt, ht = t.populations()
    assert np.abs(fb - ft).max() < 1e-12 and np.abs(gb - gt).max() < 1e-12
    assert not ht.any()
    ob, ot = b.observe(), t.observe()
    assert not ot["psi"].any()
    for k in ("rho", "phi", "ux", "uy", "uz", "mu_rho", "mu_phi", "P"):
        assert np.abs(ob[k] - ot[k]).max() < 1e-12, k


def test_mu3_is_the_derivative_of_the_bulk_density():
    k1, k2, k3, al = 0.2, 0.13, 0.27, 0.9
    h = 1e-6
    rng = np.random.default_rng(3)
    for _ in range(10):
        r, p, s = 1 + rng.uniform(-0.05, 0.05), rng.uniform(-1, 1), rng.uniform(0, 1)
        m = O.mu3(k1, k2, k3, al, r, p, s, 0.0, 0.0, 0.0)
        for a, d in enumerate(np.eye(3)):
            x1 = np.array([r, p, s]) + h * d
            x0 = np.array([r, p, s]) - h * d
            fd = (O.psi_bulk3(k1, k2, k3, *x1) - O.psi_bulk3(k1, k2, k3, *x0)) / (2 * h)
            assert abs(m[a] - fd) < 1e-9, (a, m[a], fd)
    # bulk phases: pure components are minima (all potentials vanish)
    for C in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        r, p, s = C[0] + C[1] + C[2], C[0] - C[1], C[2]
        assert max(abs(v) for v in O.mu3(k1, k2, k3, al, r, p, s, 0, 0, 0)) < 1e-15


def _lap(X, c, w):
    out = np.zeros_like(X)
    for i in range(1, len(w)):
        out += w[i] * (np.roll(X, (-c[i][2], -c[i][1], -c[i][0]), axis=(0, 1, 2)) - X)
    return 6.0 * out


def test_potentials_are_the_derivatives_of_the_discrete_functional():
    # E = sum_x [bulk density] - sum_m alpha^2 kappa_m / 2 sum_x C_m (L C_m)
    # with L the lattice Laplacian (symmetric), so dE/dC_m(x) carries
    # -alpha^2 kappa_m (L C_m)(x): the chain rule then gives mu_rho, mu_phi,
    # mu_psi.  A periodic lattice, no solids.
    kind, shape = 0, (7, 6, 1)
    k1, k2, al = 0.16, 0.12, 1.0
    k3 = 0.2
    phi0, psi0, rho0, _ = _fields(kind, shape, seed=1)
    c, w = O.tables(kind)
    p = O.make_params(kind, shape, kappa1=k1, kappa2=k2, alpha=al)
    obs = O.Lattice3(p, k3, 0.05, 1.0, phi0, psi0, rho0).observe()

    def energy(r, f, s):
        C = (0.5 * (r + f - s), 0.5 * (r - f - s), s)
        e = sum(O.psi_bulk3(k1, k2, k3, a, b, d) for a, b, d in zip(r.ravel(), f.ravel(), s.ravel()))
        for k, Cm in zip((k1, k2, k3), C):
            e -= al * al * k / 2 * np.sum(Cm * _lap(Cm, c, w))
        return e

    h = 1e-5
    for cell in ((0, 2, 3), (0, 5, 6), (0, 0, 0)):
        for name, idx in (("mu_rho", 0), ("mu_phi", 1), ("mu_psi", 2)):
            F = [rho0.copy(), phi0.copy(), psi0.copy()]
            F[idx][cell] += h
            ep = energy(*F)
            F[idx][cell] -= 2 * h
            em = energy(*F)
            fd = (ep - em) / (2 * h)
            assert abs(obs[name][cell] - fd) < 1e-8, (name, cell, obs[name][cell], fd)


def test_conservation_with_moving_walls():
    kind, shape, bc = 1, (12, 10, 8), (0, 0, 1)
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -0.01; wu[2, 1, 0] = 0.01
    phi0, psi0, rho0, u0 = _fields(kind, shape, seed=2)
    L = O.Lattice3(O.make_params(kind, shape, bc=bc, wall_u=wu, **KW), 0.2, 0.07, 0.9, phi0, psi0, rho0, u0)
    o0 = L.observe()
    s0 = {k: o0[k].sum() for k in ("rho", "phi", "psi")}
    a0 = {k: np.abs(o0[k]).sum() for k in ("rho", "phi", "psi")}
    L.step(500)
    o1 = L.observe()
    for k in ("rho", "phi", "psi"):
        assert abs(o1[k].sum() - s0[k]) / a0[k] < 1e-12, k


def test_laplace_law_of_a_pair():
    # a drop of component 1 (C1 = 1) in component 3 (C3 = 1), C2 = 0:
    # Delta p = gamma_13 / R with gamma_13 = alpha (kappa1 + kappa3) / 6; here
    # kappa3 = 0.1 makes gamma_13 19% below the (1, 2) tension.  With
    # M_psi = M / 3 a pair with C2 = 0 evolves as the binary system would
    # (dC3/dt = -dC1/dt), so C2 stays near zero while the drop settles.
    n, R, A = 100, 20.0, 0.04
    xi = 1.5
    al = xi / math.sqrt(2.0)
    k1 = k2 = 4 * A
    k3 = 0.1
    sh = (1, n, n)
    c1 = 0.5 * (1 + synth.droplet_phi(sh, R, xi, center=(49.5, 49.5, 0), dims=2))
    p = O.make_params(0, (n, n, 1), kappa1=k1, kappa2=k2, alpha=al, tau_f=1.0, tau_g=1.0, M=0.1)
    L = O.Lattice3(p, k3, 0.1 / 3, 1.0, c1, 1 - c1).step(6000)
    o = L.observe()
    dp = o["P"][0, 49:51, 49:51].mean() - o["P"][0, 0, 0]
    g13, g12 = al * (k1 + k3) / 6, al * (k1 + k2) / 6
    assert abs(dp / (g13 / R) - 1) < 0.03, dp / (g13 / R)
    assert abs(dp / (g12 / R) - 1) > 0.15
    c2 = 0.5 * (o["rho"] - o["phi"] - o["psi"])
    assert np.abs(c2).max() < 2e-3
    assert np.hypot(o["ux"], o["uy"]).max() < 1e-4


def _pair_profile(C0, al):
    """Newton solution of C(1 - C)(1 - 2C) - alpha^2 (C[x+1] - 2C[x] + C[x-1])
    = g (g unknown, uniform) on a periodic 1D lattice, with sum C fixed."""
    n = C0.size
    C, g = C0.copy(), 0.0
    for _ in range(80):
        lap = np.roll(C, 1) + np.roll(C, -1) - 2 * C
        R = C * (1 - C) * (1 - 2 * C) - al * al * lap - g
        J = np.diag((1 - 6 * C + 6 * C * C) + 2 * al * al) - al * al * (np.eye(n, k=1) + np.eye(n, k=-1))
        J[0, -1] -= al * al
        J[-1, 0] -= al * al
        Jf = np.zeros((n + 1, n + 1))
        Jf[:n, :n] = J
        Jf[:n, n] = -1.0
        Jf[n, :n] = 1.0
        d = np.linalg.solve(Jf, -np.append(R, C.sum() - C0.sum()))
        C += d[:n]
        g += d[n]
        if np.abs(d).max() < 1e-15:
            break
    return C


def test_flat_interface_of_every_pair():
    k1, k2, k3, al, M, n = 0.05, 0.04, 0.06, 1.5, 0.3, 64
    x = np.arange(n)
    slab = 0.5 * (1 + np.tanh((n / 4 - np.abs(x - (n - 1) / 2)) / (2 * al)))
    got = {}
    for m, q in ((0, 1), (0, 2), (1, 2)):
        C = [np.zeros(n) for _ in range(3)]
        C[m], C[q] = slab.copy(), 1 - slab
        rho, phi, psi = C[0] + C[1] + C[2], C[0] - C[1], C[2]
        sh = (1, 1, n)
        p = O.make_params(0, (n, 1, 1), kappa1=k1, kappa2=k2, alpha=al, tau_f=1.0, tau_g=1.0, M=M)
        L = O.Lattice3(p, k3, M, 1.0, phi.reshape(sh), psi.reshape(sh), rho.reshape(sh)).step(80000)
        o = L.observe()
        c = (0.5 * (o["rho"] + o["phi"] - o["psi"]).ravel(), 0.5 * (o["rho"] - o["phi"] - o["psi"]).ravel(),
             o["psi"].ravel())
        absent = c[3 - m - q]
        assert max(np.ptp(o[k]) for k in ("mu_rho", "mu_phi", "mu_psi")) < 5e-7, (m, q)
        assert np.abs(absent).max() < 3e-6, (m, q, np.abs(absent).max())
        assert np.abs(c[m] - _pair_profile(slab, al)).max() < 5e-6, (m, q)
        assert np.abs(c[m] - slab).max() < 5e-3          # the continuum profile, to the lattice error
        assert np.abs(o["ux"]).max() < 1e-9
        got[(m, q)] = c[m]
    vals = list(got.values())
    assert max(np.abs(a - b).max() for a in vals for b in vals) < 5e-6


def test_population_hand_over_continues_the_run():
    # the state between steps is the post-stream populations: a lattice made
    # from other fields that takes over another's populations continues its
    # run exactly (moving walls and a solid box, which keeps its own cells)
    kind, shape, bc = 1, (12, 10, 8), (0, 0, 1)
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -0.01; wu[2, 1, 0] = 0.01
    mask = np.zeros((8, 10, 12), np.uint8); mask[3:5, 4:6, 2:4] = 1
    phi0, psi0, rho0, u0 = _fields(kind, shape, seed=3)
    p = O.make_params(kind, shape, bc=bc, wall_u=wu, **KW)
    whole = O.Lattice3(p, 0.2, 0.07, 0.9, phi0, psi0, rho0, u0, mask).step(120)
    first = O.Lattice3(p, 0.2, 0.07, 0.9, phi0, psi0, rho0, u0, mask).step(60)
    other = _fields(kind, shape, seed=4)
    second = O.Lattice3(p, 0.2, 0.07, 0.9, *other, mask)
    pops = first.populations()
    second.set_populations(*pops)
    for a, b in zip(second.populations(), pops):
        assert np.array_equal(a, b)
    second.step(60)
    for a, b in zip(second.populations(), whole.populations()):
        assert np.array_equal(a, b)
    ow, os_ = whole.observe(), second.observe()
    for k in ("rho", "phi", "psi", "ux", "mu_psi", "P"):
        assert np.array_equal(ow[k], os_[k]), k
