"""Pins of the oracle's lattice tables and per-node formulas (CPU).

P1: velocity-set tables against exact rationals and isotropy identities.
P2: moment identities of f^eq (eq. feq), the Guo term (eq. Fi) and g^eq
    (eq. geq) for random states -- a dropped term, a wrong sign or a wrong
    weight in any of them breaks one of these sums.
mu: the chemical potentials (eqs. mu_rho, mu_phi) against the closed forms of
    the symmetric case, where they reduce to A(phi^3-phi) - kappa lap phi.
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("kind,name", [(0, "D2Q9"), (1, "D3Q19")])
def test_tables_match_golden_rationals(kind, name):
    c, w = O.tables(kind)
    g = GOLD["lattice"][name]
    assert c.tolist() == g["c"]
    for wi, num in zip(w, g["w_num"]):
        assert Fraction(wi).limit_denominator(1000) == Fraction(num, g["w_den"])


@pytest.mark.parametrize("kind", [0, 1])
def test_tables_isotropy(kind):
    c, w = O.tables(kind)
    d = 2 if kind == 0 else 3
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-15
    I = np.eye(3)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2[:d, :d], cs2 * I[:d, :d], atol=1e-15)
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(M3).max() < 1e-15
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    for a, b, cc, dd in itertools.product(range(d), repeat=4):
        ref = cs2 ** 2 * (I[a, b] * I[cc, dd] + I[a, cc] * I[b, dd] + I[a, dd] * I[b, cc])
        assert abs(M4[a, b, cc, dd] - ref) < 1e-15
    # opposites adjacent: c_opp(i) = -c_i with opp = i+1 for odd i
    for i in range(1, len(w)):
        j = i + 1 if i % 2 else i - 1
        assert (c[j] == -c[i]).all() and w[j] == w[i]


def _rand_states(kind, n=20, seed=7):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        u = rng.uniform(-0.08, 0.08, 3)
        F = rng.uniform(-1e-3, 1e-3, 3)
        if kind == 0:
            u[2] = F[2] = 0.0
        yield (rng.uniform(0.8, 1.2), rng.uniform(-1.1, 1.1), rng.uniform(-0.05, 0.05),
               rng.uniform(0.1, 5.0), rng.uniform(0.55, 2.0), u, F)


@pytest.mark.parametrize("kind", [0, 1])
def test_feq_moments(kind):
    c, w = O.tables(kind)
    d = 2 if kind == 0 else 3
    for rho, phi, mu, G, tau, u, F in _rand_states(kind):
        fe = O.feq(kind, rho, u)
        assert abs(fe.sum() - rho) < 1e-14
        assert np.abs(c.T @ fe - rho * u).max() < 1e-15
        P = np.einsum("i,ia,ib->ab", fe, c, c)
        ref = rho * (np.eye(3) / 3.0 + np.outer(u, u))
        assert np.abs(P[:d, :d] - ref[:d, :d]).max() < 1e-15


@pytest.mark.parametrize("kind", [0, 1])
def test_guo_moments(kind):
    c, w = O.tables(kind)
    d = 2 if kind == 0 else 3
    for rho, phi, mu, G, tau, u, F in _rand_states(kind):
        S = O.guo(kind, tau, u, F)
        k = 1.0 - 1.0 / (2.0 * tau)
        assert abs(S.sum()) < 1e-17
        assert np.abs(c.T @ S - k * F).max() < 1e-17
        P = np.einsum("i,ia,ib->ab", S, c, c)
        ref = k * (np.outer(u, F) + np.outer(F, u))
        assert np.abs(P[:d, :d] - ref[:d, :d]).max() < 1e-17


@pytest.mark.parametrize("kind", [0, 1])
def test_geq_moments(kind):
    c, w = O.tables(kind)
    d = 2 if kind == 0 else 3
    for rho, phi, mu, G, tau, u, F in _rand_states(kind):
        ge = O.geq(kind, phi, mu, G, u)
        assert abs(ge.sum() - phi) < 1e-14
        assert np.abs(c.T @ ge - phi * u).max() < 1e-15
        P = np.einsum("i,ia,ib->ab", ge, c, c)
        ref = G * mu * np.eye(3) + phi * np.outer(u, u)
        assert np.abs(P[:d, :d] - ref[:d, :d]).max() < 1e-14


def test_mu_symmetric_closed_form():
    # kappa1 = kappa2 = 4A, alpha^2 = kappa/(2A), rho = 1:
    #   mu_phi = A (phi^3 - phi) - kappa lap(phi),  mu_rho = -kappa lap(rho) (+0 bulk)
    A, kappa = 0.04, 0.09
    k1, k2, al = O.paper_form(A, kappa)
    rng = np.random.default_rng(3)
    for _ in range(50):
        phi, lp, lr = rng.uniform(-1.2, 1.2), rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1)
        mr, mp = O.mu(k1, k2, al, 1.0, phi, lr, lp)
        assert abs(mp - (A * (phi ** 3 - phi) - kappa * lp)) < 1e-15
        assert abs(mr - (-kappa * lr)) < 1e-15


def test_mu_general_form_derivative_of_functional():
    # mu_rho, mu_phi are the partial derivatives of the bulk free-energy
    # density of eq. (functional): check against a central difference of it.
    k1, k2, al = 0.2, 0.13, 0.9
    def psi(r, p):
        s, t = r + p, r - p
        return k1 / 32 * s * s * (s - 2) ** 2 + k2 / 32 * t * t * (t - 2) ** 2
    h = 1e-6
    for r, p in [(1.0, 0.3), (0.95, -0.8), (1.1, 1.05)]:
        mr, mp = O.mu(k1, k2, al, r, p, 0.0, 0.0)
        assert abs(mr - (psi(r + h, p) - psi(r - h, p)) / (2 * h)) < 1e-9
        assert abs(mp - (psi(r, p + h) - psi(r, p - h)) / (2 * h)) < 1e-9
    # gradient terms: mu_phi gains -alpha^2/4 [(k1+k2) lap phi - (k2-k1) lap rho]
    m0 = O.mu(k1, k2, al, 1.0, 0.2, 0.0, 0.0)
    m1 = O.mu(k1, k2, al, 1.0, 0.2, 0.01, 0.02)
    assert abs((m1[1] - m0[1]) - al ** 2 / 4 * (-(k1 + k2) * 0.02 + (k2 - k1) * 0.01)) < 1e-16
    assert abs((m1[0] - m0[0]) - al ** 2 / 4 * (-(k1 + k2) * 0.01 + (k2 - k1) * 0.02)) < 1e-16


def test_paper_form_interface_and_tension():
    g = GOLD["static_droplet_2d"]
    k1, k2, al = O.paper_form(g["A"], g["kappa"])
    # xi = sqrt(2) alpha, sigma = alpha (k1 + k2) / 6
    assert abs(np.sqrt(2) * al - g["xi"]) < 1e-14
    assert abs(al * (k1 + k2) / 6 - g["sigma"]) < 1e-14
