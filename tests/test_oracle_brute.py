"""P9: the C oracle against the independent NumPy transcription on tiny
lattices with moving walls, a roller and random smooth fields, 100 steps."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.brute import Brute
from paper_2212_01617_amd import synth


def _case(kind, shape, bc, wall_u, mask=None, rollers=()):
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    phi0 = synth.droplet_phi(sh, 2.5, 1.2, noise=1e-3, dims=3 if kind else 2) \
        + 0.05 * synth.smooth_random_field(sh, 21)
    rho0 = 1.0 + 0.01 * synth.smooth_random_field(sh, 3)
    u0 = 0.01 * np.stack([synth.smooth_random_field(sh, 5 + a) for a in range(3)])
    if kind == 0:
        u0[2] = 0
    kw = dict(kappa1=0.16, kappa2=0.12, alpha=1.0, tau_f=0.8, tau_g=1.1, M=0.1)
    L = O.Lattice(O.make_params(kind, shape, bc=bc, wall_u=wall_u, rollers=rollers, **kw),
                  phi0, rho0, u0, mask)
    B = Brute(kind, shape, phi0, rho0, u0, mask, bc=bc, wall_u=wall_u, rollers=rollers, **kw)
    return L, B


CASES = {
    "d2q9_walls": (0, (8, 8, 1), (0, 1, 0), [[[0] * 3] * 2, [[-0.01, 0, 0], [0.01, 0, 0]], [[0] * 3] * 2]),
    "d3q19_walls": (1, (8, 8, 8), (0, 0, 1), [[[0] * 3] * 2, [[0] * 3] * 2, [[-0.01, 0, 0], [0.02, 0.005, 0]]]),
    "d3q19_box": (1, (8, 6, 7), (1, 0, 1), np.random.default_rng(0).uniform(-0.01, 0.01, (3, 2, 3))),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_matches_brute(name):
    kind, shape, bc, wu = CASES[name]
    L, B = _case(kind, shape, bc, np.asarray(wu, float))
    L.step(100)
    B.step(100)
    fa, ga = L.populations()
    fb, gb = B.populations()
    assert np.abs(fa - fb).max() < 1e-13
    assert np.abs(ga - gb).max() < 1e-13
    a, b = L.observe(), B.observe()
    for k in b:
        assert np.abs(a[k] - b[k]).max() < 1e-13, k


def test_oracle_matches_brute_roller():
    mask = np.zeros((1, 10, 10), np.uint8)
    mask[0, 2:4, 2:4] = 2
    mask[0, 6, 6] = 1
    L, B = _case(0, (10, 10, 1), (0, 0, 0), None, mask=mask, rollers=[((2.5, 2.5, 0.0), 0.01, 2)])
    L.step(100)
    B.step(100)
    fa, ga = L.populations()
    fb, gb = B.populations()
    assert np.abs(fa - fb).max() < 1e-13 and np.abs(ga - gb).max() < 1e-13
