"""P3: the oracle's Laplacian and gradient stencils (with the solid fill).

Closed forms: exact on quadratics; on axis-aligned cos(kx) the Laplacian is
-4 sin^2(k/2) cos(kx) and the gradient of sin(kx) is sin(k) cos(kx), for both
velocity sets.  At walls the fluid-neighbour-mean fill keeps constants and
fields linear along the wall exact.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2212_01617_amd import synth


def _lat(kind, shape, bc=(0, 0, 0), mask=None):
    p = O.make_params(kind, shape, bc=bc, A=0.04, kappa=0.09)
    sh = (shape[2], shape[1], shape[0])
    return O.Lattice(p, np.zeros(sh), mask=mask), sh


@pytest.mark.parametrize("kind", [0, 1])
def test_quadratic_exact(kind):
    shape = (12, 10, 1) if kind == 0 else (10, 9, 8)
    L, sh = _lat(kind, shape)
    x, y, z = synth.grid(sh)
    X = 0.3 * x * x - 0.2 * x * y + 0.1 * y * y + (0.05 * z * z + 0.07 * y * z if kind else 0) + x
    lap, grad = L.stencils(X)
    inner = (slice(2, -2) if kind else slice(None), slice(2, -2), slice(2, -2))
    exp_lap = 0.6 + 0.2 + (0.1 if kind else 0.0)
    assert np.abs(lap[inner] - exp_lap).max() < 1e-12
    assert np.abs(grad[0][inner] - (0.6 * x - 0.2 * y + 1)[inner]).max() < 1e-12
    assert np.abs(grad[1][inner] - (-0.2 * x + 0.2 * y + (0.07 * z if kind else 0))[inner]).max() < 1e-12


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fourier_symbols(kind, axis):
    if kind == 0 and axis == 2:
        pytest.skip("2D")
    n = 16
    shape = (n, n, 1 if kind == 0 else n)
    L, sh = _lat(kind, shape)
    coords = synth.grid(sh)
    k = 2 * math.pi * 3 / n
    X = np.cos(k * coords[axis])
    lap, _ = L.stencils(X)
    assert np.abs(lap - (-4 * math.sin(k / 2) ** 2) * X).max() < 1e-13
    _, grad = L.stencils(np.sin(k * coords[axis]))
    assert np.abs(grad[axis] - math.sin(k) * np.cos(k * coords[axis])).max() < 1e-13
    for b in range(3):
        if b != axis:
            assert np.abs(grad[b]).max() < 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_wall_fill_keeps_constant_and_tangential_linear(kind):
    shape = (8, 8, 1) if kind == 0 else (8, 8, 6)
    wall_axis = 1 if kind == 0 else 2
    bc = [0, 0, 0]
    bc[wall_axis] = 1
    L, sh = _lat(kind, shape, bc=tuple(bc))
    lap, grad = L.stencils(np.full(sh, 0.7))
    assert np.abs(lap).max() < 1e-15 and np.abs(grad).max() < 1e-15
    x, y, z = synth.grid(sh)
    lap, grad = L.stencils(0.25 * x - 1.0)  # linear along the wall, periodic-free window
    interior_x = slice(2, -2)  # the fills at x = 0, n-1 see the periodic wrap
    assert np.abs(lap[..., interior_x]).max() < 1e-14
    assert np.abs(grad[0][..., interior_x] - 0.25).max() < 1e-14


def test_solid_fill_is_fluid_neighbour_mean():
    # one solid cell in a periodic D2Q9 lattice: the Laplacian at its right
    # neighbour uses the solid's filled value = w-weighted mean of the
    # solid's fluid neighbours
    shape = (7, 7, 1)
    mask = np.zeros((1, 7, 7), np.uint8)
    mask[0, 3, 3] = 1
    L, sh = _lat(0, shape, mask=mask)
    rng = np.random.default_rng(0)
    X = rng.uniform(size=sh)
    c, w = O.tables(0)
    num = sum(w[i] * X[0, 3 + c[i][1], 3 + c[i][0]] for i in range(1, 9))
    fill = num / sum(w[1:])
    lap, _ = L.stencils(X)
    y0, x0 = 3, 4
    acc = 0.0
    for i in range(1, 9):
        yy, xx = (y0 + c[i][1]) % 7, (x0 + c[i][0]) % 7
        v = fill if (yy, xx) == (3, 3) else X[0, yy, xx]
        acc += w[i] * (v - X[0, y0, x0])
    assert abs(lap[0, y0, x0] - 6 * acc) < 1e-15
