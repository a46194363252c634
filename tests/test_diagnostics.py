"""Host diagnostics against analytic shapes: ellipses and ellipsoids of known
axes and tilt (area-fraction sampled), periodic wrap, component counting,
pressure jump and the steady-state test."""
import math

import numpy as np
import pytest

from paper_2212_01617_amd import diagnostics as Dg


def _area_fraction(shape, inside, sub=6):
    """Fraction of each cell (centres at integer coordinates) inside a shape,
    by sub x sub (x sub) point sampling.  shape = (nz, ny, nx)."""
    nz, ny, nx = shape
    o = (np.arange(sub) + 0.5) / sub - 0.5
    C = np.zeros(shape)
    zs = o if nz > 1 else np.zeros(1)
    for dz in zs:
        for dy in o:
            for dx in o:
                z, y, x = np.meshgrid(np.arange(nz) + dz, np.arange(ny) + dy, np.arange(nx) + dx, indexing="ij")
                C += inside(x, y, z)
    return C / (len(zs) * sub * sub)


def _ellipse(shape, centre, a, b, theta, plane=(0, 1), periodic=True):
    """Phase field of an ellipse (semi-axes a, b, long axis tilted by theta
    from plane axis 0 towards plane axis 1), phi = 2C - 1."""
    n = (shape[2], shape[1], shape[0])  # extents along x, y, z

    def inside(x, y, z):
        pos = [x, y, z]
        u = pos[plane[0]] - centre[plane[0]]
        v = pos[plane[1]] - centre[plane[1]]
        if periodic:
            u = (u + n[plane[0]] / 2) % n[plane[0]] - n[plane[0]] / 2
            v = (v + n[plane[1]] / 2) % n[plane[1]] - n[plane[1]] / 2
        ct, st = math.cos(theta), math.sin(theta)
        p, q = ct * u + st * v, -st * u + ct * v
        return ((p / a) ** 2 + (q / b) ** 2 <= 1.0).astype(float)

    return 2.0 * _area_fraction(shape, inside) - 1.0


def test_ellipse_deformation_and_angle():
    phi = _ellipse((1, 128, 160), (80.3, 60.7, 0.0), 30.0, 15.0, 0.5)
    d = Dg.deformation(phi, plane="xy")
    assert abs(d.D - 1.0 / 3.0) < 2e-3, d
    assert abs(d.theta - 0.5) < 5e-3, d
    assert abs(d.L / d.B - 2.0) < 1e-2


def test_ellipse_negative_tilt_and_circle():
    phi = _ellipse((1, 100, 100), (50.0, 50.0, 0.0), 24.0, 20.0, -0.3)
    d = Dg.deformation(phi, plane="xy")
    assert abs(d.D - 4.0 / 44.0) < 2e-3 and abs(d.theta + 0.3) < 1e-2
    circ = _ellipse((1, 100, 100), (49.5, 49.5, 0.0), 20.0, 20.0, 0.0)
    assert Dg.deformation(circ, plane="xy").D < 1e-3


def test_ellipse_across_periodic_boundary():
    # the same ellipse centred on the x seam and the y seam
    ref = Dg.deformation(_ellipse((1, 128, 160), (80.0, 64.0, 0.0), 30.0, 15.0, 0.4), plane="xy")
    wrapped = Dg.deformation(_ellipse((1, 128, 160), (1.0, 126.5, 0.0), 30.0, 15.0, 0.4), plane="xy")
    assert abs(wrapped.D - ref.D) < 1e-3 and abs(wrapped.theta - ref.theta) < 2e-3


def test_obstacles_are_left_out_of_the_droplet():
    # an ellipse (D = 1/3) among four solid discs whose phi reads 0, as the
    # readback gives for obstacle cells: with the solid mask D is the
    # ellipse's; without it the discs (indicator 0.5) swamp the moments
    n = 160
    phi = _ellipse((1, n, n), (80.0, 80.0, 0.0), 24.0, 12.0, 0.0)
    z, y, x = np.meshgrid(np.arange(1), np.arange(n), np.arange(n), indexing="ij")
    solid = np.zeros(phi.shape, dtype=bool)
    for cx, cy in ((40, 40), (120, 40), (40, 120), (120, 120)):
        solid |= (x - cx) ** 2 + (y - cy) ** 2 <= 19.0 ** 2
    assert not (solid & (phi > -1.0)).any()
    ref = Dg.deformation(phi, plane="xy")
    with_obstacles = np.where(solid, 0.0, phi)
    d = Dg.deformation(with_obstacles, plane="xy", periodic=(True, True, True), solid=solid)
    assert abs(d.D - ref.D) < 1e-12 and abs(d.theta - ref.theta) < 1e-12
    assert abs(d.D - 1.0 / 3.0) < 2e-3
    assert Dg.deformation(with_obstacles, plane="xy").D < 0.5 * ref.D
    assert Dg.components(with_obstacles) == Dg.components(phi)


def test_ellipsoid_in_shear_plane():
    # semi-axes 20 (tilted in xz), 12 (along y), 10 (in xz): D in xz = 1/3
    shape = (48, 40, 72)
    c = (36.2, 19.5, 23.8)
    th = 0.35

    def inside(x, y, z):
        u, v, w = x - c[0], y - c[1], z - c[2]
        p, q = math.cos(th) * u + math.sin(th) * w, -math.sin(th) * u + math.cos(th) * w
        return ((p / 20.0) ** 2 + (v / 12.0) ** 2 + (q / 10.0) ** 2 <= 1.0).astype(float)

    phi = 2.0 * _area_fraction(shape, inside, sub=4) - 1.0
    d = Dg.deformation(phi, plane="xz", periodic=(True, True, False))
    assert abs(d.D - 1.0 / 3.0) < 3e-3, d
    assert abs(d.theta - th) < 1e-2, d


def test_components_periodic_and_connectivity():
    phi = -np.ones((1, 40, 60))
    phi[0, 5:15, 10:20] = 1.0              # block A
    phi[0, 25:35, 30:40] = 1.0             # block B
    assert Dg.components(phi) == [100, 100]
    assert Dg.broken_up(phi)
    # a block cut by the x seam is one component when x is periodic
    w = -np.ones((1, 40, 60))
    w[0, 10:20, :5] = 1.0
    w[0, 10:20, 55:] = 1.0
    assert Dg.components(w) == [100]
    assert Dg.components(w, periodic=(False, True, True)) == [50, 50]
    # diagonal contact does not connect (face connectivity); small bits dropped
    d = -np.ones((1, 20, 20))
    d[0, 2:6, 2:6] = 1.0
    d[0, 6:10, 6:10] = 1.0
    d[0, 15, 15] = 1.0
    assert Dg.components(d) == [16, 16]
    one = -np.ones((1, 20, 20))
    one[0, 3:9, 3:12] = 1.0
    assert not Dg.broken_up(one)
    # 3D: a droplet through the z seam, z periodic vs walls
    v = -np.ones((10, 8, 8))
    v[:2, 2:5, 2:5] = 1.0
    v[8:, 2:5, 2:5] = 1.0
    assert Dg.components(v) == [36]
    assert Dg.components(v, periodic=(True, True, False)) == [18, 18]


def test_laplace_jump_volume_and_drift():
    phi = -np.ones((1, 30, 30))
    phi[0, 10:20, 10:20] = 1.0
    phi[0, 9, 10:20] = 0.0                 # interface cells are excluded
    P = np.where(phi > 0.5, 0.0125, 0.0025)
    assert Dg.laplace_jump(P, phi) == pytest.approx(0.01, abs=1e-15)
    v = Dg.droplet_volume(phi)
    assert v["cells_phi_pos"] == 100 and v["indicator_sum"] == pytest.approx(105.0)


def test_indicator_references_the_bulk_phases():
    # a drop in a matrix that has taken up some of its volume (phi_out > -1)
    # and with a drop phase below +1: same D and theta as the ideal field
    ideal = _ellipse((1, 96, 192), (96.0, 48.0, 0.0), 20.0, 12.0, 0.6)
    shifted = 0.5 * (ideal + 1.0) * (0.93 - (-0.95)) + (-0.95)
    a = Dg.deformation(ideal, plane="xy")
    b = Dg.deformation(shifted, plane="xy")
    assert abs(a.D - b.D) < 1e-9 and abs(a.theta - b.theta) < 1e-9
    assert abs(a.D - 8.0 / 32.0) < 3e-3
    # the old (1 + phi)/2 indicator would see the matrix as 2.5% drop phase
    naive = np.clip(0.5 * (1.0 + shifted), 0.0, 1.0)
    cen, T = Dg.second_moments(naive)
    assert T[0, 0] > 1.2 * Dg.second_moments(Dg.indicator(shifted))[1][0, 0]
    dr = Dg.mass_drift([100.0, 2.0, 50.0], [100.001, 2.0005, 50.0])
    assert dr["rho"] == pytest.approx(1e-5) and dr["phi"] == pytest.approx(1e-5)


def test_steady_tracker():
    t = Dg.SteadyTracker(dt=0.1, window=2.0, tol=5e-4)
    s = 0.0
    steady_at = None
    for k in range(60):
        s = 0.1 * (k + 1)
        D = 0.2 * (1.0 - math.exp(-s / 0.5))   # relaxes to 0.2
        if t.add(s, D) and steady_at is None:
            steady_at = s
    assert steady_at is not None and 2.0 <= steady_at <= 6.0
    o = Dg.SteadyTracker(dt=0.1, window=2.0, tol=5e-4)
    assert not any(o.add(0.1 * (k + 1), 0.2 + 1e-3 * math.sin(k)) for k in range(60))


def test_plane_sum_moments_equal_the_direct_form():
    """centred_moments (from the three plane sums) against second_moments of
    the rolled indicator, on random fields and periodicities, 2D and 3D."""
    rng = np.random.default_rng(11)
    for trial in range(30):
        nz = 1 if trial % 3 == 0 else int(rng.integers(2, 30))
        ny, nx = (int(v) for v in rng.integers(2, 40, 2))
        C = rng.uniform(0.0, 1.0, (nz, ny, nx)) ** 4
        per = tuple(bool(v) for v in rng.integers(0, 2, 3))
        c0, T0 = Dg.second_moments(Dg.centred(C, per)[0])
        c1, T1 = Dg.centred_moments(C, per)
        assert np.allclose(c1, c0, rtol=0, atol=1e-9 * (1 + np.abs(c0).max()))
        assert np.allclose(T1, T0, rtol=0, atol=1e-9 * np.abs(T0).max())
