"""Parity of the GPU ternary lattice (a third order parameter psi with its own
population h: Sec. 2.2, Remark after the mobility relation) with the
oracle's ternary step, through the C ABI.

* D2Q9 periodic with a ragged row (70 x 37), D2Q9 with moving walls, a solid
  box and a roller, D3Q19 with moving walls and a box: every field and every
  population of f, g and h against the FP64 oracle;
* with psi = 0 and no psi mobility the ternary lattice keeps psi and h at
  exactly zero and follows the binary lattice of the same parameters;
* captured-graph stepping is bitwise the launch-by-launch stepping, and a
  checkpoint restores the run bitwise;
* the entry points a ternary lattice does not support refuse it."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth

from _pair import ensure_gpu_lib, log

pytestmark = pytest.mark.gpu

KW = dict(kappa1=0.16, kappa2=0.12, alpha=1.0, tau_f=0.8, tau_g=1.1, M=0.1)
K3 = (0.2, 0.07, 0.9)  # kappa3, M3, tau_h
TOL = {"rho": 1e-5, "phi": 1e-5, "psi": 1e-5, "u": 1e-5, "mu_rho": 2e-6, "mu_phi": 2e-6, "mu_psi": 2e-6, "P": 2e-6}
POP_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _fields(kind, shape, radius, seed=0):
    """Component 1 drop in a mixture of 2 and 3; (phi, psi, rho, u)."""
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    c1 = 0.5 * (1 + synth.droplet_phi(sh, radius, 1.5, dims=3 if kind else 2))
    c3 = 0.3 * (1 - c1) + 0.02 * synth.smooth_random_field(sh, 4 + seed)
    c2 = 1 - c1 - c3
    rho0 = 1 + 0.01 * synth.smooth_random_field(sh, 3 + seed)
    u0 = 0.01 * np.stack([synth.smooth_random_field(sh, 5 + a + seed) for a in range(3)])
    if kind == 0:
        u0[2] = 0
    return c1 - c2, c3, rho0, u0


def _pair(kind, shape, steps, *, bc=(0, 0, 0), wall_u=None, mask=None, rollers=(), radius=6.0, stream=None):
    phi0, psi0, rho0, u0 = _fields(kind, shape, radius)
    ref = O.Lattice3(O.make_params(kind, shape, bc=bc, wall_u=wall_u, rollers=[r[:3] for r in rollers], **KW),
                     *K3, phi0, psi0, rho0, u0, mask)
    ref.step(steps)
    p = F.make_params(kind, shape, bc=bc, wall_u=wall_u, rollers=rollers, ternary=K3, **KW)
    gpu = F.Lattice(p, phi0, rho0, u0, mask, psi0=psi0, stream=stream)
    gpu.step(steps)
    return ref, gpu


def _compare(name, ref, gpu, mask=None):
    o = ref.observe()
    g = gpu.read(tuple(TOL))
    fluid = np.ones(ref.shape, bool) if mask is None else (np.asarray(mask).reshape(ref.shape) == 0)
    err = {}
    for k in TOL:
        if k == "u":
            err[k] = max(np.abs(g["u"][a] - o["u" + "xyz"[a]])[fluid].max() for a in range(3))
        else:
            err[k] = np.abs(g[k] - o[k])[fluid].max()
    pe = [np.abs(a - b)[:, fluid].max() for a, b in zip(ref.populations(), gpu.populations())]
    log(f"[parity] ternary {name}: " + " ".join(f"{k}={v:.2e}" for k, v in err.items())
        + " f={:.2e} g={:.2e} h={:.2e}".format(*pe))
    for k, v in TOL.items():
        assert err[k] < v, (k, err[k])
    assert max(pe) < POP_TOL, pe
    # the third component is present and has moved
    assert np.abs(o["psi"]).max() > 0.1


def test_d2q9_periodic_ragged_row():
    ref, gpu = _pair(0, (70, 37, 1), 300, radius=9.0)
    _compare("d2q9_periodic_70x37_300", ref, gpu)


def test_d2q9_walls_box_roller():
    shape = (50, 40, 1)
    mask = np.zeros((1, 40, 50), np.uint8)
    mask[0, 5:9, 30:36] = 1
    mask[0, 25:29, 8:12] = 2
    wu = np.zeros((3, 2, 3))
    wu[1, 0, 0], wu[1, 1, 0] = -0.01, 0.01
    rollers = [((9.5, 26.5, 0.0), 0.004, 2, 2.0)]
    ref, gpu = _pair(0, shape, 200, bc=(0, 1, 0), wall_u=wu, mask=mask, rollers=rollers, radius=8.0)
    _compare("d2q9_walls_box_roller_200", ref, gpu, mask)


def test_d3q19_walls_box():
    shape = (40, 24, 20)
    mask = np.zeros((20, 24, 40), np.uint8)
    mask[3:6, 4:8, 30:35] = 1
    wu = np.zeros((3, 2, 3))
    wu[2, 0, 0], wu[2, 1, 0], wu[2, 1, 1] = -0.01, 0.015, 0.005
    ref, gpu = _pair(1, shape, 100, bc=(0, 0, 1), wall_u=wu, mask=mask, radius=6.0, stream=torch.cuda.Stream())
    _compare("d3q19_walls_box_100", ref, gpu, mask)


@pytest.mark.parametrize("kind,shape,steps", [(0, (1, 1, 1), 9), (0, (3, 2, 1), 7), (1, (2, 2, 2), 5),
                                              (1, (1, 3, 1), 4), (0, (9, 5, 1), 0)])
def test_degenerate_lattices_and_zero_steps(kind, shape, steps):
    """Lattices narrower than the stencil (every neighbour a periodic image
    of the cell or of another cell), odd and zero step counts."""
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    rng = np.random.default_rng(7)
    phi0 = rng.uniform(-0.8, 0.8, sh)
    psi0 = rng.uniform(0.0, 0.3, sh)
    rho0 = 1.0 + 0.01 * rng.uniform(-1, 1, sh)
    u0 = 0.01 * rng.uniform(-1, 1, (3,) + sh)
    if kind == 0:
        u0[2] = 0
    ref = O.Lattice3(O.make_params(kind, shape, **KW), *K3, phi0, psi0, rho0, u0)
    ref.step(steps)
    gpu = F.Lattice(F.make_params(kind, shape, ternary=K3, **KW), phi0, rho0, u0, psi0=psi0)
    gpu.step(steps)
    o, g = ref.observe(), gpu.read(tuple(TOL))
    err = {k: (max(np.abs(g["u"][a] - o["u" + "xyz"[a]]).max() for a in range(3)) if k == "u"
               else np.abs(g[k] - o[k]).max()) for k in TOL}
    pe = [np.abs(a - b).max() for a, b in zip(ref.populations(), gpu.populations())]
    log(f"[parity] ternary tiny{shape} t={steps}: " + " ".join(f"{k}={v:.2e}" for k, v in err.items()))
    for k, v in TOL.items():
        assert err[k] < v, (k, err[k])
    assert max(pe) < POP_TOL


def test_psi_zero_is_the_binary_lattice():
    shape = (48, 40, 1)
    phi0, _, rho0, u0 = _fields(0, shape, 9.0)
    psi0 = np.zeros_like(phi0)
    pb = F.make_params(0, shape, **KW)
    pt = F.make_params(0, shape, ternary=(0.2, 0.0, 0.9), **KW)
    b = F.Lattice(pb, phi0, rho0, u0).step(400)
    t = F.Lattice(pt, phi0, rho0, u0, psi0=psi0).step(400)
    fb, gb = b.populations()
    ft, gt, ht = t.populations()
    assert not np.any(ht) and not np.any(t.read(("psi",))["psi"])
    df, dg = np.abs(ft - fb).max(), np.abs(gt - gb).max()
    log(f"[parity] ternary psi=0 vs binary after 400 steps: f={df:.2e} g={dg:.2e}")
    assert df < 2e-6 and dg < 2e-6


def test_graph_stepping_and_checkpoint_bitwise():
    shape = (40, 30, 1)
    phi0, psi0, rho0, u0 = _fields(0, shape, 7.0)
    p = F.make_params(0, shape, ternary=K3, **KW)
    a = F.Lattice(p, phi0, rho0, u0, psi0=psi0, stream=torch.cuda.Stream())  # captured graphs
    b = F.Lattice(p, phi0, rho0, u0, psi0=psi0)                               # one launch at a time
    a.step(37)
    b.step(37)
    for x, y in zip(a.populations(), b.populations()):
        assert np.array_equal(x, y)
    blob = a.save()
    a.step(40)
    c = F.Lattice(p, phi0, rho0, u0, psi0=psi0)
    c.load(blob)
    c.step(40)
    for x, y in zip(a.populations(), c.populations()):
        assert np.array_equal(x, y)


def test_conservation_and_reduce():
    shape = (40, 30, 1)
    phi0, psi0, rho0, u0 = _fields(0, shape, 7.0)
    p = F.make_params(0, shape, ternary=K3, **KW)
    L = F.Lattice(p, phi0, rho0, u0, psi0=psi0)
    r0 = L.reduce()
    s0 = L.read(("psi",))["psi"].sum()
    L.step(500)
    r1 = L.reduce()
    s1 = L.read(("psi",))["psi"].sum()
    n = phi0.size
    assert r1[7] == n and r1[6] == 0
    assert abs(r1[0] - r0[0]) < 1e-6 * n and abs(r1[1] - r0[1]) < 1e-6 * n
    assert abs(s1 - s0) < 1e-6 * n


def test_unsupported_entry_points_refuse_ternary():
    shape = (16, 8, 1)
    phi0, psi0, rho0, u0 = _fields(0, shape, 3.0)
    p = F.make_params(0, shape, ternary=K3, **KW)
    L = F.Lattice(p, phi0, rho0, u0, psi0=psi0)
    with pytest.raises(F.FreError):
        L.consistent_init(phi0)
    with pytest.raises(F.FreError):
        L.autotune(2)
    with pytest.raises(F.FreError):
        buf = np.empty(9 * L.N)
        F._check(F.lib().fre_read_populations(L.handle, F._ptr(buf), F._ptr(buf), buf.size))
    B = F.Batch(2, 1 << 12, 1 << 12)
    with pytest.raises(F.FreError):
        B.add(L)
