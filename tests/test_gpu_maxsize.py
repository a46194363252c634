"""The largest lattice the 32-bit population offsets allow, checked against
the oracle through a property that holds at any size: a periodic lattice
made of identical copies of a small periodic lattice evolves as that small
lattice does, copy by copy.  256 x 256 x 860 D3Q19 cells in FP32 put the
population arrays just under 4 GiB (one more plane than 862 is refused);
every 32 x 32 x 20 copy of the GPU run is compared with the FP64 oracle's
run of one copy, stepped as the benchmark steps (own stream, graphs)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2212_01617_amd import frelbm as F

from _pair import case_inputs, ensure_gpu_lib, log

pytestmark = pytest.mark.gpu

TILE = (32, 32, 20)      # nx, ny, nz of one copy
REPS = (8, 8, 43)        # copies along x, y, z
PHYS = dict(A=5.89e-3, kappa=2.36e-2, tau_f=1.0, tau_g=1.75, M=5.26)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def test_size_limit_is_where_the_offsets_end():
    ok = F.make_params(F.FRE_D3Q19, (256, 256, 862), **PHYS)
    assert F.footprint(ok) > 0
    with pytest.raises(F.FreError) as e:
        F.footprint(F.make_params(F.FRE_D3Q19, (256, 256, 863), **PHYS))
    assert e.value.status == F.FRE_EINVAL


def test_maximum_size_lattice_matches_the_oracle_copy_by_copy():
    nx, ny, nz = TILE
    phi0, rho0, u0 = case_inputs(1, TILE, radius=6, xi=2.0, noise=1e-3, seed=9, rho_amp=0.01, u_amp=0.01,
                                 center=(15.5, 12.0, 9.5))
    steps = 10
    ref = O.Lattice(O.make_params(1, TILE, **PHYS), phi0, rho0, u0).step(steps)
    a = ref.observe()
    rz, ry, rx = REPS[2], REPS[1], REPS[0]
    big = (nx * rx, ny * ry, nz * rz)
    gpu = F.Lattice(F.make_params(F.FRE_D3Q19, big, **PHYS), np.tile(phi0, (rz, ry, rx)),
                    np.tile(rho0, (rz, ry, rx)), np.tile(u0, (1, rz, ry, rx)), stream=torch.cuda.Stream())
    log(f"[maxsize] {big}: {gpu.N} cells, {gpu._nbytes / 2**30:.2f} GiB of device memory")
    gpu.step(steps)
    b = gpu.read(("rho", "phi", "u"))
    err = {}
    for k in ("rho", "phi"):
        blocks = b[k].reshape(rz, nz, ry, ny, rx, nx)
        err[k] = float(np.abs(blocks - a[k][None, :, None, :, None, :]).max())
    uerr = 0.0
    for c, name in enumerate(("ux", "uy", "uz")):
        blocks = b["u"][c].reshape(rz, nz, ry, ny, rx, nx)
        uerr = max(uerr, float(np.abs(blocks - a[name][None, :, None, :, None, :]).max()))
    err["u"] = uerr
    log("[parity] maxsize_copies: " + " ".join(f"{k}={v:.2e}" for k, v in err.items()))
    assert err["rho"] < 1e-5 and err["phi"] < 1e-5 and err["u"] < 1e-5
    gpu.close()


def test_maximum_size_ternary_lattice_matches_the_oracle_copy_by_copy():
    """The same check for a ternary lattice (three population arrays, each
    just under 4 GiB), against the oracle's ternary step of one copy."""
    nx, ny, nz = TILE
    phi0, rho0, u0 = case_inputs(1, TILE, radius=6, xi=2.0, noise=1e-3, seed=9, rho_amp=0.01, u_amp=0.01,
                                 center=(15.5, 12.0, 9.5))
    psi0 = 0.3 * (1.0 - 0.5 * (1.0 + phi0))      # C3: 0.3 of what is not component 1
    phi0 = phi0 + psi0                           # C1 = (1 + phi0) / 2 kept, C2 = 1 - C1 - C3
    k3 = (4 * PHYS["A"], PHYS["M"] / 3, PHYS["tau_g"])   # psi's Cahn-Hilliard update in its stable range
    steps = 10
    po = O.make_params(1, TILE, **PHYS)
    ref = O.Lattice3(po, *k3, phi0, psi0, rho0, u0).step(steps)
    a = ref.observe()
    rz, ry, rx = REPS[2], REPS[1], REPS[0]
    big = (nx * rx, ny * ry, nz * rz)
    gpu = F.Lattice(F.make_params(F.FRE_D3Q19, big, ternary=k3, **PHYS), np.tile(phi0, (rz, ry, rx)),
                    np.tile(rho0, (rz, ry, rx)), np.tile(u0, (1, rz, ry, rx)), psi0=np.tile(psi0, (rz, ry, rx)),
                    stream=torch.cuda.Stream())
    log(f"[maxsize] ternary {big}: {gpu.N} cells, {gpu._nbytes / 2**30:.2f} GiB of device memory")
    gpu.step(steps)
    b = gpu.read(("rho", "phi", "psi", "u"))
    err = {}
    for k in ("rho", "phi", "psi"):
        blocks = b[k].reshape(rz, nz, ry, ny, rx, nx)
        err[k] = float(np.abs(blocks - a[k][None, :, None, :, None, :]).max())
    uerr = 0.0
    for c, name in enumerate(("ux", "uy", "uz")):
        blocks = b["u"][c].reshape(rz, nz, ry, ny, rx, nx)
        uerr = max(uerr, float(np.abs(blocks - a[name][None, :, None, :, None, :]).max()))
    err["u"] = uerr
    log("[parity] maxsize_ternary_copies: " + " ".join(f"{k}={v:.2e}" for k, v in err.items()))
    assert max(err.values()) < 1e-5
    gpu.close()
