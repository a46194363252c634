"""fre_profile_step on the GPU: the per-kernel timing entry point advances
the lattice by real steps -- individually launched, bitwise the same as the
graph-replayed steps of fre_step -- and reports one positive mean duration
for each kernel the lattice's step launches (FP32 storage: the by-product
moments completed by k_combine; FP16: the separate k_moments pass).  Its
argument checks refuse before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2212_01617_amd import frelbm as F

from _pair import case_inputs, ensure_gpu_lib, log

pytestmark = pytest.mark.gpu

SLOTS = ("k_moments", "k_fill_m", "k_potential", "k_fill_c", "k_collide", "k_combine")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _lattice(storage, seed):
    shape = (70, 20, 12)
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -0.01; wu[2, 1, 0] = 0.01
    phi0, _, u0 = case_inputs(1, shape, radius=5, xi=2.0, noise=1e-4, seed=seed, shear=(2 * 0.01 / 12, 2))
    p = F.make_params(1, shape, storage=storage, bc=(0, 0, 1), wall_u=wu,
                      A=5.89e-3, kappa=2.36e-2, tau_f=1.0, tau_g=1.75, M=5.26)
    return F.Lattice(p, phi0, None, u0, stream=torch.cuda.Stream())


def test_kernel_names_in_slot_order():
    L = F.lib()
    assert [L.fre_kernel_name(k).decode() for k in range(len(SLOTS))] == list(SLOTS)
    assert L.fre_kernel_name(len(SLOTS)) is None and L.fre_kernel_name(-1) is None


@pytest.mark.parametrize("storage", [F.FRE_FP32, F.FRE_FP16])
def test_profiled_steps_are_real_steps(storage):
    a, b = _lattice(storage, 31), _lattice(storage, 31)
    a.step(3)
    prof = a.profile(7)                   # steps 3..9, from odd parity
    b.step(10)
    log(f"[profile] storage {storage}: " + " ".join(f"{k}={v * 1e3:.1f}us" for k, v in prof.items()))
    launched = set(SLOTS) - {"k_moments" if storage == F.FRE_FP32 else "k_combine"}
    assert set(prof) == launched
    assert all(np.isfinite(v) and v > 0.0 for v in prof.values())
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    ra, rb = a.read(), b.read()
    for k in ("rho", "phi", "u"):
        assert np.array_equal(ra[k], rb[k]), k
    a.close()
    b.close()


def test_argument_checks():
    L = _lattice(F.FRE_FP32, 32)
    lib = F.lib()
    ms = np.zeros(8)
    nk = C.c_int32(-7)
    p = ms.ctypes.data_as(C.c_void_p)
    assert lib.fre_profile_step(L.handle, 0, p, 8, C.byref(nk)) == F.FRE_EINVAL       # n < 1
    assert lib.fre_profile_step(L.handle, 2, p, 5, C.byref(nk)) == F.FRE_EINVAL       # fewer than 6 entries
    assert lib.fre_profile_step(L.handle, 2, None, 8, C.byref(nk)) == F.FRE_EINVAL    # NULL output
    assert lib.fre_profile_step(L.handle, 2, p, 8, None) == F.FRE_EINVAL
    assert nk.value == -7 and not ms.any()
    ref = _lattice(F.FRE_FP32, 32)
    L.step(4)
    ref.step(4)
    assert np.array_equal(L.populations()[0], ref.populations()[0])   # the refusals did not step
    L.close()
    ref.close()
