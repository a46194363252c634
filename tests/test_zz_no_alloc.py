"""The allocation-free reduction (fre_reduce_noalloc) against fre_reduce,
through the C ABI: two calls in a row on different lattices, the second
smaller, each bitwise equal to fre_reduce on the same state; and the
non-finite path (flagged, lattice failed)."""
import numpy as np
import pytest
import torch

from paper_2212_01617_amd import frelbm as F

from _pair import case_inputs, ensure_gpu_lib, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _lattices():
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -0.01; wu[2, 1, 0] = 0.01
    shape3 = (72, 40, 24)
    phi3, _, u3 = case_inputs(1, shape3, radius=8, xi=2.0, shear=(0.02 / 24, 2), seed=3)
    big = F.Lattice(F.make_params(1, shape3, bc=(0, 0, 1), wall_u=wu, A=5.89e-3, kappa=2.36e-2, tau_g=1.75,
                                  M=5.26), phi3, None, u3, stream=torch.cuda.Stream())
    shape2 = (30, 20, 1)
    phi2, _, _ = case_inputs(0, shape2, radius=5, xi=1.5, seed=4)
    small = F.Lattice(F.make_params(0, shape2, storage=F.FRE_FP16, A=0.04, kappa=0.09), phi2)
    return big, small


def test_noalloc_equals_reduce_twice_second_smaller():
    big, small = _lattices()
    big.step(31)
    small.step(17)
    for name, L in (("72x40x24 d3q19 fp32", big), ("30x20 d2q9 fp16", small)):
        a = L.reduce_noalloc()
        b = L.reduce()
        log(f"[noalloc] {name}: {a.tolist()}")
        assert np.array_equal(a, b), (name, a, b)
        assert a[7] == np.prod(L.shape) and a[6] == 0
    # a second round after more steps: the array keeps the last call's
    # contents, which must not leak into the next
    big.step(5)
    small.step(3)
    for L in (big, small):
        assert np.array_equal(L.reduce_noalloc(), L.reduce())
    big.close()
    small.close()


def test_noalloc_flags_nonfinite():
    shape = (16, 8, 1)
    phi0, _, _ = case_inputs(0, shape, radius=3, xi=1.5)
    p = F.make_params(0, shape, A=0.2, kappa=0.5, tau_f=0.5005, tau_g=0.5005, M=1.0)
    L = F.Lattice(p, phi0)
    L.step(400)
    with pytest.raises(F.FreError) as ei:
        L.reduce_noalloc()
    assert ei.value.status == F.FRE_ENUMERIC
    with pytest.raises(F.FreError) as ei:
        L.step(1)
    assert ei.value.status == F.FRE_ESTATE
