"""Launch shapes and the autotuners: a shape changes which thread updates
which cell, never the arithmetic, so every shape gives bitwise the same
populations; tuning restores the state it stepped through."""
import numpy as np
import pytest
import torch

from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth

from _pair import case_inputs, ensure_gpu_lib, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _case(storage=0):
    # ragged in x (two 64-wide blocks) and y (not a multiple of 8), walls in z
    shape = (100, 13, 11)
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -0.01; wu[2, 1, 0] = 0.01
    phi0, _, u0 = case_inputs(1, shape, radius=4, xi=1.5, u_amp=0.005, seed=7)
    p = F.make_params(1, shape, storage=storage, bc=(0, 0, 1), wall_u=wu, A=0.04, kappa=0.09)
    return p, phi0, u0


@pytest.mark.parametrize("storage", [0, 1])
def test_every_launch_shape_is_bitwise_identical(storage):
    p, phi0, u0 = _case(storage)
    ref = F.Lattice(p, phi0, None, u0)
    ref.step(9)
    fr, gr = ref.populations()
    # FP32 storage fixes the collide tile at 4 rows (on-chip moment sums)
    cr = (4, 4, 4) if storage == 0 else (8, 2, 1)
    shapes = [
        {"k_moments": (1, 0), "k_potential": (2, 0), "k_collide": (cr[0], 0)},
        {"k_moments": (8, 1), "k_potential": (1, 1), "k_collide": (cr[1], 1)},
        {"k_moments": (2, 1), "k_potential": (8, 0), "k_collide": (cr[2], 1)},
    ]
    for sh in shapes:
        L = F.Lattice(p, phi0, None, u0, stream=torch.cuda.Stream())
        L.set_launch_shape(sh)
        assert L.launch_shape() == sh
        L.step(9)                          # graph path (odd count: both parities)
        f, g = L.populations()
        assert np.array_equal(f, fr) and np.array_equal(g, gr), sh


def test_autotune_picks_valid_shapes_and_restores_state():
    p, phi0, u0 = _case(0)
    a = F.Lattice(p, phi0, None, u0)
    a.step(5)
    t0 = a.info()[0]
    f0, g0 = a.populations()
    tuned = a.autotune(4)
    log(f"[tune] {tuned}")
    assert a.info()[0] == t0
    f1, g1 = a.populations()
    assert np.array_equal(f0, f1) and np.array_equal(g0, g1)
    for k, (rows, xcd, ms) in tuned.items():
        assert rows in (1, 2, 4, 8) and xcd in (0, 1) and ms > 0
    assert tuned["k_collide"][0] == 4          # FP32: fixed collide tile
    assert {k: v[:2] for k, v in tuned.items()} == a.launch_shape()
    a.step(6)
    b = F.Lattice(p, phi0, None, u0)
    b.step(11)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_bad_shapes_are_refused():
    p, phi0, u0 = _case(0)
    L = F.Lattice(p, phi0, None, u0)
    for bad in ({"k_moments": (3, 0), "k_potential": (4, 1), "k_collide": (4, 1)},
                {"k_moments": (4, 2), "k_potential": (4, 1), "k_collide": (4, 1)},
                {"k_moments": (16, 1), "k_potential": (4, 1), "k_collide": (4, 1)},
                {"k_moments": (4, 1), "k_potential": (4, 1), "k_collide": (8, 1)}):
        with pytest.raises(F.FreError) as ei:
            L.set_launch_shape(bad)
        assert ei.value.status == F.FRE_EINVAL
    assert L.launch_shape() == {k: (4, 1) for k in L.STAGES}


def test_batch_shapes_bitwise_and_autotune_restores():
    p, phi0, u0 = _case(0)
    phi2, _, _ = case_inputs(0, (70, 33, 1), radius=8, xi=1.5, seed=2)
    p2 = F.make_params(0, (70, 33, 1), storage=1, A=0.04, kappa=0.09)
    solo = [F.Lattice(p, phi0, None, u0).step(12), F.Lattice(p2, phi2).step(12)]
    ref = [L.populations() for L in solo]
    mem = [F.Lattice(p, phi0, None, u0), F.Lattice(p2, phi2)]
    w = sum(F.Batch.needs(L)[0] for L in mem)
    fl = sum(F.Batch.needs(L)[1] for L in mem)
    B = F.Batch(max_slots=2, max_work=w, max_fill=fl)
    for L in mem:
        B.add(L)
    B.set_launch_shape(2)
    assert B.launch_shape() == 2
    B.step(3)
    B.set_launch_shape(16)
    B.step(3)
    bpc, ms = B.autotune(4)
    log(f"[tune] batch blocks/CU={bpc} {ms:.4f} ms/step")
    assert bpc in (2, 4, 8, 16) and B.launch_shape() == bpc
    assert all(L.info()[0] == 6 for L in mem)
    B.step(6)
    for L, (fr, gr) in zip(mem, ref):
        f, g = L.populations()
        assert np.array_equal(f, fr) and np.array_equal(g, gr)
