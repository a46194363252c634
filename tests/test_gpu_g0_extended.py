"""The extended rest population (fre_params.g0_extended, FP32 storage): g_0,
which is O(1), carried as its FP32 value plus the part FP32 rounds away.
Parity with the FP64 oracle closer than the default FP32 state on the
cases where the rounding of g_0 dominates; a checkpoint holds the low part
(save, load and step is bitwise equal to stepping through); extended
lattices in a mixed batch step bitwise as they do alone; the refusals: FP16
storage, a change through fre_set_params."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import synth
from paper_2212_01617_amd.params import derive_params

from _pair import case_inputs, ensure_gpu_lib, field_errors, log, pop_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def _shear_2d():
    nx, ny = 400, 200
    dp = derive_params(Re=0.5, Ca=0.1, radius=40.0, xi=2.0, H=ny, Pe=0.43)
    wu = np.zeros((3, 2, 3)); wu[1, 0, 0] = -dp.wall_u; wu[1, 1, 0] = dp.wall_u
    sh = (1, ny, nx)
    phi0 = synth.droplet_phi(sh, 40.0, 2.0, noise=1e-4, seed=0, dims=2)
    u0 = synth.shear_velocity(sh, dp.rate, axis_normal=1)
    return (nx, ny, 1), dict(bc=(0, 1, 0), wall_u=wu, **dp.phys()), phi0, u0


def test_shear_2d_300_steps_closer_than_default():
    shape, kw, phi0, u0 = _shear_2d()
    ref = O.Lattice(O.make_params(0, shape, **kw), phi0, None, u0).step(300)
    errs = {}
    for ext in (False, True):
        gpu = F.Lattice(F.make_params(0, shape, g0_extended=ext, **kw), phi0, None, u0,
                        stream=torch.cuda.Stream())
        gpu.step(300)
        errs[ext] = field_errors(ref, gpu)
        pf, pg = pop_errors(ref, gpu)
        log(f"[parity] g0_extended={ext} shear_400x200_300: " +
            " ".join(f"{k}={v:.2e}" for k, v in errs[ext].items()) + f" f={pf:.2e} g={pg:.2e}")
        assert pf < 1e-5 and pg < 1e-5
        gpu.close()
    assert errs[True]["phi"] < 2e-6 and errs[True]["u"] < 1e-5
    assert errs[True]["phi"] < 0.5 * errs[False]["phi"]


def test_consistent_init_resets_the_low_part():
    # pre-iterations reset g to equilibrium, the low part of g_0 with it;
    # then normal steps, field by field against the oracle
    shape = (64, 48, 1)
    phi0, _, _ = case_inputs(0, shape, radius=12, xi=1.5, noise=1e-4, seed=0)
    kw = dict(A=0.04, kappa=0.09, tau_f=1.0, tau_g=1.0, M=0.1)
    ref = O.Lattice(O.make_params(0, shape, **kw), phi0).consistent_init(phi0, None, 300)
    gpu = F.Lattice(F.make_params(0, shape, g0_extended=True, **kw), phi0,
                    stream=torch.cuda.Stream()).consistent_init(phi0, None, 300)
    for n in (0, 101):
        ref.step(n)
        gpu.step(n)
        err = field_errors(ref, gpu)
        pf, pg = pop_errors(ref, gpu)
        log(f"[parity] g0_extended consistent_init_drop_d2q9_{n}: " +
            " ".join(f"{k}={v:.2e}" for k, v in err.items()) + f" f={pf:.2e} g={pg:.2e}")
        assert err["phi"] < 1e-5 and err["u"] < 1e-5 and err["rho"] < 1e-5 and pf < 1e-5 and pg < 1e-5
    gpu.close()


def test_checkpoint_holds_the_low_part():
    shape = (70, 9, 12)
    phi0, rho0, u0 = case_inputs(1, shape, radius=4, xi=2.0, noise=1e-3, seed=5, rho_amp=0.01, u_amp=0.01,
                                 center=(30.0, 4.0, 5.5))
    p = F.make_params(1, shape, A=5.89e-3, kappa=2.36e-2, tau_f=1.0, tau_g=1.75, M=5.26, g0_extended=True)
    a = F.Lattice(p, phi0, rho0, u0)
    a.step(37)
    blob = a.save()
    a.step(40)
    b = F.Lattice(p, phi0, rho0, u0)
    b.load(blob)
    b.step(40)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    # the low part is there: g_0 read back is not an FP32 number everywhere
    g0 = ga[0][np.abs(ga[0]) > 0.5]
    assert np.any(g0 != g0.astype(np.float32).astype(np.float64))


def test_mixed_batch_equals_solo_bitwise():
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -0.01; wu[2, 1, 0] = 0.01
    phi3, _, u3 = case_inputs(1, (40, 20, 12), radius=5, xi=1.5, u_amp=0.005, seed=1)
    phi2, _, _ = case_inputs(0, (70, 33, 1), radius=8, xi=1.5, seed=2)
    specs = [
        (F.make_params(1, (40, 20, 12), bc=(0, 0, 1), wall_u=wu, A=0.04, kappa=0.09, g0_extended=True), phi3, u3),
        (F.make_params(1, (40, 20, 12), bc=(0, 0, 1), wall_u=wu, A=0.04, kappa=0.09), phi3, u3),
        (F.make_params(0, (70, 33, 1), A=0.04, kappa=0.09, g0_extended=True), phi2, None),
        (F.make_params(0, (70, 33, 1), storage=F.FRE_FP16, A=0.04, kappa=0.09), phi2, None),
    ]
    steps = 11
    solo = []
    for p, phi0, u0 in specs:
        L = F.Lattice(p, phi0, None, u0)
        L.step(steps)
        solo.append(L.populations())
        L.close()
    lats = [F.Lattice(p, phi0, None, u0) for p, phi0, u0 in specs]
    w = f = 0
    for L in lats:
        a, b = F.Batch.needs(L)
        w += a
        f += b
    B = F.Batch(max_slots=4, max_work=w, max_fill=f)
    for L in lats:
        B.add(L)
    B.step(steps)          # graph replay on the batch's stream
    for k, L in enumerate(lats):
        fb, gb = L.populations()
        assert np.array_equal(fb, solo[k][0]) and np.array_equal(gb, solo[k][1]), k
    # the two D3Q19 FP32 members differ only in g0_extended, and their states do
    assert not np.array_equal(lats[0].populations()[1], lats[1].populations()[1])
    B.close()


def test_refusals():
    shape = (16, 8, 1)
    phi0, _, _ = case_inputs(0, shape, radius=3, xi=1.5)
    with pytest.raises(F.FreError) as e:
        F.footprint(F.make_params(0, shape, storage=F.FRE_FP16, A=0.04, kappa=0.09, g0_extended=True))
    assert e.value.status == F.FRE_EINVAL
    p = F.make_params(0, shape, A=0.04, kappa=0.09, g0_extended=True)
    L = F.Lattice(p, phi0)
    with pytest.raises(F.FreError) as e:
        L.set_params(F.make_params(0, shape, A=0.04, kappa=0.09, g0_extended=False))
    assert e.value.status == F.FRE_EINVAL
    L.close()
