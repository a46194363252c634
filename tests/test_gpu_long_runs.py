"""Parity over the long horizons of the shear cases, against the FP64
oracle's end states stored by ``tests/golden/long_runs.py``:

* the 64x32x32 D3Q19 copy of the 3D shear case after 20,000 steps: u at the
  1e-5 bar and the Taylor deformation D from both phi fields within 1%
  (observed 3.3e-8 and 1.9e-5 relative).  Its max-abs phi difference, 1.4e-5
  at the interface, is stated and held to 3e-5: single-precision storage
  alone moves this case that far (the FP64 oracle with only its stored g_0
  rounded to FP32 each step ends 4.4e-5 from the exact run in phi).  With
  g_0 carried past FP32 (g0_extended) phi, u and D all meet the bar;
* the 400x200 D2Q9 parallel-band shear after 40,000 steps: u at the 1e-5
  bar and D within 1% (observed 7.0e-7 and 1.0e-3 relative).  Its phi
  difference, 1.1e-3, is stated and held to 2e-3: the FP32 collision
  conserves momentum only to rounding, and in this 200-cell channel
  (viscous time about 240k steps) the velocity difference grows with time,
  so the interface position, its time integral, drifts apart faster.

Both are stepped as the benchmark steps (own stream, captured graphs)."""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2212_01617_amd import diagnostics as Dg
from paper_2212_01617_amd import frelbm as F

from _pair import ensure_gpu_lib, log

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import long_runs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


@pytest.fixture(scope="module")
def golden():
    return long_runs.load()


def _run(name, golden, g0_extended=False):
    meta, arrays = golden
    c = long_runs.case(name)
    m = meta[name]
    assert m["steps"] == c["steps"] and tuple(m["shape"]) == tuple(c["shape"])
    for k, v in c["phys"].items():
        assert m["phys"][k] == v, (name, k)
    assert np.array_equal(np.asarray(m["wall_u"]), np.asarray(c["wall_u"]))
    p = F.make_params(c["kind"], c["shape"], bc=c["bc"], wall_u=c["wall_u"], g0_extended=g0_extended, **c["phys"])
    gpu = F.Lattice(p, c["phi0"], None, c["u0"], stream=torch.cuda.Stream())
    gpu.step(c["steps"])
    out = gpu.read(("phi", "u"))
    gpu.close()
    err = {"phi": float(np.abs(out["phi"] - arrays[f"{name}__phi"]).max())}
    err["u"] = max(float(np.abs(out["u"][i] - arrays[f"{name}__{f}"]).max())
                   for i, f in enumerate(("ux", "uy", "uz")[:len(m["fields"]) - 1]))
    d_ref = Dg.deformation(arrays[f"{name}__phi"].astype(np.float64), plane=c["plane"], periodic=c["periodic"]).D
    d_gpu = Dg.deformation(out["phi"], plane=c["plane"], periodic=c["periodic"]).D
    rel = abs(d_gpu - d_ref) / abs(d_ref)
    log(f"[parity] {name}_{c['steps']}{'_g0ext' if g0_extended else ''}: phi={err['phi']:.2e} u={err['u']:.2e} "
        f"D_oracle={d_ref:.5f} D_gpu={d_gpu:.5f} rel={rel:.2e}")
    assert d_ref > 1e-2
    return err, rel


def test_c3_copy_20000_steps(golden):
    err, rel = _run("c3_copy", golden)
    assert err["u"] < 1e-5 and rel < 0.01
    assert err["phi"] < 3e-5


def test_c3_copy_20000_steps_extended_g0(golden):
    err, rel = _run("c3_copy", golden, g0_extended=True)
    assert err["phi"] < 1e-5 and err["u"] < 1e-5 and rel < 0.01


def test_shear_2d_40000_steps(golden):
    err, rel = _run("shear_2d", golden)
    assert err["u"] < 1e-5 and rel < 0.01
    assert err["phi"] < 2e-3


def test_shear_2d_40000_steps_extended_g0(golden):
    """With g_0 carried past FP32 the 2D shear's phi difference at 40,000
    steps falls from 1.1e-3 to about 4e-4 (stated, held to 1e-3); the rest is
    the momentum drift of the FP32 collision."""
    err, rel = _run("shear_2d", golden, g0_extended=True)
    assert err["u"] < 1e-5 and rel < 0.01
    assert err["phi"] < 1e-3
