"""Parity over the long horizons of the shear cases, against the FP64
oracle's end states stored by ``tests/golden/long_runs.py``, with the lattice
stepped as the benchmark steps it (own stream, captured graphs):

* the 64x32x32 D3Q19 copy of the 3D shear case after 20,000 steps: phi and u
  at the 1e-5 bar and the Taylor deformation D from both phi fields within
  1%;
* the 400x200 D2Q9 parallel-band shear after 40,000 steps: phi and u at the
  1e-5 bar and D within 1%;
* FP16 storage on both, rounded to nearest and rounded stochastically: the
  deviations are stated and held near what was measured, so that a
  regression of the FP16 path fails.

The 2D case is the sensitive one: this 200-cell channel's viscous time
(about 240,000 steps) is far longer than the run, so a rounding of the
collision that is the same from step to step and from cell to cell is not
damped, and the interface position integrates it."""
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


def _run(name, golden, storage=F.FRE_FP32, sr=False):
    meta, arrays = golden
    c = long_runs.case(name)
    m = meta[name]
    assert m["steps"] == c["steps"] and tuple(m["shape"]) == tuple(c["shape"])
    for k, v in c["phys"].items():
        assert m["phys"][k] == v, (name, k)
    assert np.array_equal(np.asarray(m["wall_u"]), np.asarray(c["wall_u"]))
    p = F.make_params(c["kind"], c["shape"], storage=storage, bc=c["bc"], wall_u=c["wall_u"],
                      stochastic_rounding=sr, **c["phys"])
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
    tag = ("_fp16" if storage == F.FRE_FP16 else "") + ("_stochastic" if sr else "")
    log(f"[parity] {name}{tag}_{c['steps']}: phi={err['phi']:.2e} u={err['u']:.2e} "
        f"D_oracle={d_ref:.5f} D_gpu={d_gpu:.5f} rel={rel:.2e}")
    assert d_ref > 1e-2
    return err, rel


def test_c3_copy_20000_steps(golden):
    err, rel = _run("c3_copy", golden)
    assert err["phi"] < 1e-5 and err["u"] < 1e-5 and rel < 0.01


def test_shear_2d_40000_steps(golden):
    err, rel = _run("shear_2d", golden)
    # measured: phi 1.7e-6, u 4.7e-9, D 3.1e-6 relative
    assert err["phi"] < 1e-5 and err["u"] < 1e-5 and rel < 0.01


def test_c3_copy_20000_steps_fp16(golden):
    err, rel = _run("c3_copy", golden, storage=F.FRE_FP16)
    # measured: phi 1.1e-4, u 4.1e-6, D 3.4e-4 relative; held at about 3x
    assert err["phi"] < 3.5e-4 and err["u"] < 1.2e-5 and rel < 1e-3


def test_shear_2d_40000_steps_fp16(golden):
    err, rel = _run("shear_2d", golden, storage=F.FRE_FP16)
    # measured: phi 6.3e-2, u 3.2e-4, D 16% low.  Half-precision storage
    # rounds every population at about 5e-4 relative each step; in this
    # slow channel the rounding of the steady parts of the flow repeats
    # from step to step and is not damped within the run.  Held at 2x.
    assert err["phi"] < 0.13 and err["u"] < 6.5e-4 and rel < 0.33


def test_c3_copy_20000_steps_fp16_stochastic(golden):
    err, rel = _run("c3_copy", golden, storage=F.FRE_FP16, sr=True)
    # measured: phi 2.9e-6, u 1.9e-6, D 1.7e-6 relative (round-to-nearest:
    # 9.5e-5, 2.7e-6, 4.4e-4); held at about 3x
    assert err["phi"] < 1e-5 and err["u"] < 6e-6 and rel < 1e-5


def test_shear_2d_40000_steps_fp16_stochastic(golden):
    err, rel = _run("shear_2d", golden, storage=F.FRE_FP16, sr=True)
    # unbiased rounding: the step-to-step repetition of the rounding error
    # that round-to-nearest integrates in this channel averages out.
    # measured: phi 1.6e-3, u 4.5e-6, D 6.0e-5 relative (round-to-nearest:
    # 6.3e-2, 3.2e-4, 16%); held at about 3x
    assert err["phi"] < 5e-3 and err["u"] < 1.5e-5 and rel < 2.5e-4
