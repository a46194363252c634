"""Four-roller calibration on the GPU: the extension rate at the centre of a
single-phase four-roller cell is proportional to the roller speed at low
speed (Stokes flow), and served roller requests take their angular speed
from it."""
import math

import pytest
import torch

from paper_2212_01617_amd import serve
from paper_2212_01617_amd.params import derive_params

from _pair import ensure_gpu_lib, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def test_calibration_is_linear_and_used_by_requests():
    n = 64
    k1 = serve.calibrate_rollers(n, tip_speed=1e-3)
    k2 = serve.calibrate_rollers(n, tip_speed=2e-3)
    rr = serve.roller_radius(n)
    estimate = rr / (math.hypot(n / 4.0, n / 4.0) - rr)   # stagnation-flow estimate of eps / omega
    log(f"[rollers] N={n}: eps/omega = {k1:.4f} (tip 1e-3), {k2:.4f} (tip 2e-3); estimate {estimate:.4f}")
    assert k1 > 0.0 and abs(k2 / k1 - 1.0) < 0.02
    assert 0.2 < k1 / estimate < 5.0
    req = serve.Request(0, 0.0, 0, n, "rollers", 0, 0.2, 0.5)
    p, *_ = serve.lattice_inputs(req)
    rate = derive_params(Re=req.Re, Ca=req.Ca, radius=req.radius, xi=req.xi, Pe=serve.SERVE_PE).rate
    assert abs(abs(p.rollers[0].omega) - rate / k2) < 1e-12 * rate / k2 + 1e-18
