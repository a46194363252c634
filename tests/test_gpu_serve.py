"""Serving on the GPU: a small mixed request stream through the real batch
engine.  Every request retires, memory and slots stay within their limits,
each retired lattice holds bitwise the populations of the same lattice
advanced alone for the same number of steps (at most one chunk past its
outcome's step: a retiring member is decided while the next chunk runs), and agrees with the FP64
oracle stepped for that many steps (FP32 storage at the 1e-5 bar, FP16
storage at its stated error)."""
import numpy as np
import pytest
import torch

from paper_2212_01617_amd import frelbm as F
from paper_2212_01617_amd import serve

from _pair import check_against_oracle, ensure_gpu_lib, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def test_serving_mix_equals_solo_runs():
    rs = serve.make_requests(8, rate=200.0, seed=11, d2_sizes=(32, 48), d3_sizes=(24, 32), Re=(0.1, 0.5))
    eng = serve.GpuEngine(budget_bytes=1 << 30, max_members=4, keep_final=True)
    budget = 3 * max(eng.footprint(r) for r in rs)
    srv = serve.Server(eng, budget, max_members=4, chunk=100, strain_cap=1.0, step_cap=3000)
    rep = srv.run(rs)
    s = rep.summary()
    log(f"[serve] {s}")
    assert s["requests"] == len(rs) and s["invalid"] == 0
    assert rep.peak_bytes <= budget and rep.peak_members <= 4
    assert eng.batch.info()[0] == 0
    for o in rep.outcomes:
        assert o.reason in ("steady", "breakup", "cap")
        t, (fa, ga) = eng.final[o.rid]
        # a retiring lattice is decided while the next chunk runs, so it may
        # have taken that chunk too (+1: a solo step to join at odd parity)
        assert o.steps <= t <= o.steps + srv.chunk + 1
        p, phi0, u0, mask, _ = serve.lattice_inputs(rs[o.rid])
        L = F.Lattice(p, phi0, None, u0, mask)
        L.step(t)
        fb, gb = L.populations()
        same = np.array_equal(fa, fb) and np.array_equal(ga, gb)
        log(f"[serve] request {o.rid} ({rs[o.rid].shape}, {o.reason}, t={t}): equal to solo: {same}")
        assert same, o.rid
        check_against_oracle(f"served_request_{o.rid}", p, L, t, phi0, None, u0, mask)
