"""Breakup in shear on the GPU serving engine (qualitative, after Sec. 3.1, Breakup):
a 2D drop of radius 16 at Re = 1 stays whole at Ca = 0.2 and breaks up at
Ca = 2, both served together in one batch.  The 3D four-roller run on a
small cell: the drop on the stagnation point deforms in the extensional
flow, measured with the roller cells left out of the drop."""
import pytest
import torch

from paper_2212_01617_amd import campaign

from _pair import ensure_gpu_lib, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_gpu_lib()


def test_subcritical_stays_whole_supercritical_breaks():
    rows = campaign.breakup_sweep([0.2, 2.0], kind=0, n=80, Re=1.0, xi=1.5, strain_cap=20.0,
                                  budget_bytes=1 << 30, log=log)
    log(f"[campaign] {rows}")
    assert rows[0]["reason"] in ("steady", "cap") and rows[0]["strain"] >= 10.0
    assert rows[1]["reason"] == "breakup" and rows[1]["strain"] > 2.0
    assert campaign.critical_range(rows) == (0.2, 2.0)


def test_four_roller_drop_deforms():
    # Pe = 10 as in the served runs: at the paper's 0.43 a drop this small
    # dissolves by diffusion within a few hundred steps
    rows = campaign.four_roller_run([0.1], steps=2000, every=500, shape=(64, 64, 16), radius=8.0, xi=1.5, Pe=10.0,
                                    log=log)
    log(f"[rollers] {[{k: v for k, v in r.items() if k != 'history'} for r in rows]}")
    r = rows[0]
    assert r["reason"] == "cap" and r["steps"] == 2000
    # counting the rollers (phi reads 0 there) as half drop gave D ~ 0.01
    assert 0.05 < r["D"] < 0.9
    assert [h[2] for h in r["history"]] == [1, 1, 1, 1]
