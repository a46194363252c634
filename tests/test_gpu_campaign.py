"""Breakup in shear on the GPU serving engine (qualitative, after Sec. 3.2):
a 2D drop of radius 16 at Re = 1 stays whole at Ca = 0.2 and breaks up at
Ca = 2, both served together in one batch."""
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
