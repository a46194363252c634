"""The breakup sweep on the host: one shear request per capillary number,
served together, and the critical range read off the outcomes -- driven by
the synthetic engine of the serving tests (no GPU)."""
from paper_2212_01617_amd import campaign, serve

from test_serve import Clock, FakeEngine


def test_sweep_requests_are_shear_drops_of_the_serving_geometry():
    rs = campaign.sweep_requests([0.5, 1.0], kind=0, n=150, Re=0.0625, xi=1.5)
    assert [r.Ca for r in rs] == [0.5, 1.0]
    assert all(r.flow == "shear" and r.arrival == 0.0 and r.radius == 30.0 for r in rs)
    assert rs[0].shape == (300, 150, 1)


def test_sweep_outcomes_and_critical_range():
    clock = Clock()
    eng = FakeEngine(clock, 1 << 40)   # breaks up for Ca >= 0.39, steady below
    rows = campaign.breakup_sweep([0.1, 0.2, 0.3, 0.4, 0.6], n=32, Re=0.5, engine=eng, budget_bytes=1 << 40)
    assert [r["reason"] for r in rows] == ["steady"] * 3 + ["breakup"] * 2
    assert all(r["strain"] > 3.0 for r in rows[3:])
    assert campaign.critical_range(rows) == (0.3, 0.4)
    assert campaign.critical_range(rows[:3]) == (0.3, None)
    assert campaign.critical_range([{"Ca": 1.0, "reason": "cap"}]) == (1.0, None)


def test_progress_lines_come_from_samples_and_retirements():
    clock = Clock()
    lines = []
    rows = campaign.breakup_sweep([0.2, 0.6], n=32, Re=0.5, engine=FakeEngine(clock, 1 << 40),
                                  budget_bytes=1 << 40, log=lines.append)
    assert [r["reason"] for r in rows] == ["steady", "breakup"]
    assert sum("retired" in s for s in lines) == 2
    assert any(s.endswith(" samples") for s in lines)
