"""Serving loop on the host: the request stream, admission by memory budget
and free slots in arrival order, retirement on steady deformation, breakup
or the cap, and the report -- driven by a synthetic engine and a virtual
clock (no GPU)."""
import math

import numpy as np
import pytest

from paper_2212_01617_amd import serve


def test_request_stream_is_seeded_and_mixed():
    a = serve.make_requests(256, rate=20.0, seed=0)
    b = serve.make_requests(256, rate=20.0, seed=0)
    assert [vars(r) for r in a] == [vars(r) for r in b]
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert np.all(gaps > 0) and abs(gaps.mean() - 1 / 20.0) < 0.2 / 20.0
    for key, lo, hi in (("kind", 0.4, 0.6), ("storage", 0.4, 0.6)):
        frac = np.mean([getattr(r, key) for r in a])
        assert lo < frac < hi
    assert 0.4 < np.mean([r.flow == "shear" for r in a]) < 0.6
    assert all(0.05 <= r.Ca <= 0.4 and 0.1 <= r.Re <= 1.0 for r in a)
    assert all(r.n in range(64, 513, 16) for r in a if r.kind == 0)
    assert all(r.n in range(48, 161, 16) for r in a if r.kind == 1)
    assert all(r.radius == pytest.approx(0.2 * r.n) for r in a)


def _ellipse_phi(D, R=10.0, n=48, split=False, xz=False):
    ratio = (1 + D) / (1 - D)
    a, b = R * math.sqrt(ratio), R / math.sqrt(ratio)
    y, x = np.meshgrid(np.arange(n) - (n - 1) / 2, np.arange(n) - (n - 1) / 2, indexing="ij")
    if split:
        r = np.minimum(np.hypot(x - 12, y), np.hypot(x + 12, y))
        f = np.tanh((6.0 - r) / 2.0)
    else:
        r = np.sqrt((x / a) ** 2 + (y / b) ** 2) * math.sqrt(a * b)
        f = np.tanh((math.sqrt(a * b) - r) / 2.0)
    # (z, y, x) layout: the ellipse lies in the x-y plane, or in x-z
    return f[:, None, :] if xz else f[None]


class FakeEngine:
    """Every request relaxes D towards 0.1 + 0.5 Ca with a time constant of
    one strain unit; Ca >= 0.39 breaks up after 3 strain units; Re < 0.105
    relaxes too slowly and hits the cap.  Cost: 1 ns of virtual time per
    lattice update."""

    def __init__(self, clock, budget, max_slots=None, refuse_every=0):
        self.clock = clock
        self.budget = budget
        self.used = 0
        self.members = {}
        self.order = []
        self.max_slots = max_slots
        self.refuse_every = refuse_every
        self.calls = 0

    def footprint(self, req):
        return req.cells * 160

    def periodic(self, req):
        return (True, True, True)

    def admit(self, req):
        self.calls += 1
        if self.refuse_every and self.calls % self.refuse_every == 0:
            return None
        self.used += self.footprint(req)
        assert self.used <= self.budget
        if self.max_slots is not None:
            assert len(self.members) < self.max_slots
        h = object()
        rate = 1e-3 if req.Re >= 0.105 else 1e-6
        self.members[h] = [req, 0, rate]
        self.order.append(req.rid)
        return h, rate

    def step(self, n):
        for m in self.members.values():
            m[1] += n
        self.clock.t += 1e-9 * n * sum(m[0].cells for m in self.members.values())

    def phi(self, h):
        req, t, rate = self.members[h]
        s = t * rate
        xz = req.flow == "shear" and req.kind == 1   # the server's shear plane
        if req.Ca >= 0.39 and s > 3.0:
            return _ellipse_phi(0.0, split=True, xz=xz)
        D = (0.1 + 0.5 * req.Ca) * (1 - math.exp(-s))
        return _ellipse_phi(D, xz=xz)

    def retire(self, h):
        req = self.members.pop(h)[0]
        self.used -= self.footprint(req)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def _requests(n=40, seed=3):
    rs = serve.make_requests(n, rate=50.0, seed=seed, d2_sizes=(32, 48), d3_sizes=(16, 24))
    return rs


def test_scheduler_admits_in_order_within_budget_and_retires_everyone():
    clock = Clock()
    rs = _requests()
    budget = 6 * max(r.cells for r in rs) * 160
    eng = FakeEngine(clock, budget, max_slots=5)
    srv = serve.Server(eng, budget, max_members=5, chunk=500, strain_cap=25.0, step_cap=200_000,
                       clock=clock, sleep=clock.sleep)
    rep = srv.run(rs)
    assert sorted(o.rid for o in rep.outcomes) == [r.rid for r in rs]
    assert eng.order == sorted(eng.order, key=lambda k: rs[k].arrival)  # no overtaking
    assert rep.peak_bytes <= budget and rep.peak_members <= 5
    by = {o.rid: o for o in rep.outcomes}
    for r in rs:
        o = by[r.rid]
        assert o.admitted >= r.arrival and o.retired >= o.admitted
        if r.Re < 0.105:
            assert o.reason == "cap"
        elif r.Ca >= 0.39:
            assert o.reason == "breakup" and 3.0 < o.strain <= 3.0 + 0.1 + 1e-9
        else:
            assert o.reason == "steady", (r, o)
            assert abs(o.D - (0.1 + 0.5 * r.Ca)) < 0.03
            # the window test needs at least 2 strain units of samples
            assert o.strain >= 2.0
    s = rep.summary()
    assert s["requests"] == len(rs)
    assert s["steady"] + s["breakup"] + s["capped"] == len(rs) and s["dissolved"] == 0
    assert s["p50_time_to_steady_s"] <= s["p99_time_to_steady_s"]
    assert s["aggregate_mlups"] > 0


def test_step_cap_is_exact_when_samples_are_sparse():
    # even requests take 1e-6 strain per step: their first D sample would
    # fall due after 100,000 steps, far beyond the step cap
    clock = Clock()
    rs = _requests(6, seed=4)

    class Slow(FakeEngine):
        def admit(self, req):
            got = super().admit(req)
            if got is not None and req.rid % 2 == 0:
                self.members[got[0]][2] = 1e-6
                return got[0], 1e-6
            return got

    budget = 8 * max(r.cells for r in rs) * 160
    eng = Slow(clock, budget)
    rep = serve.Server(eng, budget, max_members=6, chunk=500, strain_cap=25.0, step_cap=3000,
                       clock=clock, sleep=clock.sleep).run(rs)
    assert len(rep.outcomes) == 6
    for o in rep.outcomes:
        assert o.steps <= 3000
        if o.rid % 2 == 0:
            assert o.reason == "cap" and o.steps == 3000


def test_engine_refusal_waits_and_retries():
    clock = Clock()
    rs = _requests(12, seed=5)
    budget = 4 * max(r.cells for r in rs) * 160
    eng = FakeEngine(clock, budget, refuse_every=3)
    srv = serve.Server(eng, budget, max_members=8, chunk=500, clock=clock, sleep=clock.sleep)
    rep = srv.run(rs)
    assert len(rep.outcomes) == len(rs)
    assert eng.order == sorted(eng.order, key=lambda k: rs[k].arrival)


def test_request_larger_than_budget_is_rejected_up_front():
    clock = Clock()
    rs = _requests(3)
    eng = FakeEngine(clock, 10)
    with pytest.raises(ValueError):
        serve.Server(eng, 10, max_members=2, clock=clock, sleep=clock.sleep).run(rs)


def test_dissolved_drop_retires():
    clock = Clock()
    rs = _requests(4, seed=9)

    class Dissolving(FakeEngine):
        def phi(self, h):
            req, t, rate = self.members[h]
            if req.rid == 1 and t * rate > 1.0:
                return -0.97 * np.ones((1, 48, 48))   # no phi > 0 left
            return super().phi(h)

    budget = 4 * max(r.cells for r in rs) * 160
    eng = Dissolving(clock, budget)
    rep = serve.Server(eng, budget, max_members=4, chunk=500, clock=clock, sleep=clock.sleep).run(rs)
    by = {o.rid: o for o in rep.outcomes}
    assert by[1].reason == "dissolved" and rep.summary()["dissolved"] == 1


def test_failed_run_retires():
    clock = Clock()
    rs = _requests(4, seed=9)

    class Failing(FakeEngine):
        def phi(self, h):
            req, t, rate = self.members[h]
            if req.rid == 2 and t * rate > 0.5:
                raise serve.RunFailed("non-finite")
            return super().phi(h)

    budget = 4 * max(r.cells for r in rs) * 160
    eng = Failing(clock, budget)
    rep = serve.Server(eng, budget, max_members=4, chunk=500, clock=clock, sleep=clock.sleep).run(rs)
    by = {o.rid: o for o in rep.outcomes}
    assert by[2].reason == "failed" and rep.summary()["failed"] == 1 and len(by) == 4


def test_invalid_requests_are_reported_not_run():
    clock = Clock()
    rs = _requests(6)

    class Picky(FakeEngine):
        def footprint(self, req):
            if req.rid == 2:
                raise serve.InvalidRequest("refused")
            return super().footprint(req)

    budget = 4 * max(r.cells for r in rs) * 160
    eng = Picky(clock, budget)
    rep = serve.Server(eng, budget, max_members=4, chunk=500, clock=clock, sleep=clock.sleep).run(rs)
    by = {o.rid: o for o in rep.outcomes}
    assert len(by) == 6 and by[2].reason == "invalid" and 2 not in eng.order
    assert rep.summary()["invalid"] == 1


def test_lattice_inputs_follow_the_request():
    # host-only part of the GPU engine: shapes, walls, rollers, parameters
    from paper_2212_01617_amd import frelbm as F
    r = serve.Request(0, 0.0, 1, 48, "shear", 1, 0.1, 1.0)
    p, phi0, u0, mask, rate = serve.lattice_inputs(r)
    assert (p.nx, p.ny, p.nz) == (96, 48, 48) and list(p.bc) == [0, 0, 1]
    assert p.wall_u[2][1][0] == pytest.approx(rate * 48 / 2) and p.storage == 1
    assert phi0.shape == (48, 48, 96) and u0.shape == (3, 48, 48, 96) and mask is None
    r2 = serve.Request(1, 0.0, 0, 64, "rollers", 0, 0.2, 0.5)
    p2, phi2, u2, mask2, rate2 = serve.lattice_inputs(r2)
    assert (p2.nx, p2.ny, p2.nz) == (64, 64, 1) and p2.n_rollers == 4 and u2 is None
    assert set(np.unique(mask2)) == {0, 2, 3, 4, 5}
    om = [p2.rollers[k].omega for k in range(4)]
    assert sum(om) == pytest.approx(0.0) and all(abs(abs(o) - abs(om[0])) < 1e-15 for o in om)
    # the droplet clears the rollers
    assert np.all(phi2[mask2 > 0] < 0)


def test_zero_step_cap_samples_once_and_retires():
    # members admitted at the cap are sampled at step 0 and retire without
    # any step being taken
    clock = Clock()
    rs = _requests(6, seed=5)
    eng = FakeEngine(clock, budget=1 << 40)
    srv = serve.Server(eng, 1 << 40, max_members=8, chunk=100, step_cap=0, clock=clock, sleep=clock.sleep)
    rep = srv.run(rs)
    assert sorted(o.rid for o in rep.outcomes) == sorted(r.rid for r in rs)
    assert all(o.reason == "cap" and o.steps == 0 for o in rep.outcomes)
    assert rep.lattice_updates == 0 and not eng.members


def test_counted_updates_stop_at_each_retirement_step():
    # samples are decided while the next chunk runs, so a retiring member is
    # stepped once more; its outcome and the aggregate count only the steps
    # up to the sample it retired on
    clock = Clock()
    rs = _requests(10, seed=6)
    eng = FakeEngine(clock, budget=1 << 40)
    stepped = {}
    base_step, base_retire = eng.step, eng.retire

    def step(n):
        for m in eng.members.values():
            stepped[m[0].rid] = stepped.get(m[0].rid, 0) + n
        base_step(n)

    def retire(h):
        eng.final = getattr(eng, "final", {})
        rid = eng.members[h][0].rid
        eng.final[rid] = stepped.get(rid, 0)
        base_retire(h)

    eng.step, eng.retire = step, retire
    rep = serve.Server(eng, 1 << 40, max_members=4, chunk=300, strain_cap=4.0, step_cap=20_000,
                       clock=clock, sleep=clock.sleep).run(rs)
    assert len(rep.outcomes) == len(rs)
    for o in rep.outcomes:
        assert o.steps <= eng.final[o.rid] <= o.steps + 300
        assert abs(o.strain - o.steps * (1e-3 if rs[o.rid].Re >= 0.105 else 1e-6)) < 1e-12
    assert rep.lattice_updates == sum(o.steps * o.cells for o in rep.outcomes)
