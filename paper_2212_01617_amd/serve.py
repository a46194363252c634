"""Continuous-batching server for many droplet runs on one GPU.

Requests (a droplet in shear between moving walls, or in the extensional
flow of four rollers; D2Q9 or D3Q19; FP32 or FP16 storage) arrive as a
Poisson process.  They are admitted in arrival order when their device
footprint fits the memory budget and a batch slot is free, advanced
together by one batched step (``frelbm.Batch``), sampled for the Taylor
deformation D every 0.1 strain units, and retired when D is steady, the
droplet has broken up, or a cap is reached (diagnostics.SteadyTracker,
diagnostics.broken_up).  The report gives p50/p99 time-to-steady (arrival
to retirement, host clock, read-back included) and the aggregate lattice
update rate.

The scheduler is independent of the GPU: an engine object supplies
footprints, admission, stepping and sampling, so the scheduling logic can
be exercised on the host with a synthetic engine.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import diagnostics as Dg
from . import synth

SAMPLE_STRAIN = 0.1


class InvalidRequest(ValueError):
    """The library refuses the request's parameters."""


class RunFailed(RuntimeError):
    """A served lattice went non-finite (it is retired as failed)."""


@dataclass
class Request:
    rid: int
    arrival: float      # seconds after the start of the run
    kind: int           # 0 D2Q9, 1 D3Q19
    n: int              # lattice size parameter N
    flow: str           # "shear" or "rollers"
    storage: int        # 0 FP32, 1 FP16
    Ca: float
    Re: float
    xi: float = 2.0
    Pe: float | None = None  # Peclet number; None: SERVE_PE

    @property
    def radius(self) -> float:
        """Drop radius, 0.2 of the smallest box dimension (N for every shape)."""
        return 0.2 * min(d for d in self.shape if d > 1)

    @property
    def shape(self) -> tuple:
        """(nx, ny, nz) of the lattice: shear boxes are twice as long as wide
        along the flow, four-roller cells are N^2 (2D) or N^3 (3D)."""
        n = self.n
        if self.kind == 0:
            return (2 * n, n, 1) if self.flow == "shear" else (n, n, 1)
        return (2 * n, n, n) if self.flow == "shear" else (n, n, n)

    @property
    def cells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


def make_requests(n: int = 256, rate: float = 20.0, seed: int = 0,
                  d2_sizes=tuple(range(64, 513, 16)), d3_sizes=tuple(range(48, 161, 16)),
                  Ca=(0.05, 0.4), Re=(0.1, 1.0), xi: float = 2.0) -> list[Request]:
    """The mixed request stream: exponential inter-arrival gaps at ``rate``
    per second; half D2Q9, half D3Q19 (sizes drawn from the given lists);
    half shear, half four-roller; half FP32, half FP16; Ca and Re uniform.
    Every draw is a SplitMix64 uniform of (seed, request, field)."""
    u = synth.uniform(seed, 8 * n).reshape(n, 8)
    out = []
    t = 0.0
    for k in range(n):
        t += -math.log(1.0 - u[k, 0]) / rate
        kind = 0 if u[k, 1] < 0.5 else 1
        sizes = d2_sizes if kind == 0 else d3_sizes
        size = sizes[min(int(u[k, 2] * len(sizes)), len(sizes) - 1)]
        flow = "shear" if u[k, 3] < 0.5 else "rollers"
        storage = 0 if u[k, 4] < 0.5 else 1
        ca = Ca[0] + (Ca[1] - Ca[0]) * u[k, 5]
        re = Re[0] + (Re[1] - Re[0]) * u[k, 6]
        out.append(Request(k, t, kind, int(size), flow, storage, float(ca), float(re), xi))
    return out


@dataclass
class Outcome:
    rid: int
    reason: str           # "steady", "breakup", "dissolved", "cap", "failed" (non-finite) or "invalid"
    arrival: float
    admitted: float
    retired: float
    steps: int
    strain: float
    D: float
    cells: int

    @property
    def latency(self) -> float:
        return self.retired - self.arrival


@dataclass
class Report:
    outcomes: list
    wall: float
    lattice_updates: float
    peak_bytes: int
    peak_members: int

    def summary(self) -> dict:
        lat = np.array([o.latency for o in self.outcomes]) if self.outcomes else np.zeros(1)
        st = [o for o in self.outcomes if o.reason == "steady"]
        tts = np.array([o.latency for o in st])
        return {
            "requests": len(self.outcomes),
            "steady": len(st),
            "breakup": sum(o.reason == "breakup" for o in self.outcomes),
            "capped": sum(o.reason == "cap" for o in self.outcomes),
            "dissolved": sum(o.reason == "dissolved" for o in self.outcomes),
            "failed": sum(o.reason == "failed" for o in self.outcomes),
            "invalid": sum(o.reason == "invalid" for o in self.outcomes),
            "p50_time_to_steady_s": float(np.percentile(tts, 50)) if st else None,
            "p99_time_to_steady_s": float(np.percentile(tts, 99)) if st else None,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "aggregate_mlups": self.lattice_updates / self.wall / 1e6 if self.wall > 0 else 0.0,
            "wall_s": self.wall,
            "peak_bytes": self.peak_bytes,
            "peak_members": self.peak_members,
        }


@dataclass
class _Member:
    req: Request
    handle: object
    rate: float            # strain per step
    sample_every: int      # steps between D samples
    admitted: float
    t: int = 0
    next_sample: int = 0
    tracker: Dg.SteadyTracker = field(default_factory=Dg.SteadyTracker)
    D: float = 0.0


class Server:
    """Admission, stepping and retirement over an engine.

    engine.footprint(req) -> bytes (raises InvalidRequest for parameters the
    library refuses, e.g. a wall speed beyond the Mach guard);
    engine.admit(req) -> (handle, strain per step) or None when the engine
    cannot take it now; engine.step(n); engine.phi(handle) -> phi field
    (raises RunFailed for a lattice gone non-finite); engine.periodic(req) -> periodic flags (x, y, z); engine.retire(handle);
    optionally engine.prepare(requests), called once before the clock starts."""

    def __init__(self, engine, budget_bytes: int, max_members: int, chunk: int = 200,
                 strain_cap: float = 25.0, step_cap: int = 200_000, clock=time.monotonic,
                 sleep=time.sleep, on_retire=None):
        self.on_retire = on_retire  # called with each Outcome as it retires
        self.engine = engine
        self.budget = int(budget_bytes)
        self.max_members = int(max_members)
        self.chunk = int(chunk)
        self.strain_cap = strain_cap
        self.step_cap = int(step_cap)
        self.clock = clock
        self.sleep = sleep

    def _due(self, m: _Member) -> int:
        """Step count at which member m is next sampled."""
        return min(m.next_sample, self.step_cap)

    def _read(self, m: _Member):
        """phi of member m at its current step (None for a run gone
        non-finite), with that step."""
        try:
            return m, m.t, self.engine.phi(m.handle)
        except RunFailed:
            return m, m.t, None

    def _decide(self, m: _Member, t: int, phi):
        """From phi sampled at step t: sample D (and breakup); return the
        retirement reason or None."""
        if phi is None:
            return "failed"
        req = m.req
        per = self.engine.periodic(req)
        comps = Dg.components(phi, per)
        if len(comps) >= 2:
            return "breakup"
        if not comps:
            return "dissolved"
        plane = "xz" if (req.flow == "shear" and req.kind == 1) else "xy"
        solid = self.engine.solid(m.handle) if hasattr(self.engine, "solid") else None
        m.D = Dg.deformation(phi, plane=plane, periodic=per, solid=solid).D
        strain = t * m.rate
        if m.tracker.add(strain, m.D):
            return "steady"
        if strain >= self.strain_cap or t >= self.step_cap:
            return "cap"
        return None

    def run(self, requests) -> Report:
        outcomes = []
        ok = []
        for r in sorted(requests, key=lambda r: r.arrival):
            try:
                need = self.engine.footprint(r)
            except InvalidRequest:
                outcomes.append(Outcome(r.rid, "invalid", r.arrival, r.arrival, r.arrival, 0, 0.0, 0.0, r.cells))
                continue
            if need > self.budget:
                raise ValueError(f"request {r.rid} needs more than the whole memory budget")
            ok.append(r)
        if hasattr(self.engine, "prepare"):
            self.engine.prepare(ok)   # per-geometry set-up, before the clock starts
        pending = deque(ok)
        active: list[_Member] = []
        samples = []   # (member, step, phi) read at the end of the last chunk
        used = 0
        lu = 0.0
        peak_bytes = peak_members = 0
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission in arrival order (no overtaking)
            while pending and pending[0].arrival <= now and len(active) < self.max_members:
                r = pending[0]
                need = self.engine.footprint(r)
                if used + need > self.budget:
                    break
                got = self.engine.admit(r)
                if got is None:
                    break
                handle, rate = got
                pending.popleft()
                every = max(1, int(round(SAMPLE_STRAIN / rate)))
                active.append(_Member(r, handle, rate, every, now, next_sample=every))
                used += need
            peak_bytes = max(peak_bytes, used)
            peak_members = max(peak_members, len(active))
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            # step up to the next sample that falls due (or the step cap, which
            # a slow request may reach before its first sample), at most one
            # chunk; a member sampled at the step cap retires and sets no bound
            live = [m for m in active if m.t < self.step_cap]
            n = min([self.chunk] + [self._due(m) - m.t for m in live]) if live else 0
            n = max(n, 1) if live else 0
            if n:
                self.engine.step(n)   # asynchronous: the samples below are decided meanwhile
            # decide the samples read at the end of the previous chunk; a
            # member that retires has been stepped once more, which its
            # outcome does not count
            done = []
            for m, t, phi in samples:
                reason = self._decide(m, t, phi)
                if reason:
                    done.append((m, reason, t))
            samples = []
            retiring = {id(m) for m, _, _ in done}
            lu += n * sum(m.req.cells for m in active if id(m) not in retiring)
            for m, reason, t in done:
                self.engine.retire(m.handle)
                active.remove(m)
                used -= self.engine.footprint(m.req)
                outcomes.append(Outcome(m.req.rid, reason, m.req.arrival, m.admitted, self.clock() - t0,
                                        t, t * m.rate, m.D, m.req.cells))
                if self.on_retire:
                    self.on_retire(outcomes[-1])
            for m in active:
                m.t += n
                if m.t >= self._due(m):
                    if m.t >= m.next_sample:
                        m.next_sample += m.sample_every
                    samples.append(self._read(m))
        wall = self.clock() - t0
        return Report(outcomes, wall, lu, peak_bytes, peak_members)


# ---------------------------------------------------------------------------
# GPU engine: lattices in one frelbm.Batch
# ---------------------------------------------------------------------------
# Peclet number of the served runs.  At the Pe = 0.43 of the paper's shear
# validation, drops of radius 0.2 N <= 32 at a few per cent volume fraction
# give up much of their volume by diffusion within the step cap (the uniform
# mixture has less free energy than the drop), so served runs use Pe = 10.
SERVE_PE = 10.0

# Four-roller cells: the extension rate eps at the centre per unit roller
# angular speed, by cell size N, once calibrated in this process.  Cylinders
# along z in a z-periodic box drive a two-dimensional flow, so one D2Q9 run
# serves 2D and 3D cells of the same N.
_ROLLER_RATE: dict[int, float] = {}


def roller_radius(n: int) -> float:
    """Roller radius of an N-cell four-roller box."""
    return 0.117 * n


def calibrate_rollers(n: int, tip_speed: float = 1e-3, tol: float = 1e-3, max_chunks: int = 12) -> float:
    """Extension rate at the centre of the N x N four-roller cell per unit
    roller angular speed, from a single-phase run at Stokes-like speeds
    (tip speed `tip_speed`) stepped until the centre rate changes by less
    than `tol` relative over a chunk of a quarter viscous time over the
    half box; the rate is the least-squares slope of u_x against x over the
    6 x 6 cells around the centre.  Cached per N."""
    from . import frelbm as F
    rr = roller_radius(n)
    cs, signs = synth.four_roller_geometry(n, n, rr)
    om = tip_speed / rr
    mask = synth.roller_mask((1, n, n), cs, rr)
    rollers = [(c, s * om, 2, rr) for c, s in zip(cs, signs)]
    p = F.make_params(F.FRE_D2Q9, (n, n, 1), rollers=rollers, A=1e-3, kappa=4e-3, tau_f=1.0, tau_g=1.0, M=0.1)
    L = F.Lattice(p, -np.ones((1, n, n)), None, None, mask)
    nu = (1.0 - 0.5) / 3.0
    chunk = max(100, int(0.25 * (n / 2.0) ** 2 / nu))
    c0 = n // 2 - 3
    xs = np.arange(c0, c0 + 6) - (n - 1) / 2.0
    prev = None
    eps = 0.0
    for _ in range(max_chunks):
        L.step(chunk)
        ux = L.read(("u",))["u"][0, 0, c0:c0 + 6, c0:c0 + 6]
        eps = float((ux * xs[None, :]).sum() / (6.0 * (xs * xs).sum()))
        if prev is not None and abs(eps - prev) <= tol * abs(eps):
            break
        prev = eps
    L.close()
    _ROLLER_RATE[n] = eps / om
    return _ROLLER_RATE[n]


def lattice_inputs(req: Request):
    """Parameters and initial fields of a request (shear: walls normal to the
    last axis moving at -+u_w with the linear shear profile; rollers: four
    cylinders along z, all axes periodic), Peclet number req.Pe (default
    SERVE_PE)."""
    from . import frelbm as F
    from .params import derive_params
    nx, ny, nz = req.shape
    sh = (nz, ny, nx)
    R = req.radius
    Pe = SERVE_PE if req.Pe is None else req.Pe
    if req.flow == "shear":
        wall_axis = 1 if req.kind == 0 else 2
        H = (ny, nz)[wall_axis - 1]
        dp = derive_params(Re=req.Re, Ca=req.Ca, radius=R, xi=req.xi, H=H, Pe=Pe)
        wu = np.zeros((3, 2, 3))
        wu[wall_axis, 0, 0] = -dp.wall_u
        wu[wall_axis, 1, 0] = dp.wall_u
        bc = [0, 0, 0]
        bc[wall_axis] = 1
        phi0 = synth.droplet_phi(sh, R, req.xi, noise=1e-4, seed=req.rid, dims=2 if req.kind == 0 else 3)
        u0 = synth.shear_velocity(sh, dp.rate, axis_normal=wall_axis)
        p = F.make_params(req.kind, (nx, ny, nz), storage=req.storage, bc=tuple(bc), wall_u=wu, **dp.phys())
        return p, phi0, u0, None, dp.rate
    # four rollers: the angular speed that gives the extension rate eps at the
    # centre, from the calibration of this N when there is one (see
    # calibrate_rollers), else the stagnation-flow estimate: tip speed eps * d
    # with d the gap from the centre to the roller surface
    dp = derive_params(Re=req.Re, Ca=req.Ca, radius=R, xi=req.xi, Pe=Pe)
    rr = roller_radius(nx)
    cs, signs = synth.four_roller_geometry(nx, ny, rr, nz=nz)
    k = _ROLLER_RATE.get(nx)
    om = dp.rate / k if k else dp.rate * (math.hypot(nx / 4.0, ny / 4.0) - rr) / rr
    mask = synth.roller_mask(sh, cs, rr)
    rollers = [(c, s * om, 2, rr) for c, s in zip(cs, signs)]
    # the drop sits on the stagnation point, the rollers' centre of symmetry
    phi0 = synth.droplet_phi(sh, R, req.xi, center=(nx / 2.0, ny / 2.0, (nz - 1) / 2.0), noise=1e-4,
                             seed=req.rid, dims=2 if req.kind == 0 else 3)
    p = F.make_params(req.kind, (nx, ny, nz), storage=req.storage, rollers=rollers, **dp.phys())
    return p, phi0, None, mask, dp.rate


class GpuEngine:
    """Lattices in torch-allocated device buffers, stepped by one Batch."""

    def __init__(self, budget_bytes: int, max_members: int, keep_final: bool = False,
                 calibrate_rollers: bool = True):
        from . import frelbm as F
        self.F = F
        cap = max(1 << 16, budget_bytes // 2048)
        self.batch = F.Batch(max_slots=max_members, max_work=cap, max_fill=cap)
        self.cap = cap
        self.work = self.fill = 0
        self.slots = {}
        self.keep_final = keep_final
        self.final = {}
        self._fp = {}
        self.masks = {}
        self.calibrate = calibrate_rollers

    def footprint(self, req: Request) -> int:
        if req.rid not in self._fp:
            p, *_ = lattice_inputs(req)
            try:
                self._fp[req.rid] = self.F.footprint(p)
            except self.F.FreError as e:
                if e.status != self.F.FRE_EINVAL:
                    raise
                raise InvalidRequest(str(e)) from e
        return self._fp[req.rid]

    def periodic(self, req: Request):
        if req.flow == "shear":
            return (True, req.kind != 0, req.kind == 0)
        return (True, True, True)

    def prepare(self, requests):
        """Calibrate the roller speed of every four-roller cell size the
        requests use (once per N and process)."""
        if self.calibrate:
            for n in sorted({r.shape[0] for r in requests if r.flow == "rollers"} - set(_ROLLER_RATE)):
                calibrate_rollers(n)

    def admit(self, req: Request):
        if self.calibrate and req.flow == "rollers" and req.shape[0] not in _ROLLER_RATE:
            calibrate_rollers(req.shape[0])
        p, phi0, u0, mask, rate = lattice_inputs(req)
        L = self.F.Lattice(p, phi0, None, u0, mask)
        w, f = self.F.Batch.needs(L)
        if self.work + w > self.cap or self.fill + f > self.cap:
            L.close()
            return None
        slot = self.batch.add(L)
        self.work += w
        self.fill += f
        self.slots[id(L)] = (slot, w, f, req.rid)
        if mask is not None:
            self.masks[id(L)] = mask != 0
        return L, rate

    def step(self, n: int):
        self.batch.step(n)

    def phi(self, L):
        try:
            L.reduce()          # FP64 totals and the non-finite check
        except self.F.FreError as e:
            if e.status == self.F.FRE_ENUMERIC:
                raise RunFailed(str(e)) from e
            raise
        return L.read(("phi",))["phi"]

    def solid(self, L):
        """Obstacle cells of a lattice (None without obstacles)."""
        return self.masks.get(id(L))

    def retire(self, L):
        slot, w, f, rid = self.slots.pop(id(L))
        self.masks.pop(id(L), None)
        if self.keep_final:
            self.final[rid] = (L.info()[0], L.populations())
        self.batch.remove(slot)
        self.work -= w
        self.fill -= f
        L.close()


def main(argv=None):
    """Serve the mixed request stream on the GPU and print the summary as one
    JSON line (each retirement is printed as it happens).  With the defaults
    this is the full sweep: 256 requests, Poisson arrivals at 20/s, D2Q9
    N = 64..512 and D3Q19 N = 48..160 in steps of 16, shear and four-roller,
    FP32 and FP16, Ca in [0.05, 0.4], Re in [0.1, 1], a 32 GiB budget."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__.split("\n\n")[0])
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--max-members", type=int, default=32)
    ap.add_argument("--strain-cap", type=float, default=25.0)
    ap.add_argument("--step-cap", type=int, default=200_000)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--out", default="", help="also write every outcome to this JSON file")
    args = ap.parse_args(argv)
    rs = make_requests(args.requests, rate=args.rate, seed=args.seed)
    budget = int(args.budget_gib * (1 << 30))
    eng = GpuEngine(budget_bytes=budget, max_members=args.max_members)

    def show(o):
        print(json.dumps({"rid": o.rid, "reason": o.reason, "steps": o.steps, "strain": round(o.strain, 3),
                          "D": round(o.D, 4), "cells": o.cells, "latency_s": round(o.latency, 3)}), flush=True)

    srv = Server(eng, budget, max_members=args.max_members, chunk=args.chunk, strain_cap=args.strain_cap,
                 step_cap=args.step_cap, on_retire=show)
    rep = srv.run(rs)
    s = rep.summary()
    s = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}
    s["workload"] = (f"{args.requests} requests, Poisson {args.rate}/s, D2Q9 N 64-512 / D3Q19 N 48-160, "
                     f"shear/rollers, FP32/FP16, caps {args.strain_cap} strain units or {args.step_cap} steps, "
                     f"{args.budget_gib} GiB budget, at most {args.max_members} members")
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"summary": s, "outcomes": [o.__dict__ for o in rep.outcomes]}, fh)
    print(json.dumps({"mode": "serving", **s}), flush=True)
    eng.batch.close()


if __name__ == "__main__":
    main()
