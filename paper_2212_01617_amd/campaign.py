"""Critical capillary number of drop breakup in shear, on the serving engine.

Sec. 3.2 reports that a drop of radius a = 30 in shear breaks up above
Ca_c ~ 0.7 in 2D and ~ 0.42 in 3D, and shows a 2D breakup with end-pinching
and capillary waves at Ca = 3.5 (Re = 1, a = 40).  A sweep serves one shear
request per capillary number through the batch (all admitted at once); each
retires on breakup (two or more components of {phi > 0}), on a steady
deformation, or at the strain cap, and the critical range is read off the
outcomes.  Geometry and parameters are those of the serving requests: a
2N x N (x N) box with walls normal to the last axis, drop radius 0.2 N,
Peclet number ``serve.SERVE_PE``.

    python -m paper_2212_01617_amd.campaign --n 150 --Re 0.0625 --xi 1.5 \\
        --cas 0.5,0.7,1.0,1.5,2.0 --cap 30
"""
from __future__ import annotations

import argparse
import json
import sys

from . import serve


def sweep_requests(cas, *, kind: int = 0, n: int = 150, Re: float = 0.0625, xi: float = 1.5,
                   storage: int = 0, Pe: float | None = None) -> list:
    """One shear request per capillary number, all arriving at t = 0."""
    return [serve.Request(k, 0.0, kind, int(n), "shear", storage, float(ca), float(Re), float(xi), Pe)
            for k, ca in enumerate(cas)]


class _Logged:
    """An engine that reports its work: every `every`-th sample and every
    retirement go to `log`."""

    def __init__(self, engine, log, every: int = 50):
        self._e, self._log, self._every, self._n = engine, log, every, 0

    def __getattr__(self, name):
        return getattr(self._e, name)

    def phi(self, h):
        out = self._e.phi(h)
        self._n += 1
        if self._n % self._every == 0:
            self._log(f"[campaign] {self._n} samples")
        return out

    def retire(self, h):
        self._log(f"[campaign] a run retired after {self._n} samples")
        return self._e.retire(h)


def breakup_sweep(cas, *, kind: int = 0, n: int = 150, Re: float = 0.0625, xi: float = 1.5,
                  storage: int = 0, strain_cap: float = 30.0, budget_bytes: int = 8 << 30,
                  engine=None, log=None, Pe: float | None = None) -> list[dict]:
    """Serve the sweep and return one row per capillary number: the reason
    it retired ("breakup", "steady", "cap", ...), the strain reached and the
    last Taylor deformation D sampled before retirement.  `log`, if given,
    receives progress lines."""
    reqs = sweep_requests(cas, kind=kind, n=n, Re=Re, xi=xi, storage=storage, Pe=Pe)
    own = engine is None
    eng = serve.GpuEngine(budget_bytes, max_members=len(reqs)) if own else engine
    srv = serve.Server(_Logged(eng, log) if log else eng, budget_bytes, max_members=len(reqs), chunk=4000,
                       strain_cap=strain_cap, step_cap=1 << 62)
    rep = srv.run(reqs)
    if own:
        eng.batch.close()
    by_id = {o.rid: o for o in rep.outcomes}
    return [{"Ca": r.Ca, "reason": by_id[r.rid].reason, "strain": round(by_id[r.rid].strain, 2),
             "D": round(by_id[r.rid].D, 4), "steps": by_id[r.rid].steps} for r in reqs]


def critical_range(rows) -> tuple:
    """(largest Ca that did not break, smallest Ca that broke); None for a
    side with no such run.  A capped run counts as not broken within the cap.
    A first value above the second means the outcomes were not monotone in
    Ca (e.g. a run that would break later than the cap)."""
    intact = [r["Ca"] for r in rows if r["reason"] in ("steady", "cap")]
    broken = [r["Ca"] for r in rows if r["reason"] == "breakup"]
    return (max(intact) if intact else None, min(broken) if broken else None)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kind", type=int, default=0, help="0 D2Q9, 1 D3Q19")
    ap.add_argument("--n", type=int, default=150, help="box 2N x N (x N), drop radius 0.2 N")
    ap.add_argument("--Re", type=float, default=0.0625)
    ap.add_argument("--xi", type=float, default=1.5)
    ap.add_argument("--cas", default="0.5,0.7,1.0,1.5,2.0")
    ap.add_argument("--cap", type=float, default=30.0, help="strain cap")
    ap.add_argument("--storage", type=int, default=0)
    ap.add_argument("--Pe", type=float, default=serve.SERVE_PE)
    a = ap.parse_args(argv)
    rows = breakup_sweep([float(c) for c in a.cas.split(",")], kind=a.kind, n=a.n, Re=a.Re, xi=a.xi,
                         storage=a.storage, strain_cap=a.cap, Pe=a.Pe,
                         log=lambda line: print(line, file=sys.stderr, flush=True))
    lo, hi = critical_range(rows)
    print(json.dumps({"kind": a.kind, "n": a.n, "radius": 0.2 * a.n, "Re": a.Re, "xi": a.xi,
                      "Pe": a.Pe, "runs": rows, "critical_Ca_between": [lo, hi]}), flush=True)


if __name__ == "__main__":
    main()
