"""Long oracle runs stored for the GPU parity tests.

Two cases from the benchmark set are run in the FP64 oracle for their long
horizons, and their end states are stored in ``long_runs.npz`` (phi and the
velocity components, as float32: their rounding, 6e-8 relative, lies far
below the 1e-5 parity bar):

* ``c3_copy``: the 64x32x32 D3Q19 copy of the 3D shear case (the per-cell
  parameters and shear rate of the 256x128x128 lattice: Re = 1, Ca = 0.1,
  walls in z at -+u_w, R = 6.25, xi = 2), 20,000 steps;
* ``shear_2d``: the 400x200 D2Q9 parallel-band shear (Re = 0.5, Ca = 0.1,
  R = 40, xi = 2, walls in y), 40,000 steps.

Inputs are the seeded synthetic fields of ``synth`` and the parameter rule of
``params`` (shear rate from Re, surface tension from Ca, A and kappa from
sigma and xi, M from the Peclet number); the stored metadata records the
parameters used, so a test can check that it rebuilds the same case.

    python tests/golden/long_runs.py          # about 25 minutes: the 3D case takes
                                              # about 10 on 8 cores, the 2D one runs
                                              # on one (the oracle threads over planes)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(os.path.dirname(_HERE))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

from paper_2212_01617_amd import synth  # noqa: E402
from paper_2212_01617_amd.params import derive_params  # noqa: E402

PATH = os.path.join(_HERE, "long_runs.npz")


def case(name: str) -> dict:
    """Inputs of one stored case: kind, (nx, ny, nz), steps, bc, wall_u,
    physical parameters, phi0, u0, the deformation plane and periodicity."""
    if name == "c3_copy":
        dp = derive_params(Re=1.0, Ca=0.1, radius=25.0, xi=2.0, H=128, Pe=0.43)
        nx, ny, nz = 64, 32, 32
        uw = dp.rate * nz / 2.0
        wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -uw; wu[2, 1, 0] = uw
        sh = (nz, ny, nx)
        return dict(kind=1, shape=(nx, ny, nz), steps=20000, bc=(0, 0, 1), wall_u=wu, phys=dp.phys(),
                    phi0=synth.droplet_phi(sh, 6.25, 2.0, noise=1e-4, seed=0),
                    u0=synth.shear_velocity(sh, dp.rate, axis_normal=2), plane="xz",
                    periodic=(True, True, False))
    if name == "shear_2d":
        nx, ny = 400, 200
        dp = derive_params(Re=0.5, Ca=0.1, radius=40.0, xi=2.0, H=ny, Pe=0.43)
        wu = np.zeros((3, 2, 3)); wu[1, 0, 0] = -dp.wall_u; wu[1, 1, 0] = dp.wall_u
        sh = (1, ny, nx)
        return dict(kind=0, shape=(nx, ny, 1), steps=40000, bc=(0, 1, 0), wall_u=wu, phys=dp.phys(),
                    phi0=synth.droplet_phi(sh, 40.0, 2.0, noise=1e-4, seed=0, dims=2),
                    u0=synth.shear_velocity(sh, dp.rate, axis_normal=1), plane="xy",
                    periodic=(True, False, True))
    raise KeyError(name)


CASES = ("c3_copy", "shear_2d")


def load() -> tuple[dict, dict]:
    """(metadata per case, arrays keyed '<case>__<field>')."""
    with np.load(PATH, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        arrays = {k: z[k] for k in z.files if k != "meta"}
    return meta, arrays


def main() -> None:
    from oracle import oracle as O
    meta, arrays = {}, {}
    for name in CASES:
        c = case(name)
        t0 = time.time()
        ref = O.Lattice(O.make_params(c["kind"], c["shape"], bc=c["bc"], wall_u=c["wall_u"], **c["phys"]),
                        c["phi0"], None, c["u0"])
        ref.step(c["steps"])
        obs = ref.observe()
        fields = ("phi", "ux", "uy", "uz") if c["kind"] == 1 else ("phi", "ux", "uy")
        for f in fields:
            arrays[f"{name}__{f}"] = obs[f].astype(np.float32)
        meta[name] = dict(steps=c["steps"], shape=list(c["shape"]), phys=c["phys"],
                          wall_u=np.asarray(c["wall_u"]).tolist(), fields=list(fields))
        print(f"{name}: {c['steps']} steps in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(PATH, meta=np.array(json.dumps(meta)), **arrays)
    print(f"wrote {PATH} ({os.path.getsize(PATH) / 1e6:.2f} MB)", flush=True)


if __name__ == "__main__":
    main()
