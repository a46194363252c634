"""Throughput of the FRE LBM step on one MI355X.

Workload: the D3Q19 shear droplet lattice 256x128x128 (walls in z moving at
-+u_w, periodic x, y), droplet R=25, xi=2, Ca=0.1, Re=1 (A=5.89e-3,
kappa=A xi^2, M=5.26 from Pe=0.43, tau_f=1, tau_g=1.74 for Cahn-Hilliard
stability), FP32 population storage; synthetic seeded
inputs, already resident in HBM when timing starts.  A step is one full
time step of the method (all kernels).  Prints one JSON line.

Modes for profiling (each prints its own JSON line):
  --kernels-only N   N individually launched steps of the workload, FP32 or
                     with --storage 1 FP16 (for rocprofv3 kernel traces and
                     counter runs)
  --copy-probe       a plain device-to-device copy of known size, the
                     reference for scaling the FETCH_SIZE / WRITE_SIZE counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_2212_01617_amd/csrc/kernels.hip", "paper_2212_01617_amd/csrc/lbm_device.h",
                  "paper_2212_01617_amd/csrc/kernels.h")
TRAFFIC_FILE = "profiles/traffic_k_collide_d3q19_fp32_256x128x128.txt"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of k_collide from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def workload(storage: int, shape=(256, 128, 128), R: float = 25.0, sr: bool = False):
    """The shear-droplet lattice: D3Q19, walls in z moving at -+u_w, periodic
    x and y, a drop of radius R mid-domain, Ca = 0.1, Re = 1, xi = 2."""
    from paper_2212_01617_amd import frelbm as F
    from paper_2212_01617_amd import synth
    from paper_2212_01617_amd.params import derive_params
    nx, ny, nz = shape
    xi = 2.0
    dp = derive_params(Re=1.0, Ca=0.1, radius=R, xi=xi, H=nz, Pe=0.43)
    gamma, uw = dp.rate, dp.wall_u
    wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -uw; wu[2, 1, 0] = uw
    sh = (nz, ny, nx)
    phi0 = synth.droplet_phi(sh, R, xi, noise=1e-4, seed=0)
    u0 = synth.shear_velocity(sh, gamma, axis_normal=2)
    phys = dp.phys()
    p = F.make_params(F.FRE_D3Q19, (nx, ny, nz), storage=storage, bc=(0, 0, 1), wall_u=wu,
                      stochastic_rounding=sr, **phys)
    return p, phi0, u0, dict(shape=(nx, ny, nz), wall_u=wu, phys=phys)


def bytes_per_lu(q: int, storage: int) -> int:
    """Algorithmic bytes per lattice update: every population of f and g read
    once and written once (FP16 storage keeps g_0 in FP32)."""
    if storage == 0:
        return 2 * 2 * q * 4
    return 2 * (q * 2 + (q - 1) * 2 + 4)


def time_steps(L, steps, warmup, reps):
    import torch
    L.step(warmup)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(L.stream)
        L.step(steps)
        e1.record(L.stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return float(np.median(times)), times


def large_lattice(steps: int = 100) -> dict:
    """The same workload scaled 2x per axis (512x256x256, R = 50, 33.6 M
    cells), a footprint many times the 256 MB Infinity Cache, FP32 and FP16
    storage, autotuned like the main leg."""
    import torch
    from paper_2212_01617_amd import frelbm as F
    out = {"workload": "D3Q19 shear droplet 512x256x256, walls in z, R=50, xi=2, Ca=0.1, Re=1"}
    for storage, key in ((0, "fp32"), (1, "fp16")):
        p, phi0, u0, meta = workload(storage, (512, 256, 256), 50.0)
        L = F.Lattice(p, phi0, None, u0, stream=torch.cuda.Stream())
        del phi0, u0
        L.autotune(5)
        ms, _ = time_steps(L, steps, 10, 3)
        n = 512 * 256 * 256
        mlups = n / (ms * 1e-3) / 1e6
        b = bytes_per_lu(19, storage)
        out[key] = {"value": round(mlups, 1), "unit": "MLUPS", "ms_per_step": round(ms, 5), "bytes_per_lu": b,
                    "step_frac": round(mlups * 1e6 * b / 1e9 / PEAK_HBM_GBS, 4),
                    "device_bytes": int(L._nbytes)}
        L.close()
        torch.cuda.empty_cache()
    return out


def consistent_init_rate(n: int = 400) -> dict:
    """Throughput of the consistent initialisation's pre-iterations on the
    256x128x128 workload (FP32): n pre-iterations timed against zero, so the
    host upload of (u0, phi0) and the final g reset cancel out."""
    import torch
    from paper_2212_01617_amd import frelbm as F
    p, phi0, u0, _ = workload(0)
    L = F.Lattice(p, phi0, None, u0, stream=torch.cuda.Stream())
    L.autotune(5)
    t = {}
    for k in (0, n, 0, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.consistent_init(phi0, u0, k)   # synchronises
        t.setdefault(k, []).append(time.perf_counter() - t0)
    L.close()
    ms = (min(t[n]) - min(t[0])) / n * 1e3
    cells = 256 * 128 * 128
    mlups = cells / (ms * 1e-3) / 1e6
    return {"value": round(mlups, 1), "unit": "MLUPS", "ms_per_iteration": round(ms, 5),
            "bytes_per_lu": 152, "frac": round(mlups * 1e6 * 152 / 1e9 / PEAK_HBM_GBS, 4),
            "sample": f"{n} pre-iterations minus 0, best of 2, FP32, 256x128x128"}


def ternary_rate(steps: int = 200) -> dict:
    """Throughput of a ternary lattice (third order parameter psi with its
    own population h) on the 256x128x128 shear workload: a drop of component
    1 in a 2-3 mixture, FP32 storage, captured two-step graphs.  The run is
    checked to stay finite."""
    import torch
    from paper_2212_01617_amd import frelbm as F
    p, phi0, u0, meta = workload(0)
    sh = phi0.shape
    c1 = 0.5 * (1.0 + phi0)
    psi0 = 0.3 * (1.0 - c1)
    phi = c1 - (1.0 - c1 - psi0)
    # kappa3 = 4A, the kappa of the other two; psi's gradient stiffness is then
    # alpha^2 ((kappa1 + kappa2) / 4 + kappa3) = 3 kappa against phi's kappa,
    # so psi's mobility is a third of phi's to keep Gamma times the stiffness
    # where the Cahn-Hilliard update is stable (with M3 = M this lattice
    # diverges within 20 steps)
    p.ternary = 1
    p.kappa3, p.M3, p.tau_h = 4.0 * p.A, p.M / 3.0, p.tau_g
    L = F.Lattice(p, phi, None, u0, psi0=psi0, stream=torch.cuda.Stream())
    ms, _ = time_steps(L, steps, 10, 3)
    L.reduce()                      # raises if any fluid cell went non-finite
    L.close()
    cells = sh[0] * sh[1] * sh[2]
    mlups = cells / (ms * 1e-3) / 1e6
    b = 2 * 3 * 19 * 4
    return {"value": round(mlups, 1), "unit": "MLUPS", "ms_per_step": round(ms, 5), "bytes_per_lu": b,
            "step_frac": round(mlups * 1e6 * b / 1e9 / PEAK_HBM_GBS, 4),
            "workload": "D3Q19 ternary shear droplet 256x128x128, walls in z, FP32 storage"}


def four_roller_lattice(storage: int):
    """Parameters, phi0 and mask of the four-roller workload (see four_roller)."""
    from paper_2212_01617_amd import frelbm as F
    from paper_2212_01617_amd import synth
    from paper_2212_01617_amd.params import derive_params
    nx, ny, nz, rr = 256, 256, 64, 30.0
    dp = derive_params(Re=0.5, Ca=0.1, radius=24.0, xi=2.0, Pe=0.43)
    cs, signs = synth.four_roller_geometry(nx, ny, rr, nz=nz)
    om = dp.rate * (np.hypot(nx / 4.0, ny / 4.0) - rr) / rr
    sh = (nz, ny, nx)
    mask = synth.roller_mask(sh, cs, rr)
    phi0 = synth.droplet_phi(sh, 24.0, 2.0, noise=1e-4, seed=0)
    p = F.make_params(F.FRE_D3Q19, (nx, ny, nz), storage=storage,
                      rollers=[(c, sg * om, 2, rr) for c, sg in zip(cs, signs)], **dp.phys())
    return p, phi0, mask


def four_roller(steps: int = 200) -> dict:
    """The four-roller cell: D3Q19 256x256x64, all axes periodic, four
    staircase cylinders of radius 30 along z at the quarter points spinning in
    alternation, a drop of radius 24 in the centre (xi = 2, Re = 0.5,
    Ca = 0.1).  17% of the cells are solid; MLUPS count fluid cells only.
    The roller speed is the stagnation-flow estimate (tip speed eps times
    the gap from the centre to the rollers); the rate does not depend on it,
    and the calibrated speed is used by campaign.four_roller_run."""
    import torch
    from paper_2212_01617_amd import frelbm as F
    _, _, mask = four_roller_lattice(0)
    n_fluid = int((mask == 0).sum())
    out = {"workload": "D3Q19 four-roller cell 256x256x64, rollers r=30 along z, drop R=24, xi=2, Re=0.5, Ca=0.1",
           "fluid_cells": n_fluid}
    for storage, key in ((0, "fp32"), (1, "fp16")):
        p, phi0, mask = four_roller_lattice(storage)
        L = F.Lattice(p, phi0, None, None, mask, stream=torch.cuda.Stream())
        L.autotune(5)
        ms, _ = time_steps(L, steps, 20, 3)
        mlups = n_fluid / (ms * 1e-3) / 1e6
        b = bytes_per_lu(19, storage)
        out[key] = {"value": round(mlups, 1), "unit": "MLUPS", "ms_per_step": round(ms, 5), "bytes_per_lu": b,
                    "step_frac": round(mlups * 1e6 * b / 1e9 / PEAK_HBM_GBS, 4)}
        L.close()
    return out


def shard(steps: int = 1000) -> dict:
    """One GPU's share of the 256x128x128 shear lattice split eight ways
    along z (its slowest axis in memory): 256x128x16 cells, the drop's
    central planes, at its real shape.  The slab's faces are periodic here;
    the exchange with the neighbouring slabs is not part of this path."""
    import torch
    from paper_2212_01617_amd import frelbm as F
    p0, phi0, u0, meta = workload(0)
    z0 = 56
    phi_s = np.ascontiguousarray(phi0[z0:z0 + 16])
    u_s = np.ascontiguousarray(u0[:, z0:z0 + 16])
    out = {"workload": "256x128x16 slab (planes 56-71) of the D3Q19 shear droplet 256x128x128, periodic faces"}
    for storage, key in ((0, "fp32"), (1, "fp16")):
        p = F.make_params(F.FRE_D3Q19, (256, 128, 16), storage=storage, **meta["phys"])
        L = F.Lattice(p, phi_s, None, u_s, stream=torch.cuda.Stream())
        L.autotune(5)
        ms, _ = time_steps(L, steps, 50, 3)
        n = 256 * 128 * 16
        mlups = n / (ms * 1e-3) / 1e6
        b = bytes_per_lu(19, storage)
        out[key] = {"value": round(mlups, 1), "unit": "MLUPS", "ms_per_step": round(ms, 5),
                    "step_frac": round(mlups * 1e6 * b / 1e9 / PEAK_HBM_GBS, 4)}
        L.close()
    return out


def cpu_table() -> dict:
    """The FP64 oracle's rate on the host cores at one thread and at all
    threads, each measurement in a child process of its own (the OpenMP
    thread count is fixed when the oracle library loads): the 100x100 D2Q9
    static drop, the 400x200 D2Q9 shear, the 64x32x32 D3Q19 copy and the full
    256x128x128 lattice (fewer steps at one thread)."""
    import subprocess
    allc = os.cpu_count() or 1
    try:
        allc = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    allc = int(os.environ.get("OMP_NUM_THREADS", allc))
    cases = (("static_drop_100x100_d2q9", 200, 200), ("shear_400x200_d2q9", 200, 200),
             ("copy_64x32x32_d3q19", 200, 200), ("shear_256x128x128_d3q19", 4, 20))
    rows = {}
    for name, st1, stn in cases:
        for th, st in ((1, st1), (allc, stn)):
            env = dict(os.environ, OMP_NUM_THREADS=str(th))
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-case", name, "--steps", str(st)],
                               env=env, capture_output=True, text=True, check=True)
            rows.setdefault(name, {})[f"{th}t"] = json.loads(r.stdout.strip().splitlines()[-1])
            print(f"[cpu] {name} {th} threads: {rows[name][f'{th}t']}", file=sys.stderr, flush=True)
    return {"threads_all": allc, "cpu_model": cpu_model(), "nproc": os.cpu_count(), "cases": rows}


def cpu_case(name: str, steps: int) -> dict:
    """One oracle timing (see cpu_table)."""
    from oracle import oracle as O
    from paper_2212_01617_amd import synth
    from paper_2212_01617_amd.params import derive_params
    if name == "static_drop_100x100_d2q9":
        phi0 = synth.droplet_phi((1, 100, 100), 20.0, 1.5, center=(49.5, 49.5, 0), noise=1e-4, seed=0, dims=2)
        L = O.Lattice(O.make_params(0, (100, 100, 1), A=0.04, kappa=0.09, tau_f=1.0, tau_g=1.0, M=0.1), phi0)
        n = 100 * 100
    elif name == "shear_400x200_d2q9":
        dp = derive_params(Re=0.5, Ca=0.1, radius=40.0, xi=2.0, H=200, Pe=0.43)
        wu = np.zeros((3, 2, 3)); wu[1, 0, 0] = -dp.wall_u; wu[1, 1, 0] = dp.wall_u
        sh = (1, 200, 400)
        L = O.Lattice(O.make_params(0, (400, 200, 1), bc=(0, 1, 0), wall_u=wu, **dp.phys()),
                      synth.droplet_phi(sh, 40.0, 2.0, noise=1e-4, seed=0, dims=2), None,
                      synth.shear_velocity(sh, dp.rate, axis_normal=1))
        n = 400 * 200
    else:
        shape, R = ((64, 32, 32), 6.25) if name == "copy_64x32x32_d3q19" else ((256, 128, 128), 25.0)
        dp = derive_params(Re=1.0, Ca=0.1, radius=25.0, xi=2.0, H=128, Pe=0.43)
        nx, ny, nz = shape
        uw = dp.rate * nz / 2.0
        wu = np.zeros((3, 2, 3)); wu[2, 0, 0] = -uw; wu[2, 1, 0] = uw
        sh = (nz, ny, nx)
        L = O.Lattice(O.make_params(1, shape, bc=(0, 0, 1), wall_u=wu, **dp.phys()),
                      synth.droplet_phi(sh, R, 2.0, noise=1e-4, seed=0), None,
                      synth.shear_velocity(sh, dp.rate, axis_normal=2))
        n = nx * ny * nz
    L.step(1)
    t0 = time.perf_counter()
    L.step(steps)
    dt = time.perf_counter() - t0
    return {"MLUPS": round(n * steps / dt / 1e6, 3), "steps": steps, "seconds": round(dt, 2)}


def cpu_model() -> str:
    """The host CPU's model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p_gpu, phi0, u0, meta, steps=60):
    from oracle import oracle as O
    nx, ny, nz = meta["shape"]
    po = O.make_params(1, (nx, ny, nz), bc=(0, 0, 1), wall_u=meta["wall_u"], **meta["phys"])
    L = O.Lattice(po, phi0, None, u0)
    L.step(1)  # first touch
    t0 = time.perf_counter()
    L.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nx * ny * nz * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{steps} steps of the full 256x128x128 D3Q19 lattice (FP64 oracle, OpenMP, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 512x256x256 leg")
    ap.add_argument("--serve", type=int, default=24, help="requests in the serving leg (0: skip)")
    ap.add_argument("--kernels-only", type=int, default=0)
    ap.add_argument("--storage", type=int, default=0, help="with --kernels-only: 0 FP32, 1 FP16")
    ap.add_argument("--four-roller", action="store_true", help="with --kernels-only: the four-roller cell")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--shape", default="", help="with --kernels-only: rows,xcd for k_moments, "
                    "k_potential, k_collide, e.g. 4,1,4,1,4,1 (default shapes if empty)")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--ternary-only", type=int, default=0, help="only the ternary leg, this many timed steps")
    ap.add_argument("--serve-steady-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-extra", action="store_true", help="skip the four-roller and shard legs")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the FP64 oracle at 1 and all threads on four cases (no GPU)")
    ap.add_argument("--cpu-case", default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_case:
        print(json.dumps(cpu_case(args.cpu_case, args.steps)), flush=True)
        return
    if args.cpu_table:
        print(json.dumps({"mode": "cpu-table", **cpu_table()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(one lattice per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2212_01617_amd import frelbm as F
    if not os.path.exists(F.LIB_PATH):
        from paper_2212_01617_amd import build
        build.build()
    torch.cuda.init()
    stream = torch.cuda.Stream()
    if args.copy_probe:
        copy_probe()
        return
    if args.ternary_only:
        print(json.dumps({"mode": "ternary", **ternary_rate(args.ternary_only)}), flush=True)
        return
    if args.serve_steady_only:
        print(json.dumps({"mode": "serving-steady", **serving_steady()}), flush=True)
        return
    if args.kernels_only:
        if args.four_roller:
            p, phi0, mask = four_roller_lattice(args.storage)
            L = F.Lattice(p, phi0, None, None, mask, stream=stream)
        else:
            p, phi0, u0, meta = workload(args.storage)
            L = F.Lattice(p, phi0, None, u0, stream=stream)
        if args.shape:
            v = [int(t) for t in args.shape.split(",")]
            L.set_launch_shape({k: (v[2 * i], v[2 * i + 1]) for i, k in enumerate(L.STAGES)})
        prof = L.profile(args.kernels_only)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "kernels-only", "steps": args.kernels_only, "launch_shape": L.launch_shape(),
                          "kernels_ms": {k: round(v, 5) for k, v in prof.items()}}), flush=True)
        return

    res = {}
    for storage in ((0,) if args.no_fp16 else (0, 1, 2)):  # 2: FP16 with stochastic rounding
        p, phi0, u0, meta = workload(min(storage, 1), sr=storage == 2)
        L = F.Lattice(p, phi0, None, u0, stream=stream)
        tuned = L.autotune(10) if not args.no_tune else None
        ms, all_ms = time_steps(L, args.steps, args.warmup, args.reps)
        n_fluid = meta["shape"][0] * meta["shape"][1] * meta["shape"][2]
        prof = L.profile(100)   # per-kernel means over 100 individually launched steps
        ok = L.reduce()
        res[storage] = dict(ms=ms, all_ms=all_ms, n=n_fluid, prof=prof, L=L, meta=meta,
                            p=p, phi0=phi0, u0=u0, sums=ok, shape=L.launch_shape())

    r = res[0]
    n = r["n"]
    mlups = n / (r["ms"] * 1e-3) / 1e6
    b = bytes_per_lu(19, 0)
    dom = max(r["prof"], key=r["prof"].get)
    dom_ms = r["prof"][dom]
    achieved = b * n / (dom_ms * 1e-3) / 1e9
    out = {
        "metric": "MLUPS and %HBM roofline (D3Q19 FP32 vs FP16-store); p50/p99 run latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 5),
        "ms_per_step_min_max": [round(min(r["all_ms"]), 5), round(max(r["all_ms"]), 5)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D3Q19 shear droplet 256x128x128, walls in z, R=25, xi=2, Ca=0.1, Re=1, FP32 storage",
                   "storage": "fp32", "fluid_cells": n, "bytes_per_lu": b},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch",
                     "kernel": dom, "kernel_ms": round(dom_ms, 5),
                     "step_frac": round(mlups * 1e6 * b / 1e9 / PEAK_HBM_GBS, 4)},
        "kernels_ms": {k: round(v, 5) for k, v in r["prof"].items()},
        "launch_shape": {k: {"rows": v[0], "xcd": v[1]} for k, v in r["shape"].items()},
    }
    cp = copy_rate()
    out["copy_ceiling_GBps"] = cp["GBps"]
    out["roofline"]["frac_of_copy_ceiling"] = round(achieved / cp["GBps"], 4)
    if 1 in res:
        r16 = res[1]
        m16 = r16["n"] / (r16["ms"] * 1e-3) / 1e6
        b16 = bytes_per_lu(19, 1)
        out["fp16_store"] = {"value": round(m16, 1), "unit": "MLUPS", "ms_per_step": round(r16["ms"], 5),
                             "ms_per_step_min_max": [round(min(r16["all_ms"]), 5), round(max(r16["all_ms"]), 5)],
                             "bytes_per_lu": b16, "step_frac": round(m16 * 1e6 * b16 / 1e9 / PEAK_HBM_GBS, 4),
                             "kernels_ms": {k: round(v, 5) for k, v in r16["prof"].items()},
                             "launch_shape": {k: {"rows": v[0], "xcd": v[1]} for k, v in r16["shape"].items()}}
    if 2 in res:
        r2 = res[2]
        m2 = r2["n"] / (r2["ms"] * 1e-3) / 1e6
        out["fp16_store"]["stochastic_rounding"] = {
            "value": round(m2, 1), "unit": "MLUPS", "ms_per_step": round(r2["ms"], 5),
            "kernels_ms": {k: round(v, 5) for k, v in r2["prof"].items()}}
    for v in res.values():
        v["L"].close()
    res.clear()
    if not args.no_large:
        out["large_lattice"] = large_lattice()
    out["consistent_init"] = consistent_init_rate()
    out["ternary"] = ternary_rate()
    if not args.no_extra:
        out["four_roller"] = four_roller()
        out["shard"] = shard()
    if args.serve:
        out["serving"] = serving(args.serve)
        if not args.no_extra:
            out["serving_steady"] = serving_steady()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(r["p"], r["phi0"], r["u0"], r["meta"])
    print(json.dumps(out), flush=True)


def serving(n_requests: int) -> dict:
    """Continuous batching of a mixed droplet request stream (Poisson
    arrivals at 20/s; D2Q9 N in 64..256 and D3Q19 N in 48..96, shear and
    four-roller, FP32 and FP16, Ca in [0.05, 0.4], Re in [0.1, 1]; R = 0.2 N,
    xi = 2) under a 16 GiB budget; caps of 10 strain units or 20000 steps."""
    from paper_2212_01617_amd import serve
    rs = serve.make_requests(n_requests, rate=20.0, seed=0, d2_sizes=tuple(range(64, 257, 16)),
                             d3_sizes=tuple(range(48, 97, 16)))
    budget = 16 << 30
    eng = serve.GpuEngine(budget_bytes=budget, max_members=32)
    srv = serve.Server(eng, budget, max_members=32, chunk=200, strain_cap=10.0, step_cap=20_000)
    rep = srv.run(rs)
    s = rep.summary()
    s = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}
    s["workload"] = (f"{n_requests} requests, Poisson 20/s, D2Q9 N 64-256 / D3Q19 N 48-96, shear/rollers, "
                     "FP32/FP16, caps 10 strain units or 20000 steps, 16 GiB budget")
    eng.batch.close()
    return s


def serving_steady(n_requests: int = 16) -> dict:
    """Continuous batching of 2D shear drops that settle within the caps, so
    that time-to-steady is measured: D2Q9, N in {64, 80, 96} (2N x N boxes,
    R = 0.2 N), Ca in [0.05, 0.2], Re in [0.5, 1], FP32 and FP16, Poisson
    arrivals at 20/s; caps of 40 strain units or 200,000 steps."""
    import dataclasses
    from paper_2212_01617_amd import serve
    base = serve.make_requests(n_requests, rate=20.0, seed=1, d2_sizes=(64, 80, 96), d3_sizes=(64,),
                               Ca=(0.05, 0.2), Re=(0.5, 1.0))
    rs = [dataclasses.replace(r, kind=0, flow="shear") for r in base]
    budget = 16 << 30
    eng = serve.GpuEngine(budget_bytes=budget, max_members=n_requests)
    srv = serve.Server(eng, budget, max_members=n_requests, chunk=200, strain_cap=40.0, step_cap=200_000)
    rep = srv.run(rs)
    s = rep.summary()
    s = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}
    s["workload"] = (f"{n_requests} requests, Poisson 20/s, D2Q9 shear N 64-96, Ca 0.05-0.2, Re 0.5-1, FP32/FP16, "
                     "caps 40 strain units or 200000 steps, 16 GiB budget")
    eng.batch.close()
    return s


def copy_rate(nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """A plain device-to-device copy of nbytes (read once, written once),
    repeated after one warm-up copy: its rate is the copy ceiling of HBM on
    this box, measured beside the 8 TB/s peak.  The same launches are the
    reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "reps": reps, "ms": round(ms, 4),
            "GBps": round(2 * nbytes / ms / 1e6, 1)}


def copy_probe(nbytes: int = 1 << 30, reps: int = 5) -> None:
    print(json.dumps({"mode": "copy-probe", **copy_rate(nbytes, reps)}), flush=True)


if __name__ == "__main__":
    main()
