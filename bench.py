#!/usr/bin/env python3
"""Throughput of the hybrid-mesh DG hot path on one MI355X.

Workload (default): the four-slab hybrid mesh on 48^3 cubes (hex | wedge |
pyramid+tet | tet slabs, interior vertices jittered by 10% of h, seed 0),
order N = 4, Gaussian pressure pulse (width 0.05, centre from the seed),
u = 0, rigid walls, single-rate LSERK4 at the derived stable step for T = 0.5.
One "step" is one LSERK4 step: five stages, each one fused kernel per
element type.  The metric is GDOF/s per RK stage: element-node dofs of one
scalar field updated per stage per second (x1e-9).

Prints one JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def tet_alg_bytes(N: int, lattice: bool) -> int:
    """Algorithmic HBM bytes per tetrahedron per stage of the fused kernel.

    State: read U and res, write U and res (4 fields, FP32): 64 B per node.
    Traces: write the element's own traces and read the neighbour's (4 fields,
    FP32): 32 B per trace point, on 4 faces; a trace point is a face-lattice
    node ((N+1)(N+2)/2 per face) with lattice traces, else a cubature point
    ((N+1)^2 per face).
    Element data: 10 geometry floats read as 12, (kappa, 1/rho), 4 face
    records (normal + J^s, neighbour slot, orientation, penalties):
    48 + 8 + 4 * (16 + 4 + 1 + 8).
    """
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    npt = (N + 1) * (N + 2) // 2 if lattice else (N + 1) ** 2
    return 64 * Np + 32 * 4 * npt + 48 + 8 + 4 * (16 + 4 + 1 + 8)


def csrc_hash() -> str:
    """sha256 (first 16 hex) over the library's native sources, in name order."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1507_02557_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name: str, also: str = ""):
    """HBM bytes per launch of a kernel from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings),
    or None when the sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("source_hash") != csrc_hash():
        return None
    for name, b in data.get("bytes_per_launch", {}).items():
        if kernel_name in name and also in name:
            return float(b)
    return None


def cpu_baseline(n: int, N: int, stages: int):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.solver import LSERK_A, LSERK_B, Disc
    from paper_1507_02557_amd.inputs import four_slab_mesh, gaussian_pulse, pulse_centre

    mesh = four_slab_mesh(n, seed=0, jitter=0.1)
    d = Disc(mesh, N)
    c = pulse_centre(0)
    U = d.project(lambda x, y, z, t: gaussian_pulse(x, y, z, c))
    dt = d.dt_min(0.5)
    res = {t: np.zeros_like(U[t]) for t in d.types}
    dofs = sum(d.els[t].size * d.refs[t].Np for t in d.types)
    t0 = time.perf_counter()
    for s in range(stages):
        R = d.rhs(U)
        for t in d.types:
            res[t] = LSERK_A[s % 5] * res[t] + dt * R[t]
            U[t] = U[t] + LSERK_B[s % 5] * res[t]
    el = time.perf_counter() - t0
    threads = max([1] + [p.get("num_threads", 1) for p in threadpool_info()])
    return {"value": dofs * stages / el / 1e9, "unit": "GDOF/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 oracle, {stages} LSERK4 stages on the n={n} four-slab mesh "
                      f"({mesh.n_elem} elements, {dofs} dofs/field, N={N}); {el:.1f} s on "
                      f"{os.cpu_count()} visible host cores"}


def copy_calibration(mib: int):
    """One plain device-to-device copy of known size: under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE give the counter scale for HBM traffic."""
    import torch

    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--cpu-n", type=int, default=12)
    ap.add_argument("--cpu-stages", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib)
        return

    import numpy as np
    import torch

    from paper_1507_02557_amd import hdg
    from paper_1507_02557_amd.inputs import four_slab_mesh, gaussian_pulse, pulse_centre

    N = args.order
    mesh = four_slab_mesh(args.n, seed=0, jitter=0.1)
    c = pulse_centre(0)
    T = 0.5
    prof_steps = max(2, args.steps // 4)

    def run(precision: int, dt: float | None):
        s = hdg.Solver(mesh, N, bc=hdg.BC_RIGID_WALL, precision=precision)
        s.project_function(lambda x, y, z, t: gaussian_pulse(x, y, z, c))
        if dt is None:
            _, dtmin = s.dt(0.5)
            dt = T / math.ceil(T / dtmin)
        s.step(dt, args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(dt, args.steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        # per-kernel durations (events on the launch stream around each launch)
        s.profile(True)
        s.step(dt, prof_steps)
        kms, kcnt = s.profile_read()
        s.profile(False)
        state = {t: s.get_field(t).clone() for t in s.types}
        return s, dt, ms, kms, kcnt, state

    s, dt, ms, kms, kcnt, state32 = run(hdg.PREC_FP32, None)
    dofs = sum(s.info[t][0] * s.info[t][1] for t in s.types)
    stages = 5 * args.steps
    gdofs = dofs * stages / (ms * 1e-3) / 1e9
    avg_ms = {hdg.TET: kms[3] / max(kcnt[3], 1)}
    per_type = {name: round(float(kms[t] / max(kcnt[t], 1)), 4)
                for t, name in ((0, "hex"), (1, "wedge"), (2, "pyr"), (3, "tet")) if kcnt[t]}
    Ktet = s.info[hdg.TET][0]
    lattice = s.get_path()[1] == 1
    tet_kernel = f"TetMfma<{N}, " if lattice else f"TetStage<{N}, "
    alg_bytes = tet_alg_bytes(N, lattice) * Ktet
    achieved = alg_bytes / (avg_ms[hdg.TET] * 1e-3) / 1e9
    E = s.energy()
    info = dict(s.info)
    types = list(s.types)
    s.close()
    del s

    # the same workload with split-FP16 matrix-core products
    s16, _, ms16, kms16, kcnt16, state16 = run(hdg.PREC_FP16X2, dt)
    gdofs16 = dofs * stages / (ms16 * 1e-3) / 1e9
    num = sum(float(((state16[t].double() - state32[t].double()) ** 2).sum()) for t in types)
    den = sum(float((state32[t].double() ** 2).sum()) for t in types)
    mixed = {
        "precision": "split FP16 operands (hi + lo, power-of-two scales), FP32 accumulation, 16x16x32 MFMA, "
                     "tetrahedra; other types FP32",
        "value": round(gdofs16, 4),
        "unit": "GDOF/s",
        "speedup_vs_fp32_plain": round(gdofs16 / gdofs, 4),
        "stage_ms": round(ms16 / stages, 4),
        "kernel_ms_per_launch": {name: round(float(kms16[t] / max(kcnt16[t], 1)), 4)
                                 for t, name in ((0, "hex"), (1, "wedge"), (2, "pyr"), (3, "tet")) if kcnt16[t]},
        "rel_l2_vs_fp32_path": math.sqrt(num / den),
        "steps_compared": args.warmup + args.steps + prof_steps,
    }
    s16.close()
    del s16

    out = {
        "metric": "GDOF/s per RK stage: mixed-precision vs FP32 plain, at rel L2 <= 1e-5 vs FP64",
        "value": round(gdofs, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"four-slab hybrid mesh n={args.n} (jitter 0.1h, seed 0), N={N}, Gaussian pulse, "
                        f"rigid walls, single-rate LSERK4, FP32 plain",
            "elements": {name: int(info[t][0]) for t, name in ((0, "hex"), (1, "wedge"), (2, "pyr"), (3, "tet"))},
            "dofs_per_field": int(dofs),
            "dt": dt,
            "stage_ms": round(ms / stages, 4),
            "kernel_ms_per_launch": per_type,
            "energy_after": E,
            "mixed_precision": mixed,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("tet_mfma_kernel" if lattice else "stage_kernel") + f"<{tet_kernel}...>",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(tet_kernel, ", 0>" if lattice else ""),
            "alg_bytes_per_launch": int(alg_bytes),
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, N, args.cpu_stages)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
