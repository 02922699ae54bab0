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


def alg_bytes(t: int, N: int, lattice: bool) -> int:
    """Algorithmic HBM bytes per element per stage of the fused kernel of type t.

    State: read U and res, write U and res (4 fields, FP32): 64 B per node.
    Traces: write the element's own trace and read the neighbour's (4 fields,
    FP32): 32 B per trace point; a triangle shared by tetrahedra/pyramids
    carries (N+1)(N+2)/2 lattice points with lattice traces, every other face
    (N+1)^2 cubature points.
    Geometry: the smaller of what the element needs to rebuild it (its
    vertices in FP64, 24 B each) and the stored per-element factors (tet: 12
    floats + 4 face normals with J^s).  Material (kappa, 1/rho): 8 B.  Face
    records (neighbour slot, orientation, penalties): 13 B per face.
    """
    n1 = N + 1
    nfn, nfq = (N + 1) * (N + 2) // 2, n1 * n1
    tri = nfn if lattice else nfq
    if t == 3:  # tetrahedron
        np_ = (N + 1) * (N + 2) * (N + 3) // 6
        return 64 * np_ + 32 * 4 * tri + min(4 * 24, 48 + 4 * 16) + 8 + 4 * 13
    if t == 2:  # pyramid: base quad + 4 triangles
        np_ = (N + 1) * (N + 2) * (2 * N + 3) // 6
        return 64 * np_ + 32 * (nfq + 4 * tri) + 5 * 24 + 8 + 5 * 13
    if t == 1:  # wedge: 2 triangles (wedge-wedge: cubature) + 3 quads
        np_ = n1 * nfn
        return 64 * np_ + 32 * 5 * nfq + 6 * 24 + 8 + 5 * 13
    np_ = n1 ** 3  # hexahedron
    return 64 * np_ + 32 * 6 * nfq + 8 * 24 + 8 + 6 * 13


def tet_alg_bytes(N: int, lattice: bool) -> int:
    return alg_bytes(3, N, lattice)


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
    ap.add_argument("--no-mrab", action="store_true", help="skip the multi-rate (MRAB3) measurement")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1"}))
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
    Ktet = s.info[hdg.TET][0]
    lattice = s.get_path()[1] == 1
    # kernel names as rocprofv3 reports them (for the committed traffic counters)
    kname = {3: (f"TetMfma<{N}, ", ", 0>") if lattice else (f"TetStage<{N}, ", ""),
             2: (f"PyrMfma<{N}, ", "") if (lattice and N in (3, 4)) else (f"PyrStage<{N}, ", ""),
             1: (f"WedgeStage<{N}, ", ""), 0: (f"HexStage<{N}, ", "")}
    kfull = {3: "tet_mfma_kernel" if lattice else "stage_kernel",
             2: "pyr_mfma_kernel" if (lattice and N in (3, 4)) else "stage_kernel",
             1: "stage_kernel", 0: "stage_kernel"}
    roof = {}
    for t, name in ((0, "hex"), (1, "wedge"), (2, "pyr"), (3, "tet")):
        if not kcnt[t]:
            continue
        ms_t = kms[t] / kcnt[t]
        b = alg_bytes(t, N, lattice) * s.info[t][0]
        ach = b / (ms_t * 1e-3) / 1e9
        roof[name] = {"bound": "hbm", "kernel": f"{kfull[t]}<{kname[t][0]}...>", "ms_per_launch": round(ms_t, 4),
                      "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(ach / HBM_PEAK_GBS, 4),
                      "traffic": measured_traffic(*kname[t]), "alg_bytes_per_launch": int(b),
                      "alg_bytes_per_element": alg_bytes(t, N, lattice)}
    dominant = max(roof, key=lambda k: roof[k]["ms_per_launch"])
    per_type = {k: v["ms_per_launch"] for k, v in roof.items()}
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

    # the same workload advanced by the multi-rate AB3 scheme (three levels,
    # Section 2.4): simulated time per second against single-rate LSERK4
    multi = None
    if not args.no_mrab:
        L = 3
        smr = hdg.Solver(mesh, N, bc=hdg.BC_RIGID_WALL)
        smr.project_function(lambda x, y, z, t: gaussian_pulse(x, y, z, c))
        dtmin_mr, cnt, _ = smr.mrab_setup(L)
        smr.mrab_advance(0)  # start-up (two coarse steps of LSERK4 at dt_min)
        smr.mrab_advance(1)  # warm-up coarse step
        torch.cuda.synchronize()
        n_coarse = max(2, args.steps // 4)
        m0 = torch.cuda.Event(enable_timing=True)
        m1 = torch.cuda.Event(enable_timing=True)
        m0.record()
        t_adv = smr.mrab_advance(n_coarse)
        m1.record()
        torch.cuda.synchronize()
        ms_mr = m0.elapsed_time(m1)
        rate_mr = t_adv / (ms_mr * 1e-3)
        rate_rk = dt * args.steps / (ms * 1e-3)
        multi = {
            "scheme": f"MRAB3, {L} levels (coarse step 2^{L - 1} dt_min), FP32",
            "elements_per_level": [int(x) for x in cnt],
            "dt_min": dtmin_mr,
            "coarse_steps_timed": n_coarse,
            "ms_per_coarse_step": round(ms_mr / n_coarse, 4),
            "simulated_time_per_s": rate_mr,
            "lserk4_simulated_time_per_s": rate_rk,
            "speedup_vs_lserk4": round(rate_mr / rate_rk, 4),
            "energy_after": smr.energy(),
        }
        smr.close()
        del smr

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
            "multi_rate": multi,
        },
        "roofline": dict(roof[dominant], type=dominant),
    }
    out["config"]["roofline_by_type"] = roof
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, N, args.cpu_stages)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
