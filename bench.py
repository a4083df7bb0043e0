#!/usr/bin/env python3
"""Throughput of the SLLBM hot path on one MI355X.

Workload (one "step" = one fused stream + collide pass over the whole mesh): the 3D
periodic compressible Taylor-Green vortex at Ma 0.8, Re 400 on 32^3 cells of order
p = 3 with GLL support points (96^3 = 884,736 nodes) and the D3V125 Gauss-Hermite
velocity set; FP64 populations (headline) and FP32 storage side by side.

Prints ONE JSON line.  value = GQUPS = nodes * Q * steps / s (one update = one
(node, velocity) pair with both f and g).  Inputs are resident in HBM before timing.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_UPDATE = {"f64": 32, "f32": 16}   # read + write of f_i and g_i


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ncell", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--kernel", choices=["auto", "gather", "tiled"], default="auto")
    return ap.parse_args()


def traffic_from_profiles(prec):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel build (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        import paper_2412_09051_amd as S
        stamp = os.path.getmtime(S.LIB_PATH)
        e = d.get(prec)
        if not e or e.get("kernel_source_hash") != kernel_source_hash():
            return None
        return e.get("bytes_per_launch")
    except Exception:
        return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_09051_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


KERNEL_NAMES = {0: "k_step_gather", 2: "k_step_tile"}


def gpu_leg(prec, steps, warmup, ncell, kernel="auto"):
    import torch
    import numpy as np
    import paper_2412_09051_amd as S
    import workloads as W
    mesh, phys = W.tgv_case(ncell=ncell)
    m = S.sllbm_mesh_build(mesh)
    vs = S.sllbm_velset_gauss_hermite(3, 5, phys.T0)
    plan = S.sllbm_interp_plan(m, vs, phys.dt, S.SLLBM_F32 if prec == "f32" else S.SLLBM_F64)
    if kernel != "auto":
        S.sllbm_plan_select_kernel(plan, {"gather": 1, "tiled": 2}[kernel])
    kname = KERNEL_NAMES[S.sllbm_plan_info(plan)["kernel"]]
    prm = S.Params.from_physics(phys)
    N, Q = plan.N, plan.Q
    xyz = S.sllbm_mesh_nodes(m)
    rho, u, T = W.tgv_fields(xyz)
    dev = torch.device("cuda")
    dt = torch.float32 if prec == "f32" else torch.float64
    a = torch.empty(2 * Q * N, dtype=dt, device=dev)
    b = torch.empty_like(a)
    S.sllbm_init_equilibrium(plan, prm, torch.tensor(rho, device=dev), torch.tensor(np.ascontiguousarray(u.T), device=dev),
                             torch.tensor(T, device=dev), a)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        S.sllbm_step(plan, prm, a, b, stream)
        a, b = b, a
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t_all0.record(stream)
    for k in range(steps):
        ev[k][0].record(stream)
        S.sllbm_step(plan, prm, a, b, stream)      # one kernel launch per step on `stream`
        ev[k][1].record(stream)
        a, b = b, a
    t_all1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = t_all0.elapsed_time(t_all1)
    per_launch = [s.elapsed_time(e) for s, e in ev]
    avg_launch_ms = sum(per_launch) / len(per_launch)
    tot = S.sllbm_moments(plan, prm, a, totals=True)
    torch.cuda.synchronize()
    ok = all(math.isfinite(x) for x in tot)
    updates = N * Q
    gqups = updates * steps / (total_ms * 1e-3) / 1e9
    alg_bytes = updates * BYTES_PER_UPDATE[prec]
    achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
    return {
        "N": N, "Q": Q, "ms_per_step": total_ms / steps, "wall_s": wall, "gqups": gqups,
        "avg_launch_ms": avg_launch_ms, "achieved_GBs": achieved, "alg_bytes_per_launch": alg_bytes,
        "finite": ok, "mass": float(tot[0]), "kernel": kname,
    }


def cpu_leg(ncell, steps):
    """The oracle, as it stands, on the host cores: one (or more) full step(s) of the
    same workload in FP64."""
    import numpy as np
    import oracle
    import workloads as W
    mesh, phys = W.tgv_case(ncell=ncell)
    o = oracle.TensorOracle(mesh, phys)
    rho, u, T = W.tgv_fields(o.coords())
    pop = o.init(rho, u, T)
    t0 = time.perf_counter()
    for _ in range(steps):
        pop = o.step(pop)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": o.N * o.Q * steps / el / 1e9, "unit": "GQUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full step(s) of the {o.N}-node mesh, FP64, {el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    r64 = gpu_leg("f64", args.steps, args.warmup, args.ncell, args.kernel)
    r32 = None if args.no_fp32 else gpu_leg("f32", args.steps, args.warmup, args.ncell, args.kernel)
    cpu = None if args.no_cpu else cpu_leg(args.ncell, args.cpu_steps)
    traffic = traffic_from_profiles("f64")
    out = {
        "metric": "GQUPS (node x velocity updates/s, f and g together)",
        "value": round(r64["gqups"], 4),
        "unit": "GQUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D periodic compressible Taylor-Green vortex Ma 0.8 Re 400, "
                               f"{args.ncell}^3 cells p=3 GLL ({r64['N']} nodes), D3V125 Gauss-Hermite, FP64",
                   "nodes": r64["N"], "Q": r64["Q"], "order_p": 3, "velocity_set": "D3V125"},
        "roofline": {"bound": "hbm", "achieved": round(r64["achieved_GBs"], 2), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(r64["achieved_GBs"] / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "kernel": r64["kernel"] + "<double,3,3>",
                     "alg_bytes_per_launch": r64["alg_bytes_per_launch"],
                     "avg_launch_ms": round(r64["avg_launch_ms"], 4)},
        "cpu_baseline": cpu,
        "hbm_pct_algorithmic": round(100.0 * r64["gqups"] * 32 / PEAK_HBM_GBS, 2),
    }
    if r32:
        out["fp32"] = {"value": round(r32["gqups"], 4), "unit": "GQUPS", "ms_per_step": round(r32["ms_per_step"], 4),
                       "roofline": {"bound": "hbm", "achieved": round(r32["achieved_GBs"], 2), "peak": PEAK_HBM_GBS,
                                    "unit": "GB/s", "frac": round(r32["achieved_GBs"] / PEAK_HBM_GBS, 4),
                                    "kernel": r32["kernel"] + "<float,3,3>",
                                    "avg_launch_ms": round(r32["avg_launch_ms"], 4)}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
