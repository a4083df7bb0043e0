#!/usr/bin/env python3
"""Throughput of the SLLBM hot path on one MI355X.

Workload (one "step" = one stream + collide pass over the whole mesh): the 3D periodic
compressible Taylor-Green vortex at Ma 0.8, Re 400 on 32^3 cells of order p = 3 with GLL
support points (96^3 = 884,736 nodes) and the reduced degree-9 velocity set D3Q45 the paper
uses (Sec. 3.2); FP64 populations (headline) and FP32 storage side by side, and the same on
the D3V125 Gauss-Hermite product set.  Further workloads (the supersonic NACA 0012 O-grid,
the 2D shear wave at roofline scale, the supersonic channel, the learned correction of the
mixing layer) are reported in objects of their own.

Prints ONE JSON line.  value = GQUPS = nodes * Q * steps / s (one update = one
(node, velocity) pair with both f and g).  Inputs are resident in HBM before timing.  Every
leg times REPS = 5 samples of --steps steps (after --warmup untimed ones) with HIP events and
reports their median.  Per-kernel times come from HIP events the library records around each
of its launches on the timing stream (sllbm_plan_profile).
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# algorithmic bytes per update: read + write of f_i and g_i; the curvilinear plan adds
# its (p+1)^2 weights and a cell id per row (f and g share the row)
BYTES_PER_UPDATE = {"f64": 32, "f32": 16}


def curv_bytes_per_update(prec):
    """f and g read and written, plus the plan row of the (node, velocity) pair: its cell
    and source (one int32) and the departure point's reference coordinates (two values of
    the plan's precision)."""
    return BYTES_PER_UPDATE[prec] + 4 + (8 if prec == "f32" else 16)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="steps per timed sample (median of --reps samples)")
    ap.add_argument("--reps", type=int, default=5, help="timed samples per leg (the median is reported)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ncell", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--precision-steps", type=int, default=1000,
                    help="steps of the side-by-side FP64 / FP32 Taylor-Green comparison (0 = skip)")
    ap.add_argument("--no-ogrid", action="store_true", help="skip the curvilinear O-grid workload")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction (mixing layer) workload")
    ap.add_argument("--learned-steps", type=int, default=None,
                    help="coarse steps of each mixing-layer run (default: to the end of the self-similar window)")
    ap.add_argument("--learned-mach", default="0.7",
                    help="convective Mach numbers of the learned-correction legs, comma separated (first one is 'learned')")
    ap.add_argument("--learned-ncell", type=int, default=16,
                    help="coarse cells per axis of the mixing layer (64: the workload's coarse mesh in the paper's "
                         "160 x 176 x 98 box; smaller: the same cell size in a box scaled with it)")
    ap.add_argument("--learned-ratio", type=int, default=4, help="refinement per axis of the fine mixing layer")
    ap.add_argument("--learned-targets", choices=["injected", "trajectory"], default="injected",
                    help="training targets: one step from the restricted fine state, or along the plain coarse run")
    ap.add_argument("--learned-set", choices=["gh", "cub"], default="gh",
                    help="velocity set of the 'learned' legs (D3V125, or D3Q45 at Pr 0.71 as in the paper)")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned-correction legs (--learned-* options) and print their results as "
                         "one JSON line")
    ap.add_argument("--learned-speed", action="store_true",
                    help="time the plain and the learned coarse step (relaxation and correction in one pass) "
                         "on the 64^3-cell mixing layer, D3V125 at Pr 1 and D3Q45 at Pr 0.71 and 1, and print one "
                         "JSON line")
    ap.add_argument("--no-extra", action="store_true", help="skip the C1-R (2D roofline-scale) and C4 (channel) lines")
    ap.add_argument("--kernel", choices=["auto", "gather", "tiled"], default="auto")
    ap.add_argument("--velocity-set", choices=["d3q45", "d3v125"], default="d3q45",
                    help="velocity set of the headline TGV legs: the reduced degree-9 set D3Q45 the paper "
                         "uses (Sec. 3.2), or the D3V125 product rule (then reported beside it)")
    ap.add_argument("--no-cubature", action="store_true",
                    help="skip the legs on the other TGV velocity set and on the reduced sets D2Q19 / D3Q45 "
                         "of the other workloads")
    ap.add_argument("--make-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: write profiles/traffic.json from the output directories of the two counter "
                         "runs (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE) of this script with --no-cpu --no-learned "
                         "--precision-steps 0 --steps 3 --warmup 1 --reps 1 --copy-calibration")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for byte counters)")
    return ap.parse_args()


def traffic_from_profiles(key):
    """HBM bytes per launch of a workload's dominant kernel (key: tgv_f64, ogrid_f32, ...)
    from the committed rocprofv3 counter summary, if it was taken on the current kernel
    sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(key)
        if not e or e.get("kernel_source_hash") != kernel_source_hash():
            return None
        return e.get("bytes_per_launch")
    except Exception:
        return None


# the sources of the step kernels whose HBM traffic profiles/traffic.json records, and the
# device headers they include
KERNEL_SOURCES = ("sllbm_tile.hip", "sllbm_csr_kernel.hip", "sllbm_kernels.hip", "sllbm_device_common.h",
                  "sllbm_kernels.h")


# the workload lines whose dominant kernel's HBM traffic profiles/traffic.json records, in the
# order `bench.py --no-cpu --no-learned --precision-steps 0` runs them
TRAFFIC_LEGS = ("tgv45_f64", "tgv45_f32", "tgv_f64", "tgv_f32", "ogrid_f32", "ogrid_f64", "ogrid19_f32", "ogrid19_f64",
                "c1r_f64", "c1r_f32", "c4_f32", "c4pr_f32", "c1rq19_f64", "c1rq19_f32", "c4paper_f32")


def make_traffic(fetch_dir, write_dir, out_path=None):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs, FETCH_SIZE then WRITE_SIZE
    (KiB per dispatch), of `bench.py --no-cpu --no-learned --precision-steps 0 --steps 3
    --warmup 1 --reps 1 --copy-calibration`: per workload line (split at each k_init
    dispatch: every line starts with sllbm_init_equilibrium) the mean bytes per launch of its
    dominant streaming kernel, each counter scaled by what it reads for the run's 1 GiB
    device-to-device copy, tagged with the hash of the kernel sources."""
    import csv
    import glob
    import re

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {d}")
        rows = {}
        for r in csv.DictReader(open(f[0])):
            if r["Counter_Name"] != counter:
                continue
            rows.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        return [(k, v[0], v[1]) for k, v in sorted(rows.items())]

    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    if len(fe) != len(wr):
        raise SystemExit(f"the two runs dispatched {len(fe)} and {len(wr)} kernels")
    copy_f = [v for _, n, v in fe if "copyBuffer" in n]
    copy_w = [v for _, n, v in wr if "copyBuffer" in n]
    if not copy_f or not copy_w:
        raise SystemExit("no 1 GiB copy in the runs (--copy-calibration)")
    gib = 1 << 30
    ff, fw = gib / (max(copy_f) * 1024), gib / (max(copy_w) * 1024)
    segs, cur = [], None
    for (_, n, f), (_, _, w) in zip(fe, wr):
        if "k_init" in n:
            cur = []
            segs.append(cur)
        if cur is not None and "copyBuffer" not in n:
            cur.append((n, f, w))
    if len(segs) != len(TRAFFIC_LEGS):
        raise SystemExit(f"{len(segs)} workload lines in the runs, {len(TRAFFIC_LEGS)} expected")
    h = kernel_source_hash()
    res = {"_note": "HBM bytes per launch of each workload's dominant kernel: FETCH_SIZE and WRITE_SIZE (KiB per "
                    "dispatch, rocprofv3 --pmc, one counter per run) scaled by what the same counters read for a 1 GiB "
                    "device copy (fetch factor %.3f, write factor %.3f); kernel_source_hash covers the step kernels' "
                    "sources and device headers (bench.py KERNEL_SOURCES) at the time of the counter runs" % (ff, fw)}
    for key, seg in zip(TRAFFIC_LEGS, segs):
        names = {}
        for n, f, w in seg:
            if re.search(r"k_step_(tile|csr)|k_stream_col", n):
                names.setdefault(n, []).append((f, w))
        n, vals = max(names.items(), key=lambda kv: sum(a for a, b in kv[1]))
        fm = sum(a for a, b in vals) / len(vals) * 1024 * ff
        wm = sum(b for a, b in vals) / len(vals) * 1024 * fw
        short = re.sub(r"\(.*", "", n).replace("void ", "")
        res[key] = {"kernel": short, "bytes_per_launch": int(round(fm)) + int(round(wm)), "read_bytes": int(round(fm)),
                    "write_bytes": int(round(wm)), "kernel_source_hash": h, "dispatches": len(vals)}
        print(key, short, len(vals), round(fm / 1e9, 3), round(wm / 1e9, 3))
    out_path = out_path or os.path.join(ROOT, "profiles", "traffic.json")
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_09051_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


REPS = 5   # timed samples per leg; the reported time is their median


def timed_loop(torch, stream, one, steps, reps=None):
    """reps (default REPS) samples of `steps` calls of one(n), each bracketed by a
    synchronisation and timed with events on `stream`: (median ms, [ms of each sample], wall
    seconds of all samples)."""
    reps = REPS if reps is None else reps
    samples = []
    w0 = time.perf_counter()
    for _ in range(reps):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        for n in range(steps):
            one(n)
        t1.record(stream)
        torch.cuda.synchronize()
        samples.append(t0.elapsed_time(t1))
    return float(np.median(samples)), samples, time.perf_counter() - w0


def timed_steps(S, plan, prm, a, b, steps, warmup, torch):
    """warmup untimed steps, then REPS timed samples of `steps` steps; per-kernel times
    from the plan's event profile over all samples."""
    stream = torch.cuda.current_stream()
    buf = [a, b]

    def one(n):
        S.sllbm_step(plan, prm, buf[0], buf[1], stream)
        buf[0], buf[1] = buf[1], buf[0]

    for n in range(warmup):
        one(n)
    torch.cuda.synchronize()
    S.sllbm_plan_profile(plan, True)
    med, samples, wall = timed_loop(torch, stream, one, steps)
    prof = S.sllbm_plan_profile_read(plan)
    S.sllbm_plan_profile(plan, False)
    return buf[0], med, wall, prof, samples


def gpu_leg(prec, steps, warmup, ncell, kernel="auto", vel="d3v125"):
    import torch
    import numpy as np
    import paper_2412_09051_amd as S
    import workloads as W
    mesh, phys = W.tgv_case(ncell=ncell)
    m = S.sllbm_mesh_build(mesh)
    vs = S.sllbm_velset_cubature(3, phys.T0) if vel == "d3q45" else S.sllbm_velset_gauss_hermite(3, 5, phys.T0)
    plan = S.sllbm_interp_plan(m, vs, phys.dt, S.SLLBM_F32 if prec == "f32" else S.SLLBM_F64)
    if kernel != "auto":
        S.sllbm_plan_select_kernel(plan, {"gather": 1, "tiled": 2}[kernel])
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
    a, total_ms, wall, prof, samples = timed_steps(S, plan, prm, a, b, steps, warmup, torch)
    tot = S.sllbm_moments(plan, prm, a, totals=True)
    torch.cuda.synchronize()
    updates = N * Q
    return summarize(prof, total_ms, wall, steps, updates, BYTES_PER_UPDATE[prec], samples=samples,
                     finite=all(math.isfinite(x) for x in tot), N=N, Q=Q, mass=float(tot[0]))


def precision_leg(ncell, steps=1000, every=100, vel="gh"):
    """The Taylor-Green workload in FP64 and in FP32 storage side by side from the same
    nodal fields: per field (rho, u over all components, T) max_k |q32 - q64| / max_k |q64|
    every `every` steps, and the volume-weighted kinetic energy of each run; vel "cub" on
    the reduced set D3Q45."""
    import torch
    import numpy as np
    import paper_2412_09051_amd as S
    import workloads as W
    mesh, phys = W.tgv_case(ncell=ncell)
    m = S.sllbm_mesh_build(mesh)
    vs = S.sllbm_velset_cubature(3, phys.T0) if vel == "cub" else S.sllbm_velset_gauss_hermite(3, 5, phys.T0)
    prm = S.Params.from_physics(phys)
    xyz = S.sllbm_mesh_nodes(m)
    rho, u, T = W.tgv_fields(xyz)
    V = torch.tensor(S.sllbm_mesh_volumes(m), device="cuda")
    dev = torch.device("cuda")
    runs = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        plan = S.sllbm_interp_plan(m, vs, phys.dt, S.SLLBM_F32 if prec == "f32" else S.SLLBM_F64)
        N, Q = plan.N, plan.Q
        a = torch.empty(2 * Q * N, dtype=dt, device=dev)
        b = torch.empty_like(a)
        S.sllbm_init_equilibrium(plan, prm, torch.tensor(rho, device=dev),
                                 torch.tensor(np.ascontiguousarray(u.T), device=dev), torch.tensor(T, device=dev), a)
        runs[prec] = [plan, a, b]
    hist = {"step": [], "rho": [], "u": [], "T": [], "ke_f64": [], "ke_f32": []}
    fields = {}

    def moments(plan, pop):
        N = plan.N
        r = torch.empty(N, dtype=torch.float64, device=dev)
        uu = torch.empty(3 * N, dtype=torch.float64, device=dev)
        t = torch.empty(N, dtype=torch.float64, device=dev)
        S.sllbm_moments(plan, prm, pop, r, uu, t)
        return r, uu.view(3, N), t

    for n in range(steps + 1):
        if n % every == 0:
            for prec in ("f64", "f32"):
                fields[prec] = moments(runs[prec][0], runs[prec][1])
            r64, u64, t64 = fields["f64"]
            r32, u32, t32 = fields["f32"]
            hist["step"].append(n)
            hist["rho"].append(float((r32 - r64).abs().max() / r64.abs().max()))
            hist["u"].append(float((u32 - u64).abs().max() / u64.abs().max()))
            hist["T"].append(float((t32 - t64).abs().max() / t64.abs().max()))
            for prec in ("f64", "f32"):
                r, uu, _ = fields[prec]
                hist["ke_" + prec].append(float((0.5 * r * (uu * uu).sum(0) * V).sum() / V.sum()))
        if n == steps:
            break
        for prec in ("f64", "f32"):
            plan, a, b = runs[prec]
            S.sllbm_step(plan, prm, a, b)
            runs[prec][1], runs[prec][2] = b, a
    torch.cuda.synchronize()
    del runs
    torch.cuda.empty_cache()
    return {"workload": f"3D Taylor-Green vortex {ncell}^3 cells p=3, {'D3Q45' if vel == 'cub' else 'D3V125'}, "
                        f"FP32 storage against FP64, same initial fields",
            "steps": steps, "max_rel_diff_at_end": {k: round(hist[k][-1], 9) for k in ("rho", "u", "T")},
            "history": {k: [round(x, 10) for x in v] for k, v in hist.items()}}


def tensor_case_leg(case, prec, steps, warmup, Pr=1.0, vel="gh"):
    """Another tensor-product workload: C1-R (2D shear wave at roofline scale) or C4 (the
    supersonic channel, with the mass rescaling every 10 steps), at Prandtl number Pr, on the
    product rule (vel "gh") or the reduced set ("cub": the time step keeps CFL 0.9 on the
    set's largest component)."""
    import dataclasses
    import torch
    import paper_2412_09051_amd as S
    import workloads as W
    if case == "c1r":
        mesh, phys = W.shear_wave_case(ncell=1024, p=4)
        fields = W.shear_wave_fields
        fix_every = 0
    else:
        mesh, phys = W.channel_case()
        fields = W.channel_fields
        fix_every = 10
    if vel == "cub":
        vs = S.sllbm_velset_cubature(mesh.dim, phys.T0)
        phys = dataclasses.replace(phys, dt=phys.dt * W.ZETA_MAX_GH5 / float(np.max(np.abs(vs["zeta"]))))
    else:
        vs = S.sllbm_velset_gauss_hermite(mesh.dim, 5, phys.T0)
    m = S.sllbm_mesh_build(mesh)
    plan = S.sllbm_interp_plan(m, vs, phys.dt, S.SLLBM_F32 if prec == "f32" else S.SLLBM_F64)
    prm = S.Params.from_physics(phys, Pr=Pr)
    N, Q = plan.N, plan.Q
    rho, u, T = fields(S.sllbm_mesh_nodes(m))
    dt = torch.float32 if prec == "f32" else torch.float64
    a = torch.empty(2 * Q * N, dtype=dt, device="cuda")
    b = torch.empty_like(a)
    S.sllbm_init_equilibrium(plan, prm, torch.tensor(rho, device="cuda"), torch.tensor(np.ascontiguousarray(u.T), device="cuda"),
                             torch.tensor(T, device="cuda"), a)
    mref = float(S.sllbm_moments(plan, prm, a, totals=True)[0]) if fix_every else 0.0
    stream = torch.cuda.current_stream()
    ctl = None
    if case == "c4":
        # the force starts at F_x = rho_w Re_tau^2 mu_w^2 / delta_c^3 and is then held by
        # the device-side PI controller, updated with the mass rescaling
        ctl = W.channel_controller()
        S.sllbm_force_reset(plan, phys.force, stream)
        prm = dataclasses.replace(prm, force_device=1)
    fixp = dataclasses.replace(prm, mass_fix=1, mass_ref=mref)

    buf = [a, b]

    def one(n):
        a, b = buf
        if fix_every and n % fix_every == 0:
            if ctl:
                S.sllbm_force_update(plan, a, dt=fix_every * phys.dt, stream=stream, **ctl)
            S.sllbm_step(plan, fixp, a, b, stream)
        else:
            S.sllbm_step(plan, prm, a, b, stream)
        buf[0], buf[1] = b, a

    for n in range(warmup):
        one(n)
    torch.cuda.synchronize()
    S.sllbm_plan_profile(plan, True)
    med, samples, _ = timed_loop(torch, stream, one, steps)
    a, b = buf
    prof = S.sllbm_plan_profile_read(plan)
    S.sllbm_plan_profile(plan, False)
    try:
        tot = S.sllbm_moments(plan, prm, a, totals=True)
    except S.SllbmError:              # non-finite or non-physical nodes (EUNSTABLE)
        tot = [float("nan")]
    extra = {}
    if ctl:
        st = S.sllbm_force_read(plan, stream)
        extra["force_control"] = {"force_x": float(st["force"][0]), "force_x0": float(phys.force[0]),
                                  "mean_momentum": float(st["mean_momentum"]), "target": ctl["target"],
                                  "updates": st["updates"]}
    r = summarize(prof, med, 0.0, steps, N * Q, BYTES_PER_UPDATE[prec], samples=samples,
                  finite=all(math.isfinite(x) for x in tot), N=N, Q=Q, **extra)
    del a, b
    torch.cuda.empty_cache()
    return r


def summarize(prof, total_ms, wall, steps, updates, bytes_per_update, samples=None, **extra):
    """total_ms: the (median) time of `steps` steps; samples: the ms of every timed sample."""
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    name, (kms, launches) = dom
    avg_ms = kms / max(launches, 1)
    alg = updates * bytes_per_update
    out = {
        "ms_per_step": total_ms / steps, "wall_s": wall,
        "median_of": len(samples) if samples else 1,
        "samples_ms_per_step": [round(x / steps, 5) for x in samples] if samples else None,
        "gqups": updates * steps / (total_ms * 1e-3) / 1e9,
        "kernels": {k: {"avg_ms": round(v[0] / max(v[1], 1), 4), "launches": v[1]} for k, v in prof.items()},
        "dominant": name, "avg_launch_ms": avg_ms, "alg_bytes_per_launch": alg,
        "achieved_GBs": alg / (avg_ms * 1e-3) / 1e9,
        "step_GBs": alg * steps / (total_ms * 1e-3) / 1e9,
    }
    out.update(extra)
    return out


def ogrid_leg(prec, steps, warmup, vel="d2v25"):
    import torch
    import paper_2412_09051_amd as S
    import workloads as W
    mesh, phys = W.naca_ogrid()
    m = S.sllbm_mesh_build(mesh)
    vs = S.sllbm_velset_cubature(2, phys.T0) if vel == "d2q19" else S.sllbm_velset_gauss_hermite(2, 5, phys.T0)
    t0 = time.perf_counter()
    plan = S.sllbm_interp_plan(m, vs, phys.dt, S.SLLBM_F32 if prec == "f32" else S.SLLBM_F64)
    plan_s = time.perf_counter() - t0
    prm = S.Params.from_physics(phys)
    N, Q = plan.N, plan.Q
    rho, u, T = W.naca_fields(S.sllbm_mesh_nodes(m))
    dev = torch.device("cuda")
    dt = torch.float32 if prec == "f32" else torch.float64
    a = torch.empty(2 * Q * N, dtype=dt, device=dev)
    b = torch.empty_like(a)
    S.sllbm_init_equilibrium(plan, prm, torch.tensor(rho, device=dev), torch.tensor(u.T.copy(), device=dev),
                             torch.tensor(T, device=dev), a)
    a, total_ms, wall, prof, samples = timed_steps(S, plan, prm, a, b, steps, warmup, torch)
    tot = S.sllbm_moments(plan, prm, a, totals=True)
    torch.cuda.synchronize()
    return summarize(prof, total_ms, wall, steps, N * Q, curv_bytes_per_update(prec), samples=samples,
                     finite=all(math.isfinite(x) for x in tot), N=N, Q=Q, plan_build_s=plan_s,
                     bpu=curv_bytes_per_update(prec))


MIX_BOX_CELLS = (2.5, 2.75, 1.5)      # coarse cell size per axis in initial momentum thicknesses


def mixing_dtheta(S, torch, plan, prm, pop, shape, du, V, box):
    """Momentum thickness of a population field (Sec. 4.4): the moments on the device, the
    plane averages and the y integral by the package's diagnostic."""
    from paper_2412_09051_amd import diagnostics as D
    N = plan.N
    rho = torch.empty(N, dtype=torch.float64, device="cuda")
    u = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    S.sllbm_moments(plan, prm, pop, rho, u, None)
    Nx, Ny, Nz = shape
    return D.momentum_thickness(rho.view(Nz, Ny, Nx), u[:N].view(Nz, Ny, Nx), V, du, box[0] * box[2])


def learned_leg(ncell=16, ratio=4, steps=None, n_train=8, train_iters=1500, Ma_c=0.7, alphas=(0.0, 0.25, 0.5, 1.0),
                targets="injected", vel="gh", Pr=1.0, train_seeds=(6, 7), eval_seed=5):
    return _learned_leg(ncell, ratio, steps, n_train, train_iters, Ma_c, alphas, targets, vel, Pr, train_seeds,
                        eval_seed)


def _learned_leg(ncell, ratio, steps, n_train, train_iters, Ma_c, alphas, targets, vel, Pr, train_seeds, eval_seed):
    """C5: temporal mixing layer on a coarse mesh, plain and with the learned correction,
    against the `ratio`x finer mesh; FP32 populations.  The network is trained by the
    library's kernels on restricted one-step samples (n_train per run) of fine runs with the
    perturbation seeds train_seeds; a gain alpha on its output (0 = the plain method) is
    chosen on the first training run's momentum-thickness history; everything is then
    evaluated on a run it never saw (eval_seed): momentum-thickness history and time per
    coarse step.  targets="injected": a sample starts the plain coarse step
    from the restricted fine state; "trajectory": from the plain coarse run started at the
    restricted initial state, so that the features come from coarse-evolved states as in
    use and the target includes the drift accumulated so far.  vel "cub" runs the reduced set
    D3Q45 (at the same time step) and Pr the Prandtl number (the paper's mixing layer: D3Q45,
    Pr 0.71).  steps = None runs to the end of the self-similar window; the growth rate of
    the momentum thickness is fitted inside the window (else over the run's second half)."""
    import dataclasses
    import torch
    import paper_2412_09051_amd as S
    import workloads as W
    d0 = W.MIX_DTHETA0
    # 64 coarse cells per axis: the paper's box (Sec. 4.4, 160 x 176 x 98 initial momentum
    # thicknesses); fewer: the same coarse cell in a box scaled with the cell count
    box = tuple(x * d0 for x in (160, 176, 98)) if ncell == 64 else tuple(ncell * c * d0 for c in MIX_BOX_CELLS)
    mesh, phys = W.mixing_layer_case(ncell=(ncell,) * 3, box=box, Ma_c=Ma_c)
    fmesh, fphys = W.mixing_layer_case(ncell=(ncell,) * 3, refine=ratio, box=box, Ma_c=Ma_c)
    phys, fphys = dataclasses.replace(phys, Pr=Pr), dataclasses.replace(fphys, Pr=Pr)
    vname = "D3Q45" if vel == "cub" else "D3V125"
    du = 2.0 * Ma_c * math.sqrt(1.4)
    tau_step = phys.dt * du / d0                      # tau per coarse step
    from paper_2412_09051_amd.diagnostics import MIX_WINDOW
    window = MIX_WINDOW.get(round(Ma_c, 2))
    if steps is None:
        steps = int(math.ceil(window[1] / tau_step)) if window else 1000
    mats = {}
    for name, (me, ph) in (("c", (mesh, phys)), ("f", (fmesh, fphys))):
        mm = S.sllbm_mesh_build(me)
        vs = S.sllbm_velset_cubature(3, ph.T0) if vel == "cub" else S.sllbm_velset_gauss_hermite(3, 5, ph.T0)
        pl = S.sllbm_interp_plan(mm, vs, ph.dt, S.SLLBM_F32)
        shape = tuple(me.ncell[a] * me.p + (0 if me.face_bc[a][0] < 0 else 1) for a in range(3))
        V = torch.tensor(S.sllbm_mesh_volumes(mm), device="cuda").view(shape[2], shape[1], shape[0])
        mats[name] = (mm, pl, S.Params.from_physics(ph), shape, V)
    cm, cplan, cprm, cshape, cV = mats["c"]
    fm, fplan, fprm, fshape, fV = mats["f"]
    Q, Nc, Nf = cplan.Q, cplan.N, fplan.N
    nf = S.n_features(3)
    every_h = 25

    def fine_init(seed):
        rho, u, T = W.mixing_layer_fields(S.sllbm_mesh_nodes(fm), box=box, amp=0.1, seed=seed, Ma_c=Ma_c)
        a = torch.empty(2 * Q * Nf, dtype=torch.float32, device="cuda")
        S.sllbm_init_equilibrium(fplan, fprm, torch.tensor(rho, device="cuda"), torch.tensor(u.T.copy(), device="cuda"),
                                 torch.tensor(T, device="cuda"), a)
        return a, torch.empty_like(a)

    def restrict(fa):
        c = torch.empty(2 * Q * Nc, dtype=torch.float32, device="cuda")
        S.sllbm_restrict(fplan, cplan, ratio, fa, c)
        return c

    def dth(which, pop):
        plan, prm, shape, V = (fplan, fprm, fshape, fV) if which == "f" else (cplan, cprm, cshape, cV)
        return mixing_dtheta(S, torch, plan, prm, pop, shape, du, V, box)

    def coarse_rollout(c0, net=None, timed=False):
        a, b = c0.clone(), torch.empty_like(c0)
        hist, ms = [], 0.0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for n in range(steps + 1):
            if n % every_h == 0:
                hist.append(dth("c", a))
            if n == steps:
                break
            e0.record()
            if net is not None:
                S.sllbm_step_learned(cplan, cprm, net, a, b)
            else:
                S.sllbm_step(cplan, cprm, a, b)
            e1.record()
            a, b = b, a
            if timed:
                torch.cuda.synchronize()
                ms += e0.elapsed_time(e1)
        return hist, ms

    def fine_history(seed, samples=False, timed=False):
        fa, fb = fine_init(seed)
        c_init = restrict(fa)
        cc = c_init.clone()
        hist, X, T, ms = [], [], [], 0.0
        every = max(1, steps // n_train)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        for n in range(steps + 1):
            if n % every_h == 0:
                hist.append(dth("f", fa))
            if n % 250 == 0 and n and time.perf_counter() - w0 > 30:
                print(f"# learned Ma_c {Ma_c}: fine run seed {seed} at coarse step {n} of {steps}", file=sys.stderr,
                      flush=True)
                w0 = time.perf_counter()
            if n == steps:
                break
            take = samples and n % every == 0 and len(X) < n_train
            if samples and targets == "trajectory":
                plain = torch.empty(2 * Q * Nc, dtype=torch.float32, device="cuda")
                S.sllbm_step(cplan, cprm, cc, plain)
                cc = plain
            elif take:
                plain = torch.empty(2 * Q * Nc, dtype=torch.float32, device="cuda")
                S.sllbm_step(cplan, cprm, restrict(fa), plain)
            e0.record()
            for _ in range(ratio):
                S.sllbm_step(fplan, fprm, fa, fb)
                fa, fb = fb, fa
            e1.record()
            if timed:
                torch.cuda.synchronize()
                ms += e0.elapsed_time(e1)
            if take:
                truth = restrict(fa)
                x = torch.empty(Nc, nf, dtype=torch.bfloat16, device="cuda")
                S.sllbm_features(cplan, cprm, plain, x)
                t = torch.empty(Nc, 2 * Q, dtype=torch.float32, device="cuda")
                S.sllbm_learned_targets(cplan, plain, truth, t)
                X.append(x)
                T.append(t)
        return c_init, hist, X, T, ms

    def growth_err(h, ref):
        g = [v - h[0] for v in h]
        gr = [v - ref[0] for v in ref]
        return max(abs(a - b) / abs(b) for a, b in zip(g[1:], gr[1:]))

    tau_h = tau_step * every_h * np.arange(steps // every_h + 1)      # tau of each history sample
    in_window = (tau_h >= window[0]) & (tau_h <= window[1]) if window else np.zeros(len(tau_h), bool)
    if in_window.sum() < 3:
        in_window = np.arange(len(tau_h)) >= len(tau_h) // 2

    def late_rate(h):
        """Growth rate d(dtheta)/d(tau) of the momentum thickness in the self-similar window
        (least squares over the samples inside it)."""
        return float(np.polyfit(tau_h[in_window], np.asarray(h)[in_window], 1)[0])

    def rate_err(h, ref):
        return abs(late_rate(h) - late_rate(ref)) / abs(late_rate(ref))

    # ---- training on the runs of train_seeds
    t0 = time.perf_counter()
    X, T = [], []
    for i, sd in enumerate(train_seeds):
        c_s, f_s, Xs, Ts, _ = fine_history(sd, samples=True)
        X += Xs
        T += Ts
        if i == 0:
            c_sel, f_sel = c_s, f_s          # the gain is selected on the first training run
    X, T = torch.cat(X), torch.cat(T)
    net = S.sllbm_mlp_create(nf, 2 * Q, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    losses = []
    for it in range(train_iters):
        idx = torch.randint(0, X.shape[0], (4096,), device="cuda", generator=gen)
        want = it in (0, train_iters - 1)
        l_ = S.sllbm_mlp_train_step(net, X[idx].contiguous(), T[idx].contiguous(),
                                    2e-3 if it < (2 * train_iters) // 3 else 5e-4, want_loss=want)
        if want:
            losses.append(l_)
    del X, T
    print(f"# learned Ma_c {Ma_c} {vname}: fine run and training done ({steps} coarse steps, loss {losses})",
          file=sys.stderr, flush=True)
    # ---- output gain chosen on the training run's momentum thickness
    theta = S.sllbm_mlp_get_params(net)
    o4 = nf * 64 + 64 + 2 * (64 * 64 + 64)           # W4, b4 follow
    sel, sel_growth = {}, {}
    for a in alphas:
        th = theta.copy()
        th[o4:] *= a
        S.sllbm_mlp_set_params(net, th)
        h, _ = coarse_rollout(c_sel, None if a == 0.0 else net)
        sel[a] = rate_err(h, f_sel)
        sel_growth[a] = growth_err(h, f_sel)
    alpha = min(sel, key=lambda a: sel[a] if math.isfinite(sel[a]) else math.inf)
    print(f"# learned Ma_c {Ma_c} {vname}: gain {alpha} selected ({sel})", file=sys.stderr, flush=True)
    # at gain 0 every weight is zeroed, so that the correction is exactly 0 even where training
    # diverged (0 x NaN), while the learned run still does the network's work
    th = theta.copy() if alpha else np.zeros_like(theta)
    th[o4:] *= alpha
    S.sllbm_mlp_set_params(net, th)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    # ---- evaluation on eval_seed
    c_ev, f_ev, _, _, t_f = fine_history(eval_seed, timed=True)
    hp, t_p = coarse_rollout(c_ev, None, timed=True)
    hl, t_l = coarse_rollout(c_ev, net, timed=True)
    hist = {"fine": f_ev, "plain": hp, "learned": hl}
    return {
        "workload": f"3D temporal mixing layer Ma_c {Ma_c}, coarse {ncell}^3 cells p=2 ({Nc} nodes) vs "
                    f"{ratio}x finer ({Nf} nodes), {vname}, Pr {Pr}, FP32; trained on seeds "
                    f"{', '.join(map(str, train_seeds))}, evaluated on seed {eval_seed}",
        "box_dtheta0": [round(b / d0, 3) for b in box],
        "coarse_kernel": {0: "gather", 2: "tiled (relaxation and correction in one pass)"}.get(
            S.sllbm_plan_info(cplan)["kernel"], "other"),
        "steps": steps, "targets": targets, "train_samples": n_train, "train_iters": train_iters, "train_loss": losses,
        "train_finite": bool(np.isfinite(theta).all()),
        "train_s": round(train_s, 2),
        "alpha_selection_window_rate_err": {str(k): round(v, 4) for k, v in sel.items()},
        "alpha_selection_growth_err": {str(k): round(v, 4) for k, v in sel_growth.items()},
        "alpha": alpha,
        "ms_per_coarse_step": {"fine": round(t_f / steps, 4), "plain": round(t_p / steps, 4),
                               "learned": round(t_l / steps, 4)},
        "time_to_solution_ratio": {"fine_vs_learned": round(t_f / t_l, 2), "fine_vs_plain": round(t_f / t_p, 2)},
        "dtheta": {k: [round(v, 6) for v in h] for k, h in hist.items()},
        "dtheta_growth_max_rel_err": {"plain": round(growth_err(hp, f_ev), 4), "learned": round(growth_err(hl, f_ev), 4)},
        "tau_per_step": round(tau_step, 5),
        "self_similar_window_tau": list(window) if window else None,
        "window_samples": int(in_window.sum()),
        "dtheta_rate_in_window": {"fine": late_rate(f_ev), "plain": late_rate(hp), "learned": late_rate(hl),
                                  "plain_rel_err": round(rate_err(hp, f_ev), 4),
                                  "learned_rel_err": round(rate_err(hl, f_ev), 4)},
        "dtheta_final_rel_err": {"plain": round(abs(hp[-1] - f_ev[-1]) / f_ev[-1], 4),
                                 "learned": round(abs(hl[-1] - f_ev[-1]) / f_ev[-1], 4)},
        # the workload's bar: growth rate in the self-similar window within 5 % of the fine run
        # at >= 8x lower time to solution
        "meets_5pct_at_8x": {"plain": bool(rate_err(hp, f_ev) <= 0.05 and t_f / t_p >= 8.0),
                             "learned": bool(rate_err(hl, f_ev) <= 0.05 and t_f / t_l >= 8.0)},
        "finite": {k: all(math.isfinite(v) for v in h) for k, h in hist.items()},
    }


def learned_speed_leg(vel, Pr, steps=20, ncell=64, Ma_c=0.7):
    """Cost of the learned correction at the mixing layer's coarse size (ncell^3 cells, p = 2,
    FP32, the paper's 160 x 176 x 98 initial momentum thicknesses at 64 cells): the plain step
    against one learned step (relaxation and correction in one pass), median of REPS samples,
    with the library's per-kernel event times.  The network is freshly initialised: its
    weights do not change the work."""
    import dataclasses
    import torch
    import paper_2412_09051_amd as S
    import workloads as W
    d0 = W.MIX_DTHETA0
    box = tuple(x * d0 for x in (160, 176, 98)) if ncell == 64 else tuple(ncell * c * d0 for c in MIX_BOX_CELLS)
    mesh, phys = W.mixing_layer_case(ncell=(ncell,) * 3, box=box, Ma_c=Ma_c)
    phys = dataclasses.replace(phys, Pr=Pr)
    m = S.sllbm_mesh_build(mesh)
    vs = S.sllbm_velset_cubature(3, phys.T0) if vel == "d3q45" else S.sllbm_velset_gauss_hermite(3, 5, phys.T0)
    plan = S.sllbm_interp_plan(m, vs, phys.dt, S.SLLBM_F32)
    prm = S.Params.from_physics(phys)
    rho, u, T = W.mixing_layer_fields(S.sllbm_mesh_nodes(m), Ma_c=Ma_c, box=box)
    a = torch.empty(2 * plan.Q * plan.N, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    S.sllbm_init_equilibrium(plan, prm, torch.tensor(rho, device="cuda"),
                             torch.tensor(np.ascontiguousarray(u.T), device="cuda"), torch.tensor(T, device="cuda"), a)
    net = S.sllbm_mlp_create(S.n_features(3), 2 * plan.Q, seed=1)
    stream = torch.cuda.current_stream()
    buf = [a, b]
    out = {"workload": f"mixing layer coarse {ncell}^3 cells p=2 ({plan.N} nodes), {vel.upper()}, Pr {Pr}, FP32",
           "kernel": S.sllbm_plan_info(plan)["kernel"]}
    for mode in ("plain", "learned"):
        def one(n):
            if mode == "plain":
                S.sllbm_step(plan, prm, buf[0], buf[1], stream)
            else:
                S.sllbm_step_learned(plan, prm, net, buf[0], buf[1], stream)
            buf[0], buf[1] = buf[1], buf[0]
        for n in range(3):
            one(n)
        torch.cuda.synchronize()
        S.sllbm_plan_profile(plan, True)
        med, samples, _ = timed_loop(torch, stream, one, steps)
        prof = S.sllbm_plan_profile_read(plan)
        S.sllbm_plan_profile(plan, False)
        out[mode] = {"ms_per_step": round(med / steps, 4), "samples_ms": [round(x, 3) for x in samples],
                     "kernels_ms": {k: round(v[0] / v[1], 4) for k, v in prof.items()}}
    out["learned_over_plain"] = round(out["learned"]["ms_per_step"] / out["plain"]["ms_per_step"], 3)
    out["finite"] = all(math.isfinite(x) for x in S.sllbm_moments(plan, prm, buf[0], totals=True))
    return out


def copy_calibration():
    """A plain device copy of 1 GiB, three times: the reference for the FETCH_SIZE and
    WRITE_SIZE counters of the profiled runs."""
    import torch
    n = 1 << 27                       # 2^27 doubles = 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"bytes_read": 8 * n, "bytes_written": 8 * n, "launches": 3}


def copy_ceiling(reps=10):
    """The practical HBM ceiling: a plain 1 GiB device-to-device copy, timed with events
    (bytes read + bytes written per second)."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(2 * 8 * n / (ms * 1e-3) / 1e9, 1), "bytes": 2 * 8 * n, "ms": round(ms, 4)}


def cpu_leg(ncell, steps):
    """The oracle, as it stands, on the host cores: one (or more) full step(s) of the
    same workload in FP64."""
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
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    lscpu = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Vendor ID", "CPU family", "Model", "Stepping", "CPU(s)", "Socket(s)",
                             "Core(s) per socket", "Thread(s) per core", "CPU max MHz", "L3 cache",
                             "Hypervisor vendor"):
                lscpu[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    # one thread: the oracle's step at a seeded sample of nodes, in a child process started
    # with OMP_NUM_THREADS=1 (it imports the oracle and numpy only)
    code = ("import time, numpy as np, oracle, workloads as W\n"
            f"mesh, phys = W.tgv_case(ncell={ncell})\n"
            "o = oracle.TensorOracle(mesh, phys)\n"
            "rho, u, T = W.tgv_fields(o.coords())\n"
            "pop = o.init(rho, u, T)\n"
            "nodes = np.sort(np.random.Generator(np.random.PCG64(3)).choice(o.N, 8192, replace=False)).astype(np.int64)\n"
            "t0 = time.perf_counter()\n"
            "o.step_nodes(pop, nodes)\n"
            "el = time.perf_counter() - t0\n"
            "print(len(nodes) * o.Q / el / 1e9, el)\n")
    one = None
    try:
        r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, OMP_NUM_THREADS="1"), cwd=ROOT,
                           capture_output=True, text=True, timeout=900)
        v, t1 = (float(x) for x in r.stdout.split()[-2:])
        one = {"value": v, "unit": "GQUPS", "cores": 1, "sample": f"the step at 8192 seeded nodes, FP64, {t1:.1f} s"}
    except (subprocess.SubprocessError, ValueError):
        one = None
    return {"value": o.N * o.Q * steps / el / 1e9, "unit": "GQUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full step(s) of the {o.N}-node mesh, FP64, {el:.1f} s", "cpu_model": model,
            "lscpu": lscpu,
            "one_thread": one}


def roofline(r, traffic=None):
    return {"bound": "hbm", "achieved": round(r["achieved_GBs"], 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(r["achieved_GBs"] / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": r["dominant"], "avg_launch_ms": round(r["avg_launch_ms"], 4),
            "alg_bytes_per_launch": r["alg_bytes_per_launch"],
            "step_achieved": round(r["step_GBs"], 2), "step_frac": round(r["step_GBs"] / PEAK_HBM_GBS, 4)}


def main():
    global REPS
    args = parse()
    REPS = max(1, args.reps)
    if args.make_traffic:
        make_traffic(*args.make_traffic)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.learned_speed:
        res = []
        for vel, Pr in (("d3v125", 1.0), ("d3q45", 1.0), ("d3q45", 0.71)):
            res.append(learned_speed_leg(vel, Pr))
            print(f"# learned speed {vel} Pr {Pr}: {res[-1]['learned_over_plain']}", file=sys.stderr, flush=True)
        print(json.dumps({"learned_speed": res}))
        return
    if args.learned_only:
        lset = dict(vel="cub", Pr=0.71) if args.learned_set == "cub" else {}
        res = []
        for mc in (float(x) for x in args.learned_mach.split(",")):
            res.append(learned_leg(ncell=args.learned_ncell, ratio=args.learned_ratio, Ma_c=mc,
                                   steps=args.learned_steps, targets=args.learned_targets, **lset))
            print(f"# learned Ma_c {mc} done: time-to-solution ratio {res[-1]['time_to_solution_ratio']}",
                  file=sys.stderr, flush=True)
        print(json.dumps({"learned": res}))
        return
    vset = args.velocity_set
    tkey = "tgv45" if vset == "d3q45" else "tgv"
    r64 = gpu_leg("f64", args.steps, args.warmup, args.ncell, args.kernel, vset)
    print(f"# tgv {vset} f64 done: {r64['gqups']:.2f} GQUPS", file=sys.stderr, flush=True)
    r32 = None if args.no_fp32 else gpu_leg("f32", args.steps, args.warmup, args.ncell, args.kernel, vset)
    other = "d3v125" if vset == "d3q45" else "d3q45"
    cub = {}
    if not args.no_cubature:
        for prec in ("f64", "f32"):
            cub[prec] = gpu_leg(prec, args.steps, args.warmup, args.ncell, args.kernel, other)
            print(f"# tgv {other} {prec} done: {cub[prec]['gqups']:.2f} GQUPS", file=sys.stderr, flush=True)
    og = {}
    if not args.no_ogrid:
        for prec in ("f32", "f64"):
            og[prec] = ogrid_leg(prec, args.steps, args.warmup)
            print(f"# ogrid {prec} done: {og[prec]['gqups']:.2f} GQUPS", file=sys.stderr, flush=True)
        if not args.no_cubature:
            for prec in ("f32", "f64"):
                og["d2q19_" + prec] = ogrid_leg(prec, args.steps, args.warmup, "d2q19")
                print(f"# ogrid d2q19 {prec} done: {og['d2q19_' + prec]['gqups']:.2f} GQUPS", file=sys.stderr,
                      flush=True)
    extra = {}
    if not args.no_extra:
        # (case, precisions, Prandtl number, velocity set); the paper's channel set-up (D3Q45,
        # Pr 0.7) belongs to the reduced-set legs
        cases = [("c1r", ("f64", "f32"), 1.0, "gh"), ("c4", ("f32",), 1.0, "gh"), ("c4pr", ("f32",), 0.7, "gh")]
        if not args.no_cubature:
            cases += [("c1rq19", ("f64", "f32"), 1.0, "cub"), ("c4paper", ("f32",), 0.7, "cub")]
        for case, precs, Pr, vel in cases:
            for prec in precs:
                extra[f"{case}_{prec}"] = tensor_case_leg("c1r" if case.startswith("c1r") else "c4", prec,
                                                          max(10, args.steps // 5), 3, Pr=Pr, vel=vel)
                print(f"# {case} {prec} done: {extra[f'{case}_{prec}']['gqups']:.2f} GQUPS", file=sys.stderr, flush=True)
    prec_cmp = prec_cmp_other = None
    if not args.no_fp32 and args.precision_steps > 0:
        prec_cmp = precision_leg(args.ncell, args.precision_steps, vel="cub" if vset == "d3q45" else "gh")
        print(f"# FP32 vs FP64 on {vset} after {args.precision_steps} steps: {prec_cmp['max_rel_diff_at_end']}",
              file=sys.stderr, flush=True)
        if not args.no_cubature:
            prec_cmp_other = precision_leg(args.ncell, args.precision_steps, vel="cub" if other == "d3q45" else "gh")
            print(f"# FP32 vs FP64 on {other} after {args.precision_steps} steps: "
                  f"{prec_cmp_other['max_rel_diff_at_end']}", file=sys.stderr, flush=True)
    lrn = None
    lrn_more = {}
    if not args.no_learned:
        machs = [float(x) for x in args.learned_mach.split(",")]
        lset = dict(vel="cub", Pr=0.71) if args.learned_set == "cub" else {}
        for i, mc in enumerate(machs):
            r = learned_leg(ncell=args.learned_ncell, ratio=args.learned_ratio, Ma_c=mc, steps=args.learned_steps,
                            targets=args.learned_targets, **lset)
            print(f"# learned Ma_c {mc} done: time-to-solution ratio {r['time_to_solution_ratio']}", file=sys.stderr,
                  flush=True)
            if i == 0:
                lrn = r
            else:
                lrn_more[str(mc)] = r
    lrn_paper = None
    if not args.no_learned and not args.no_cubature and args.learned_set == "gh":
        lrn_paper = learned_leg(ncell=args.learned_ncell, ratio=args.learned_ratio, Ma_c=0.7, vel="cub", Pr=0.71,
                                steps=args.learned_steps, targets=args.learned_targets)
        print(f"# learned, the paper's mixing-layer set-up (D3Q45, Pr 0.71) done: time-to-solution ratio "
              f"{lrn_paper['time_to_solution_ratio']}", file=sys.stderr, flush=True)
    cal = copy_calibration() if args.copy_calibration else None
    ceil = copy_ceiling()
    print(f"# device copy: {ceil['GBs']} GB/s", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_leg(args.ncell, args.cpu_steps)
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
                               f"{args.ncell}^3 cells p=3 GLL ({r64['N']} nodes), "
                               f"{'D3Q45 reduced cubature' if vset == 'd3q45' else 'D3V125 Gauss-Hermite'}, FP64",
                   "nodes": r64["N"], "Q": r64["Q"], "order_p": 3, "velocity_set": vset.upper()},
        "roofline": roofline(r64, traffic_from_profiles(tkey + "_f64")),
        "cpu_baseline": cpu,
        "kernels": r64["kernels"],
        "median_of": r64["median_of"],
        "samples_ms_per_step": r64["samples_ms_per_step"],
    }
    if r32:
        out["fp32"] = {"value": round(r32["gqups"], 4), "unit": "GQUPS", "ms_per_step": round(r32["ms_per_step"], 4),
                       "median_of": r32["median_of"], "samples_ms_per_step": r32["samples_ms_per_step"],
                       "roofline": roofline(r32, traffic_from_profiles(tkey + "_f32")), "kernels": r32["kernels"]}
    if cub:
        # the same workload and time step on the other velocity set (Q = 125 or 45): the
        # per-update rate is comparable, the per-step time is not
        okey = "tgv45" if other == "d3q45" else "tgv"
        out[other] = {
            "workload": f"the same Taylor-Green vortex ({cub['f64']['N']} nodes, same time step) on the "
                        + ("reduced degree-9 velocity set D3Q45" if other == "d3q45" else
                           "D3V125 Gauss-Hermite product set"),
            **{prec: {"value": round(v["gqups"], 4), "unit": "GQUPS", "ms_per_step": round(v["ms_per_step"], 4),
                      "median_of": v["median_of"], "samples_ms_per_step": v["samples_ms_per_step"],
                      "node_updates_per_s": round(v["N"] / (v["ms_per_step"] * 1e-3), 1),
                      f"step_time_vs_{vset}": round(v["ms_per_step"] / (r64 if prec == "f64" else r32)["ms_per_step"], 4)
                      if (prec == "f64" or r32) else None,
                      "roofline": roofline(v, traffic_from_profiles(okey + "_" + prec)), "kernels": v["kernels"],
                      "finite": v["finite"]}
               for prec, v in cub.items()}}
    if og:
        def og_line(key, v):
            return {"value": round(v["gqups"], 4), "unit": "GQUPS", "ms_per_step": round(v["ms_per_step"], 4),
                    "median_of": v["median_of"], "samples_ms_per_step": v["samples_ms_per_step"],
                    "bytes_per_update": v["bpu"], "plan_build_s": round(v["plan_build_s"], 2),
                    "roofline": roofline(v, traffic_from_profiles(key)), "finite": v["finite"]}
        out["ogrid"] = {
            "workload": "supersonic NACA 0012 O-grid Ma 1.5 Re 1e4, 256x128 cells p=4 GLL (525312 nodes), D2V25, "
                        "curvilinear CSR plan",
            **{prec: og_line("ogrid_" + prec, v) for prec, v in og.items() if not prec.startswith("d2q19")}}
        if "d2q19_f32" in og:
            out["ogrid"]["d2q19"] = {
                "workload": "the same O-grid on the reduced degree-9 set D2Q19 (the paper's set for this case)",
                **{prec: dict(og_line("ogrid19_" + prec, og["d2q19_" + prec]),
                              step_time_vs_d2v25=round(og["d2q19_" + prec]["ms_per_step"] / og[prec]["ms_per_step"], 4))
                   for prec in ("f32", "f64")}}
    names = {"c1r": "2D periodic shear wave, 1024^2 cells p=4 GLL (16.8M nodes), D2V25",
             "c4": "3D supersonic channel Ma_b 1.5 Re_b 3000, 128x96x64 cells p=2 (6.3M nodes), D3V125, "
                   "isothermal walls, forcing held by the PI force controller and mass rescaling, both every 10 steps",
             "c4pr": "the same channel at the paper's Prandtl number 0.7 (the collision's quasi-equilibrium term; "
                     "the relaxation launch reads the populations twice)",
             "c1rq19": "the same 2D shear wave on the reduced velocity set D2Q19 (CFL 0.5 on its largest component; "
                       "single-pass tile with the wide weight-table count)",
             "c4paper": "the same channel with the paper's set-up: reduced velocity set D3Q45 (CFL 0.9 on its largest "
                        "component) and Prandtl number 0.7"}
    for key, v in extra.items():
        case, prec = key.split("_")
        out[key] = {"workload": names[case], "dtype": prec, "value": round(v["gqups"], 4), "unit": "GQUPS",
                    "ms_per_step": round(v["ms_per_step"], 4), "median_of": v["median_of"],
                    "samples_ms_per_step": v["samples_ms_per_step"], "roofline": roofline(v, traffic_from_profiles(key)),
                    "kernels": v["kernels"],
                    "finite": v["finite"], **({"force_control": v["force_control"]} if "force_control" in v else {})}
    if prec_cmp:
        out["fp32_vs_fp64"] = prec_cmp
    if prec_cmp_other:
        out["fp32_vs_fp64_" + other] = prec_cmp_other
    if lrn:
        out["learned"] = lrn
        if lrn_more:
            out["learned_other_mach"] = lrn_more
    if lrn_paper:
        out["learned_paper_setup"] = lrn_paper
    out["copy_ceiling"] = dict(ceil, note="1 GiB device-to-device copy, read + written bytes per second: the "
                                          "practical HBM peak; step_frac and frac are against 8 TB/s")
    if cal:
        out["copy_calibration"] = cal
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
