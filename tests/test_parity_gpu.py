"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bars: FP64 GPU path <= 1e-12 relative per field (rho, u, T; populations too) after the
stated number of steps; FP32 storage path <= 1e-5 relative in rho, u, T after 100 steps.
Both sides start from the same seeded nodal fields and build their own equilibria.
"""
import copy
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from harness import GpuRun, field_errors, oracle_moments, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


GATHER, TILED = 1, 2
SPLIT = 3
KERNELS = [pytest.param(GATHER, id="gather"), pytest.param(TILED, id="tiled")]


def _pair(mesh, phys, prec, fields, kernel=0):
    o = oracle.TensorOracle(mesh, phys)
    g = GpuRun(mesh, phys, prec, kernel)
    say("kernel in use", g.kernel)
    xyz = o.coords()
    assert np.max(np.abs(g.coords() - xyz)) < 1e-13
    rho, u, T = fields(xyz)
    return o, g, (rho, u, T)


def _run_compare(mesh, phys, prec, fields, nsteps, tol, compare_pops=True, mass_fix_every=0, kernel=0):
    o, g, (rho, u, T) = _pair(mesh, phys, prec, fields, kernel)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    mref = o.totals(p0)[0] if mass_fix_every else None
    pr = o.run(p0, nsteps, mass_fix_every=mass_fix_every, mass_ref=mref)
    g.run(nsteps, mass_fix_every=mass_fix_every, mass_ref=mref)
    errs = field_errors(g.moments(), oracle_moments(o, pr))
    say("errors", errs)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if compare_pops:
        e = rel_err(g.pop(), pr)
        say("pop error", e)
        assert e <= tol
    return o, g, pr


# ------------------------------------------------------------------ init / moments

@pytest.mark.parametrize("dim", [2, 3])
def test_init_equilibrium_and_moments(dim):
    say("case init", dim)
    if dim == 2:
        mesh, phys = W.shear_wave_case(ncell=5, p=3)
    else:
        mesh, phys = W.tgv_case(ncell=3, p=2)
    o, g, (rho, u, T) = _pair(mesh, phys, "f64", lambda x: W.random_fields(x.shape[0], dim, seed=3, u_mean=(0.4, -0.2, 0.1)))
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    assert rel_err(g.pop(), p0) < 1e-14
    mom = g.moments(totals=True)
    ref = oracle_moments(o, p0)
    for k in ("rho", "u", "T"):
        assert rel_err(mom[k], ref[k]) < 1e-14
    m, P, E = o.totals(p0)
    tot = mom["totals"]
    assert abs(tot[0] - m) < 1e-13 * abs(m)
    for a in range(dim):
        assert abs(tot[1 + a] - P[a]) < 1e-13 * max(abs(m), 1)
    assert abs(tot[1 + dim] - E) < 1e-13 * abs(E)


# ------------------------------------------------------------------ C1

@pytest.mark.parametrize("kernel", KERNELS)
def test_shear_wave_fp64_100_steps(kernel):
    say("case C1a shear wave fp64 16x16 p4 100 steps", kernel)
    mesh, phys = W.shear_wave_case()
    _run_compare(mesh, phys, "f64", lambda x: W.shear_wave_fields(x, noise=1e-3, seed=1), 100, TOL64, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_isentropic_vortex_fp64_100_steps(kernel):
    say("case C1b vortex fp64 16x16 p4 100 steps", kernel)
    mesh, phys = W.vortex_case()
    _run_compare(mesh, phys, "f64", lambda x: W.vortex_fields(x, noise=1e-3, seed=1), 100, TOL64, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_shear_wave_fp32_100_steps(kernel):
    say("case C1a shear wave fp32 100 steps", kernel)
    mesh, phys = W.shear_wave_case()
    _run_compare(mesh, phys, "f32", lambda x: W.shear_wave_fields(x, noise=1e-3, seed=1), 100, TOL32,
                 compare_pops=False, kernel=kernel)


@pytest.mark.parametrize("p,fam", [(1, "gll"), (2, "glc"), (3, "equi"), (4, "glc")])
def test_orders_and_node_families_fp64(p, fam):
    say("case 2D p", p, fam)
    mesh, phys = W.shear_wave_case(ncell=7, p=p, nodes=fam, tau_bar=0.9)
    _run_compare(mesh, phys, "f64", lambda x: W.shear_wave_fields(x, noise=1e-3, seed=2), 20, TOL64)


def test_smallest_periodic_mesh():
    say("case 2 cells p2")
    mesh, phys = W.shear_wave_case(ncell=2, p=2, cfl=0.9)
    _run_compare(mesh, phys, "f64", lambda x: W.shear_wave_fields(x, noise=1e-3, seed=2), 10, TOL64)


# ------------------------------------------------------------------ C2

@pytest.mark.parametrize("kernel", KERNELS)
def test_tgv_fp64_small(kernel):
    say("case C2 TGV fp64 6^3 p3 20 steps", kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3)
    _run_compare(mesh, phys, "f64", lambda x: W.tgv_fields(x), 20, TOL64, kernel=kernel)


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("p,ncell", [(2, 9), (4, 5)])
def test_tgv_tiled_orders_2_and_4_ragged(p, ncell, prec, tol):
    """The 3D tile kernel at p = 2 and 4, where it skews the passes of consecutive velocities
    (two barriers per velocity, double-buffered weight rows), on D3V125 with a ragged last
    tile on every axis (18 nodes per axis at p = 2, 20 at p = 4, against 8-node tiles)."""
    say("case C2 TGV tiled", prec, "p", p, "cells", ncell, "10 steps")
    mesh, phys = W.tgv_case(ncell=ncell, p=p)
    _, g, _ = _run_compare(mesh, phys, prec, lambda x: W.tgv_fields(x), 10, tol, compare_pops=(prec == "f64"),
                           kernel=TILED)
    assert g.kernel == TILED


@pytest.mark.parametrize("kernel", KERNELS)
def test_tgv_fp32_small_100_steps(kernel):
    """100 steps at the time step of the 32^3 configuration (t = 3.4, before the
    vortex's transition).  A coarse mesh at its own CFL time step would reach t = 22,
    where the transitional flow amplifies any rounding ~15x per 50 steps."""
    say("case C2 TGV fp32 6^3 p3 100 steps at the C2 time step", kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3, dt=W.TGV_DT)
    _run_compare(mesh, phys, "f32", lambda x: W.tgv_fields(x), 100, TOL32, compare_pops=False, kernel=kernel)


# ------------------------------------------------------------------ walls, inlet, outlet

def _channel_small():
    """Channel sub-box with the C4 machinery (tanh-stretched walls, isothermal walls at
    T_w = 0.9 against a fluid at T = 1, power-law viscosity, Kupershtokh forcing) at bulk
    Ma 0.5: at Ma 1.5 with T = T0 the Gauss-Hermite set is unstable within 4 steps in the
    oracle as well."""
    return W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.9, T_wall=0.9, Ma_b=0.5)


def _channel_fields(x):
    return W.channel_fields(x, box=(2.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0)


@pytest.mark.parametrize("kernel", KERNELS)
def test_channel_thermal_walls_forcing_fp64(kernel):
    say("case C4 sub-box fp64 6x8x6 p2 20 steps", kernel)
    mesh, phys = _channel_small()
    _run_compare(mesh, phys, "f64", _channel_fields, 20, TOL64, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_channel_thermal_walls_forcing_fp32(kernel):
    say("case C4 sub-box fp32 20 steps", kernel)
    mesh, phys = _channel_small()
    _run_compare(mesh, phys, "f32", _channel_fields, 20, TOL32, compare_pops=False, kernel=kernel)


def test_plain_bounce_back_2d_stretched():
    say("case 2D bounce-back stretched")
    ey = np.array([0.0, 0.15, 0.5, 1.1, 1.7, 2.05, 2.2])
    mesh = W.TensorMesh(dim=2, p=3, nodes="gll", ncell=(5, 6), edges=[W.uniform_edges(5, 0, 3.0), ey],
                        face_bc=[[-1, -1], [0, 0]], bcs=[W.BC(kind=W.BC_WALL)])
    phys = W.Physics(dt=0.04, relax_mode=0, tau_bar=0.8)
    _run_compare(mesh, phys, "f64", lambda x: W.random_fields(x.shape[0], 2, seed=5, u_amp=0.1), 15, TOL64)


def test_moving_equilibrium_walls_inlet():
    say("case 2D inlet moving equilibrium walls")
    mesh = W.TensorMesh(dim=2, p=2, nodes="gll", ncell=(6, 5), edges=[W.uniform_edges(6, 0, 3.0),
                                                                    W.uniform_edges(5, -1.0, 1.0)],
                        face_bc=[[-1, -1], [0, 1]],
                        bcs=[W.BC(kind=W.BC_INLET, rho=1.0, u=(-0.5, 0, 0), T=1.0),
                             W.BC(kind=W.BC_INLET, rho=1.0, u=(0.5, 0, 0), T=1.0)])
    phys = W.Physics(dt=0.05, relax_mode=0, tau_bar=0.9)
    _run_compare(mesh, phys, "f64", lambda x: W.random_fields(x.shape[0], 2, seed=6, u_amp=0.2), 15, TOL64)


def test_outlet_3d():
    say("case 3D outlet")
    mesh = W.TensorMesh(dim=3, p=2, nodes="glc", ncell=(3, 4, 3),
                        edges=[W.uniform_edges(3, 0, 1.5), W.uniform_edges(4, 0, 2.0), W.uniform_edges(3, 0, 1.5)],
                        face_bc=[[-1, -1], [0, 1], [-1, -1]],
                        bcs=[W.BC(kind=W.BC_INLET, rho=1.0, u=(0, 0.4, 0), T=1.0), W.BC(kind=W.BC_OUTLET)])
    phys = W.Physics(dt=0.05, relax_mode=0, tau_bar=0.9)
    _run_compare(mesh, phys, "f64", lambda x: W.random_fields(x.shape[0], 3, seed=7, u_amp=0.2, u_mean=(0, 0.4, 0)),
                 10, TOL64)


def test_pure_streaming_mode():
    say("case pure streaming")
    mesh, phys = W.shear_wave_case(ncell=6, p=4)
    phys = copy.copy(phys)
    phys.relax_mode = 2
    _run_compare(mesh, phys, "f64", lambda x: W.random_fields(x.shape[0], 2, seed=8), 5, TOL64)


@pytest.mark.parametrize("kernel", KERNELS)
def test_mass_fix_every_3_steps(kernel):
    say("case mass fix", kernel)
    mesh, phys = W.shear_wave_case(ncell=12, p=3)
    _run_compare(mesh, phys, "f64", lambda x: W.shear_wave_fields(x, noise=0.05, seed=9), 10, TOL64, mass_fix_every=3,
                 kernel=kernel)


# ------------------------------------------------------------------ full size, sampled

def _sample_nodes(N, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = set([0, 1, 255, 256, N - 257, N - 2, N - 1])
    s.update(rng.integers(0, N, n).tolist())
    return np.array(sorted(s), dtype=np.int64)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tgv_full_size_one_step_sampled(prec, kernel):
    """The bench workload (32^3 cells p=3, 96^3 nodes, D3V125) one step from the TGV
    state, checked at sampled nodes against the oracle evaluated node by node."""
    say("case C2 full size sampled", prec, kernel)
    mesh, phys = W.tgv_case()
    o = oracle.TensorOracle(mesh, phys)
    g = GpuRun(mesh, phys, prec, kernel)
    xyz = g.coords()
    rho, u, T = W.tgv_fields(xyz)
    p0 = o.init(rho, u, T)
    g.load(p0)
    g.run(1)
    got = g.pop()
    nodes = _sample_nodes(o.N, 150, 11)
    # FP32 path starts from the FP32-rounded state: give the oracle the same input
    pin = p0.astype(np.float32).astype(np.float64) if prec == "f32" else p0
    ref = o.step_nodes(pin, nodes)
    gq = np.stack([got[nodes + q * o.N] for q in range(2 * o.Q)], axis=1)
    e = rel_err(gq, ref)
    say("sampled pop error", e)
    assert e <= (TOL64 if prec == "f64" else 2e-6)


def test_kernel_selection_reports_the_kernel_in_use():
    """Automatic choice: the tile from 256 tiles up (one per compute unit), with velocity-split
    steps on a periodic mesh, else the gather kernel; an explicit choice of either where the
    tile applies."""
    say("case kernel selection")
    mesh, phys = W.tgv_case(ncell=6, p=3)          # 18^3 nodes: 12 tiles
    assert GpuRun(mesh, phys, "f64").kernel == 0
    assert GpuRun(mesh, phys, "f64", TILED).kernel == TILED
    assert GpuRun(mesh, phys, "f64", GATHER).kernel == 0
    big, physb = W.tgv_case(ncell=24, p=3)         # 72^3 nodes: 6 x 6 x 12 = 432 tiles
    assert GpuRun(big, physb, "f32").kernel == SPLIT
    assert GpuRun(big, physb, "f32", TILED).kernel == TILED
    mesh5, phys5 = W.tgv_case(ncell=5, p=3)   # 15 nodes per axis: too few for a tile + halo
    assert GpuRun(mesh5, phys5, "f64").kernel == 0


def test_plan_profile_counts_every_launch():
    """Per-kernel event timing: one entry per launch of each kernel of the step."""
    mesh, phys = W.tgv_case(ncell=8, p=3)
    g = GpuRun(mesh, phys, "f64", TILED)
    rho, u, T = W.tgv_fields(g.coords())
    g.init(rho, u, T)
    g.S.sllbm_plan_profile(g.plan, True)
    g.run(7)
    prof = g.S.sllbm_plan_profile_read(g.plan)
    g.S.sllbm_plan_profile(g.plan, False)
    say("profile", prof)
    assert g.kernel == TILED
    assert prof["k_step_tile"][1] == 7 and prof["k_relax_nodes"][1] == 7
    assert all(ms > 0 for ms, _ in prof.values())
    g.run(2)
    assert g.S.sllbm_plan_profile_read(g.plan) == prof   # stopped: nothing more recorded


# ------------------------------------------------------------------ 2D single-pass tile kernel

def _shear_2d_tiled(relax_mode, force=(0.0, 0.0)):
    """A 2D periodic mesh large enough for the tiled kernel (its single pass with D2V25)."""
    mesh, phys = W.shear_wave_case(ncell=12, p=4)
    phys = copy.copy(phys)
    phys.relax_mode = relax_mode
    if relax_mode == 1:
        phys.mu_ref, phys.T_ref, phys.mu_exp = 0.02, 1.0, 0.7
    phys.force = tuple(force) + (0.0,)
    return mesh, phys


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_2d_single_pass_viscosity_law_and_force(prec, tol):
    """mu(T) power law and a Kupershtokh body force through the single-pass 2D tile kernel."""
    say("case 2D single pass, relax mode 1 + force", prec)
    mesh, phys = _shear_2d_tiled(1, force=(0.03, -0.02))
    _run_compare(mesh, phys, prec, lambda x: W.shear_wave_fields(x, amp=0.05, noise=0.01, seed=12), 40, tol,
                 compare_pops=(prec == "f64"), kernel=TILED)


def test_2d_single_pass_pure_streaming():
    """relax mode 2: the kernel stores the streamed values as they are."""
    say("case 2D single pass, pure streaming")
    mesh, phys = _shear_2d_tiled(2)
    _run_compare(mesh, phys, "f64", lambda x: W.random_fields(x.shape[0], 2, seed=13), 6, TOL64, kernel=TILED)


def test_2d_single_pass_controlled_force():
    """The device-side force controller on the single-pass 2D kernel: force history and
    populations against the oracle's controller."""
    import dataclasses
    say("case 2D single pass, force controller")
    mesh, phys = _shear_2d_tiled(0, force=(0.02, 0.0))
    o, g, (rho, u, T) = _pair(mesh, phys, "f64", lambda x: W.shear_wave_fields(x, amp=0.05, seed=14), TILED)
    pop = o.init(rho, u, T)
    g.init(rho, u, T)
    ctl = {"axis": 0, "target": 0.9, "kp": 3.0, "ki": 2.0}
    c = oracle.ForceController(o, phys.force, **ctl)
    g.S.sllbm_force_reset(g.plan, phys.force)
    prm = dataclasses.replace(g.prm, force_device=1)
    for n in range(9):
        if n % 3 == 0:
            F = c.update(pop, 3 * phys.dt)
            g.S.sllbm_force_update(g.plan, g.a, dt=3 * phys.dt, **ctl)
            st = g.S.sllbm_force_read(g.plan)
            # the controller multiplies the mean momentum's error (1e-12 relative) by its gains
            scale = abs(phys.force[0]) + ctl["kp"] * abs(ctl["target"]) + ctl["ki"] * abs(c.integral)
            assert abs(st["force"][0] - F[0]) <= 1e-12 * scale, (n, st["force"][0], F[0])
        pop = o.step(pop)
        g.S.sllbm_step(g.plan, prm, g.a, g.b)
        g.a, g.b = g.b, g.a
    g.torch.cuda.synchronize()
    e = rel_err(g.pop(), pop)
    say("pop error", e)
    assert e <= TOL64


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_gather_two_lanes_per_node(prec, tol):
    """A gather launch of 131,072-262,143 nodes deals each node's velocities over two lanes
    (smaller launches four, larger one): 96 x 96 cells p = 4 (147,456 nodes) on the gather
    kernel, 5 steps, the whole field against the oracle."""
    say("gather, two lanes per node: shear wave 96^2 p4", prec)
    mesh, phys = W.shear_wave_case(ncell=96, p=4)
    _run_compare(mesh, phys, prec, lambda x: W.shear_wave_fields(x, noise=1e-3, seed=4), 5, tol,
                 compare_pops=(prec == "f64"), kernel=GATHER)
