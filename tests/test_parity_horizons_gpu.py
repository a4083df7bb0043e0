"""Parity of the HIP path with the FP64 oracle over 100 steps on every workload shape, and
one step of the channel at its full size and Mach number.

Bars: FP64 GPU path <= 1e-12 relative per field (rho, u, T) and on the populations after 100
steps on tensor meshes; the curvilinear FP64 path <= 1e-11 (its departure points come from
independent geometry code on each side, see test_parity_curv_gpu); FP32 storage <= 1e-5 in
rho, u and T after 100 steps.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from harness import GpuRun, field_errors, oracle_moments, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL64_CURV = 1e-11
TOL32 = 1e-5
GATHER, TILED = 1, 2
KERNELS = [pytest.param(GATHER, id="gather"), pytest.param(TILED, id="tiled")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_ORACLE_RUNS = {}


def _compare(o, g, fields, nsteps, tol, compare_pops, mass_fix_every=0, key=None):
    """key: the oracle's run of a case is kept under this name and reused by the other
    kernels and precisions of the same case (the FP32 path is judged against FP64 too)."""
    xyz = o.coords()
    assert np.max(np.abs(g.coords() - xyz)) < 1e-13
    rho, u, T = fields(xyz)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    mref = o.totals(p0)[0] if mass_fix_every else None
    if key is None or key not in _ORACLE_RUNS:
        pr = o.run(p0, nsteps, mass_fix_every=mass_fix_every, mass_ref=mref)
        if key is not None:
            _ORACLE_RUNS[key] = pr
    pr = _ORACLE_RUNS[key] if key is not None else pr
    g.run(nsteps, mass_fix_every=mass_fix_every, mass_ref=mref)
    errs = field_errors(g.moments(), oracle_moments(o, pr))
    e = rel_err(g.pop(), pr) if compare_pops else None
    say("kernel", g.kernel, "nodes", g.N, "Q", g.Q, "steps", nsteps, "errors", errs, "pop", e)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if compare_pops:
        assert e <= tol


def _prec_tol(prec):
    return (TOL64, True) if prec == "f64" else (TOL32, False)


PRECS = ["f64", "f32"]


# ------------------------------------------------------------------ C2: Taylor-Green, 100 steps

@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", KERNELS)
def test_tgv_100_steps(kernel, prec):
    """6^3 cells p = 3 at the time step of the 32^3-cell workload (t = 3.4), D3V125."""
    say("case C2 TGV 6^3 p3 100 steps", prec, kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3, dt=W.TGV_DT)
    tol, pops = _prec_tol(prec)
    _compare(oracle.TensorOracle(mesh, phys), GpuRun(mesh, phys, prec, kernel), W.tgv_fields, 100, tol, pops, key="tgv")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", KERNELS)
def test_tgv_d3q45_100_steps(kernel, prec):
    """The same on the reduced degree-9 set D3Q45 (Sec. 3.2)."""
    say("case C2 TGV D3Q45 6^3 p3 100 steps", prec, kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3, dt=W.TGV_DT)
    tol, pops = _prec_tol(prec)
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(3, phys.T0))
    _compare(o, GpuRun(mesh, phys, prec, kernel, vel="cub"), W.tgv_fields, 100, tol, pops, key="tgv45")


# ------------------------------------------------------------------ C4: channel sub-box, 100 steps

def _channel_box():
    """The channel's machinery (tanh-stretched isothermal walls at T_w = 0.9 against a fluid at
    T = 1, the mu(T) power law with omega = 0.7, Kupershtokh forcing, mass rescaling) on a
    6 x 8 x 6-cell box at bulk Ma 0.5."""
    return W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.9, T_wall=0.9, Ma_b=0.5)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", KERNELS)
def test_channel_box_100_steps(kernel, prec):
    say("case C4 box 6x8x6 p2 100 steps, mass fix every 10", prec, kernel)
    mesh, phys = _channel_box()
    tol, pops = _prec_tol(prec)
    _compare(oracle.TensorOracle(mesh, phys), GpuRun(mesh, phys, prec, kernel),
             lambda x: W.channel_fields(x, box=(2.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0), 100, tol, pops,
             mass_fix_every=10, key="channel")


# ------------------------------------------------------------------ C5: mixing-layer box, 100 steps

def _mixing_box():
    """The coarse mixing layer's cell (2.5 x 2.75 x 1.5 initial momentum thicknesses, p = 2)
    on a 6^3-cell box: moving equilibrium walls at u_x = -+du/2 (Ma_c 0.7), relax mode 1."""
    d0 = W.MIX_DTHETA0
    box = (15 * d0, 16.5 * d0, 9 * d0)
    mesh, phys = W.mixing_layer_case(ncell=(6, 6, 6), box=box, Ma_c=0.7)
    return mesh, phys, box


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", KERNELS)
def test_mixing_layer_box_100_steps(kernel, prec):
    say("case C5 box 6^3 p2 100 steps", prec, kernel)
    mesh, phys, box = _mixing_box()
    tol, pops = _prec_tol(prec)
    _compare(oracle.TensorOracle(mesh, phys), GpuRun(mesh, phys, prec, kernel),
             lambda x: W.mixing_layer_fields(x, box=box, amp=0.1, seed=5, Ma_c=0.7), 100, tol, pops,
             key="mixing")


def test_mixing_layer_box_d3q45_pr071_100_steps():
    """The paper's mixing-layer set-up (Sec. 4.4): D3Q45 at Pr = 0.71, FP64."""
    say("case C5 box D3Q45 Pr 0.71 100 steps")
    mesh, phys, box = _mixing_box()
    phys = dataclasses.replace(phys, Pr=0.71)
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(3, phys.T0))
    _compare(o, GpuRun(mesh, phys, "f64", vel="cub"),
             lambda x: W.mixing_layer_fields(x, box=box, amp=0.1, seed=5, Ma_c=0.7), 100, TOL64, True)


# ------------------------------------------------------------------ C3: airfoil O-grid, 100 steps

@pytest.mark.parametrize("prec", PRECS)
def test_airfoil_ogrid_100_steps(prec):
    """48 x 16 cells p = 4 around the NACA 0012 section at Ma 1.5 (thermal wall, inlet and
    outlet), D2V25."""
    say("case C3 O-grid 48x16 p4 100 steps", prec)
    mesh, phys = W.naca_ogrid(n_around=48, n_radial=16, p=4, Ma=1.5)
    tol, pops = (TOL64_CURV, True) if prec == "f64" else (TOL32, False)
    o = oracle.CurvOracle(mesh, phys)
    g = GpuRun(mesh, phys, prec)
    _compare(o, g, lambda x: W.naca_fields(x, Ma=1.5), 100, tol, pops, key="ogrid")


# ------------------------------------------------------------------ C4 at its full size

def _wall_layer_nodes(mesh, n_wall, n_bulk, seed):
    """Sampled node indices of the channel (x fastest): n_wall nodes in the first and last
    five node planes along y, n_bulk anywhere."""
    Nx, Ny, Nz = (mesh.axis_nodes(a) for a in range(3))
    rng = np.random.Generator(np.random.PCG64(seed))
    ys = np.concatenate([np.arange(5), np.arange(Ny - 5, Ny)])
    x = rng.integers(0, Nx, n_wall)
    z = rng.integers(0, Nz, n_wall)
    y = ys[rng.integers(0, ys.size, n_wall)]
    wall = x + Nx * (y + Ny * z)
    bulk = rng.integers(0, Nx * Ny * Nz, n_bulk)
    edge = np.array([0, Nx - 1, Nx * Ny - 1, Nx * Ny * Nz - 1])
    return np.unique(np.concatenate([wall, bulk, edge])).astype(np.int64)


@pytest.mark.parametrize("prec", PRECS)
def test_channel_full_size_one_step_sampled(prec):
    """The channel workload as benchmarked: 128 x 96 x 64 cells p = 2 (6,324,224 nodes),
    tanh-stretched isothermal walls, bulk Ma 1.5, mu(T) with omega = 0.7, the body force,
    D3V125, in the kernel choice of the plan (tile in the interior, gather in the wall
    layers).  One step from the initial field, checked at sampled nodes (most of them in the
    wall layers) against the oracle evaluated node by node."""
    say("case C4 full size one step sampled", prec)
    mesh, phys = W.channel_case()
    o = oracle.TensorOracle(mesh, phys)
    g = GpuRun(mesh, phys, prec)
    say("kernel in use", g.kernel, "nodes", g.N)
    xyz = g.coords()
    rho, u, T = W.channel_fields(xyz)
    p0 = o.init(rho, u, T)
    if prec == "f32":
        p0 = p0.astype(np.float32).astype(np.float64)     # the state the FP32 path starts from
    g.load(p0)
    g.run(1)
    nodes = _wall_layer_nodes(mesh, 400, 100, 13)
    ref = o.step_nodes(p0, nodes)
    got = np.stack([g.a[q * g.N + g.torch.tensor(nodes, device="cuda")].double().cpu().numpy()
                    for q in range(2 * g.Q)], axis=1)
    e = rel_err(got, ref)
    say("sampled pop error", e, "nodes", nodes.size)
    assert e <= (TOL64 if prec == "f64" else 2e-6)
