"""Parity of the HIP path with the FP64 oracle on the reduced velocity sets D2Q19 and
D3Q45 (Sec. 3.2): the library's closed-form sets on the GPU, the oracle's own sets solved
from the moment conditions on the CPU.

Bars as for the product-rule sets: FP64 1e-12 relative per field and on the populations
(1e-11 on curvilinear meshes, whose wall crossings the two sides locate with different
geometry code), FP32 storage 1e-5 in rho, u, T.
"""
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
GATHER, TILED, CSR = 1, 2, 1
KERNELS = [pytest.param(GATHER, id="gather"), pytest.param(TILED, id="tiled")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare(o, g, fields, nsteps, tol, compare_pops=True, mass_fix_every=0):
    say("kernel in use", g.kernel, "Q", g.Q, "nodes", g.N)
    assert g.Q == (19 if g.D == 2 else 45)
    xyz = o.coords()
    assert np.max(np.abs(g.coords() - xyz)) < 1e-13
    rho, u, T = fields(xyz)
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


def _tensor(mesh, phys, prec, kernel=0):
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(mesh.dim, phys.T0))
    return o, GpuRun(mesh, phys, prec, kernel, vel="cub")


# ------------------------------------------------------------------ D3Q45, periodic

@pytest.mark.parametrize("kernel", KERNELS)
def test_d3q45_tgv_fp64_small(kernel):
    say("D3Q45 TGV fp64 6^3 p3 20 steps", kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3)
    o, g = _tensor(mesh, phys, "f64", kernel)
    assert g.kernel == (2 if kernel == TILED else 0)
    _compare(o, g, W.tgv_fields, 20, TOL64)


@pytest.mark.parametrize("kernel", KERNELS)
def test_d3q45_tgv_fp32_small_100_steps(kernel):
    say("D3Q45 TGV fp32 6^3 p3 100 steps at the 32^3 time step", kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3, dt=W.TGV_DT)
    o, g = _tensor(mesh, phys, "f32", kernel)
    _compare(o, g, W.tgv_fields, 100, TOL32, compare_pops=False)


@pytest.mark.parametrize("p", [2, 4])
def test_d3q45_other_orders_tiled_fp64(p):
    say("D3Q45 TGV fp64 4^3 cells p", p)
    mesh, phys = W.tgv_case(ncell=4 if p == 4 else 6, p=p)
    o, g = _tensor(mesh, phys, "f64", TILED)
    _compare(o, g, W.tgv_fields, 10, TOL64)


# ------------------------------------------------------------------ D3Q45, walls

def _channel_small():
    """The channel sub-box (tanh walls, isothermal walls at 0.9, power-law viscosity,
    Kupershtokh force) at a CFL of 0.75 on the product rule's largest abscissa: D3Q45's
    largest component (3.29 against 2.86) then moves 0.86 of the smallest cell."""
    return W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.75, T_wall=0.9, Ma_b=0.5)


def _channel_fields(x):
    return W.channel_fields(x, box=(2.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_d3q45_channel_thermal_walls_forcing(prec, tol, kernel):
    say("D3Q45 channel sub-box 6x8x6 p2 20 steps", prec, kernel)
    mesh, phys = _channel_small()
    o, g = _tensor(mesh, phys, prec, kernel)
    _compare(o, g, _channel_fields, 20, tol, compare_pops=(prec == "f64"), mass_fix_every=5)


# ------------------------------------------------------------------ D2Q19

@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_d2q19_shear_wave_100_steps(prec, tol, kernel):
    """2D tensor meshes on D2Q19: the single-pass tile with the wide table count (eleven
    displacements along x), and the gather kernel."""
    say("D2Q19 shear wave 16^2 p4 100 steps", prec, kernel)
    mesh, phys = W.shear_wave_case(ncell=16, p=4)
    o, g = _tensor(mesh, phys, prec, kernel)
    assert g.kernel == (2 if kernel == TILED else 0)
    _compare(o, g, lambda x: W.shear_wave_fields(x, noise=1e-3, seed=2), 100, tol, compare_pops=(prec == "f64"))


@pytest.mark.parametrize("p", [2, 3])
def test_d2q19_tiled_lower_orders_fp64(p):
    say("D2Q19 vortex tiled p", p)
    mesh, phys = W.vortex_case(ncell=16, p=p)
    o, g = _tensor(mesh, phys, "f64", TILED)
    _compare(o, g, lambda x: W.vortex_fields(x), 20, TOL64)


def test_d2q19_bounce_back_stretched_fp64():
    say("D2Q19 stretched channel with bounce-back walls")
    tm = W.TensorMesh(dim=2, p=3, nodes="gll", ncell=(12, 6),
                      edges=[W.uniform_edges(12, 0.0, 3.0), W.tanh_edges(6, 1.5)],
                      face_bc=[[-1, -1], [0, 0]], bcs=[W.BC(kind=W.BC_WALL)])
    phys = W.Physics(dt=0.02, relax_mode=0, tau_bar=0.9)
    o, g = _tensor(tm, phys, "f64", TILED)
    assert g.kernel == 2   # wall slabs by the gather kernel, the interior by the tile
    _compare(o, g, lambda x: W.random_fields(x.shape[0], 2, seed=41, u_mean=(0.3, 0.0)), 20, TOL64)


def _warped_box(p=3):
    tm = W.TensorMesh(dim=2, p=p, nodes="gll", ncell=(6, 4),
                      edges=[np.array([0.0, 0.3, 0.7, 1.0, 1.3, 1.6, 2.0]), np.array([0.0, 0.2, 0.5, 0.8, 1.0])],
                      face_bc=[[0, 1], [2, 2]],
                      bcs=[W.BC(kind=W.BC_INLET, rho=1.05, u=(0.4, 0.05, 0.0), T=1.0),
                           W.BC(kind=W.BC_OUTLET),
                           W.BC(kind=W.BC_WALL, T_wall=0.9)])
    return W.curv_box(tm, warp=1.0)


def _curv(mesh, phys, prec):
    o = oracle.CurvOracle(mesh, phys, vel=oracle.cubature_set(2, phys.T0))
    g = GpuRun(mesh, phys, prec, vel="cub")
    assert g.kernel == CSR
    return o, g


@pytest.mark.parametrize("prec,tol", [("f64", TOL64_CURV), ("f32", TOL32)])
def test_d2q19_warped_box_walls_inlet_outlet(prec, tol):
    say("D2Q19 warped box", prec)
    mesh = _warped_box()
    phys = W.Physics(dt=0.01, relax_mode=1, tau_bar=0.9, mu_ref=0.01)
    o, g = _curv(mesh, phys, prec)
    _compare(o, g, lambda x: W.random_fields(x.shape[0], 2, seed=31, u_mean=(0.3, 0.0)), 30, tol)


@pytest.mark.parametrize("prec,tol", [("f64", TOL64_CURV), ("f32", TOL32)])
def test_d2q19_airfoil_ogrid_mach_1_5(prec, tol):
    say("D2Q19 NACA O-grid 48x16 p=4 Ma 1.5", prec)
    mesh, phys = W.naca_ogrid(n_around=48, n_radial=16, p=4, Ma=1.5)
    o, g = _curv(mesh, phys, prec)
    _compare(o, g, lambda x: W.naca_fields(x, Ma=1.5), 20, tol)


# ------------------------------------------------------------------ full size, sampled

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_d3q45_tgv_full_size_one_step_sampled(prec):
    """The 96^3-node TGV with D3Q45 on the tiled kernel, one step, sampled nodes."""
    say("D3Q45 TGV full size sampled", prec)
    mesh, phys = W.tgv_case()
    o, g = _tensor(mesh, phys, prec, TILED)
    rho, u, T = W.tgv_fields(g.coords())
    p0 = o.init(rho, u, T)
    g.load(p0)
    g.run(1)
    got = g.pop()
    rng = np.random.Generator(np.random.PCG64(13))
    nodes = np.unique(np.concatenate([[0, 1, 95, 96, o.N - 1], rng.integers(0, o.N, 150)])).astype(np.int64)
    pin = p0.astype(np.float32).astype(np.float64) if prec == "f32" else p0
    ref = o.step_nodes(pin, nodes)
    gq = np.stack([got[nodes + q * o.N] for q in range(2 * o.Q)], axis=1)
    e = rel_err(gq, ref)
    say("sampled pop error", e)
    assert e <= (TOL64 if prec == "f64" else 2e-6)


# ------------------------------------------------------------------ boundaries and modes

def test_d3q45_inlet_outlet_3d():
    say("D3Q45 3D inlet + outlet")
    mesh = W.TensorMesh(dim=3, p=2, nodes="glc", ncell=(3, 4, 3),
                        edges=[W.uniform_edges(3, 0, 1.5), W.uniform_edges(4, 0, 2.0), W.uniform_edges(3, 0, 1.5)],
                        face_bc=[[-1, -1], [0, 1], [-1, -1]],
                        bcs=[W.BC(kind=W.BC_INLET, rho=1.0, u=(0, 0.4, 0), T=1.0), W.BC(kind=W.BC_OUTLET)])
    phys = W.Physics(dt=0.04, relax_mode=0, tau_bar=0.9)
    o, g = _tensor(mesh, phys, "f64")
    _compare(o, g, lambda x: W.random_fields(x.shape[0], 3, seed=7, u_amp=0.2, u_mean=(0, 0.4, 0)), 10, TOL64)


def test_d2q19_moving_equilibrium_walls():
    say("D2Q19 moving equilibrium walls")
    mesh = W.TensorMesh(dim=2, p=2, nodes="gll", ncell=(6, 5), edges=[W.uniform_edges(6, 0, 3.0),
                                                                    W.uniform_edges(5, -1.0, 1.0)],
                        face_bc=[[-1, -1], [0, 1]],
                        bcs=[W.BC(kind=W.BC_INLET, rho=1.0, u=(-0.5, 0, 0), T=1.0),
                             W.BC(kind=W.BC_INLET, rho=1.0, u=(0.5, 0, 0), T=1.0)])
    phys = W.Physics(dt=0.04, relax_mode=0, tau_bar=0.9)
    o, g = _tensor(mesh, phys, "f64")
    _compare(o, g, lambda x: W.random_fields(x.shape[0], 2, seed=6, u_amp=0.2), 15, TOL64)


@pytest.mark.parametrize("dim", [2, 3])
def test_reduced_sets_linear_elements_gather(dim):
    """p = 1 (no tile kernel for it): the gather kernel on both reduced sets."""
    say("reduced set p=1 gather, dim", dim)
    if dim == 2:
        mesh, phys = W.shear_wave_case(ncell=24, p=1)
        fields = lambda x: W.shear_wave_fields(x, noise=1e-3, seed=2)
    else:
        mesh, phys = W.tgv_case(ncell=10, p=1, dt=W.TGV_DT)
        fields = W.tgv_fields
    o, g = _tensor(mesh, phys, "f64")
    assert g.kernel == 0
    _compare(o, g, fields, 10, TOL64)


@pytest.mark.parametrize("kernel", KERNELS)
def test_d3q45_pure_streaming_and_mass_fix(kernel):
    import dataclasses
    say("D3Q45 streaming only, then mass fix", kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3)
    o, g = _tensor(mesh, dataclasses.replace(phys, relax_mode=2), "f64", kernel)
    _compare(o, g, W.tgv_fields, 5, TOL64)
    o, g = _tensor(mesh, phys, "f64", kernel)
    _compare(o, g, W.tgv_fields, 9, TOL64, mass_fix_every=3)
