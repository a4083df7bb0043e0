"""Parity of the curvilinear (CSR) HIP path, through the C-ABI, with the FP64 oracle.

Bars.  FP64: 1e-11 relative per field and on the populations.  Both sides locate the
same departure points with independent geometry code (the oracle intersects each wall
curve with the path by bisection, the library by Newton); where a path meets the wall
at a small angle theta the crossing is fixed only to about eps / sin theta, and on the
airfoil grids below the two interpolated values agree to 2.2e-13 in one step, so 1e-11
after 10-30 steps keeps a margin while a wrong weight, row or boundary case shows up at
1e-4 or more.  FP32 storage: 1e-5.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from harness import GpuRun, field_errors, oracle_moments, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-5
CSR = 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare(mesh, phys, prec, fields, nsteps, tol, mass_fix_every=0):
    o = oracle.CurvOracle(mesh, phys)
    g = GpuRun(mesh, phys, prec)
    say("kernel in use", g.kernel, "nodes", g.N)
    assert g.kernel == CSR
    xyz = o.coords()
    assert np.max(np.abs(g.coords() - xyz)) == 0.0
    rho, u, T = fields(xyz)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    mref = o.totals(p0)[0] if mass_fix_every else None
    pr = o.run(p0, nsteps, mass_fix_every=mass_fix_every, mass_ref=mref)
    g.run(nsteps, mass_fix_every=mass_fix_every, mass_ref=mref)
    errs = field_errors(g.moments(), oracle_moments(o, pr))
    e = rel_err(g.pop(), pr)
    say("errors", errs, "pop", e)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    assert e <= tol
    return o, g, pr


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_airfoil_ogrid_mach_1_5(prec, tol):
    mesh, phys = W.naca_ogrid(n_around=48, n_radial=16, p=4, Ma=1.5)
    say("NACA O-grid 48x16 p=4 Ma 1.5", prec)
    _compare(mesh, phys, prec, lambda x: W.naca_fields(x, Ma=1.5), 20, tol)


def test_airfoil_ogrid_mach_2_fp64():
    mesh, phys = W.naca_ogrid(n_around=64, n_radial=24, p=4, Ma=2.0)
    say("NACA O-grid 64x24 p=4 Ma 2")
    _compare(mesh, phys, "f64", lambda x: W.naca_fields(x, Ma=2.0), 10, TOL64)


@pytest.mark.parametrize("p", [2, 3])
def test_airfoil_ogrid_lower_orders_fp64(p):
    mesh, phys = W.naca_ogrid(n_around=40, n_radial=12, p=p, Ma=1.5)
    say("NACA O-grid 40x12 p", p)
    _compare(mesh, phys, "f64", lambda x: W.naca_fields(x, Ma=1.5), 10, TOL64)


def _warped_box(p=3):
    """Thermal walls at y = 0, 1, equilibrium inlet at x = 0, outlet at x = 2, curved
    interior cells; the corners exercise the nearest-boundary-point rule."""
    tm = W.TensorMesh(dim=2, p=p, nodes="gll", ncell=(6, 4),
                      edges=[np.array([0.0, 0.3, 0.7, 1.0, 1.3, 1.6, 2.0]), np.array([0.0, 0.2, 0.5, 0.8, 1.0])],
                      face_bc=[[0, 1], [2, 2]],
                      bcs=[W.BC(kind=W.BC_INLET, rho=1.05, u=(0.4, 0.05, 0.0), T=1.0),
                           W.BC(kind=W.BC_OUTLET),
                           W.BC(kind=W.BC_WALL, T_wall=0.9)])
    return W.curv_box(tm, warp=1.0)


def _box_fields(x):
    return W.random_fields(x.shape[0], 2, seed=31, u_mean=(0.3, 0.0))


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("relax_mode", [0, 1])
def test_warped_box_walls_inlet_outlet(prec, tol, relax_mode):
    mesh = _warped_box()
    phys = W.Physics(dt=0.01, relax_mode=relax_mode, tau_bar=0.9, mu_ref=0.01)
    say("warped box relax_mode", relax_mode, prec)
    _compare(mesh, phys, prec, _box_fields, 30, tol)


def test_warped_box_force_and_mass_fix_fp64():
    mesh = _warped_box(p=4)
    phys = W.Physics(dt=0.01, relax_mode=0, tau_bar=0.8, force=(0.05, -0.02, 0.0))
    say("warped box force + mass fix")
    _compare(mesh, phys, "f64", _box_fields, 20, TOL64, mass_fix_every=4)


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_full_size_ogrid_one_step_sampled(prec, tol):
    """The 256 x 128 cell, p = 4 O-grid (525,312 nodes) at Ma 1.5: one step from the
    initial field on the GPU, checked at 512 sampled nodes (all wall nodes' neighbours
    included) against the oracle's step at those nodes."""
    mesh, phys = W.naca_ogrid()
    say("full-size O-grid", prec)
    o = oracle.CurvOracle(mesh, phys, geometry=False)
    g = GpuRun(mesh, phys, prec)
    assert g.kernel == CSR
    xyz = o.coords()
    rho, u, T = W.naca_fields(xyz)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    g.run(1)
    got = g.pop().reshape(2 * o.Q, o.N)
    rng = np.random.Generator(np.random.PCG64(5))
    n_ring = 256 * 4
    nodes = np.unique(np.concatenate([rng.choice(o.N, 384, replace=False),
                                      np.arange(0, n_ring, 8), np.arange(n_ring, 2 * n_ring, 8),
                                      np.arange(o.N - n_ring, o.N, 16)]))
    ref = o.step_nodes(p0, nodes)
    e = rel_err(got[:, nodes].T, ref)
    say("sampled pop error", e, "nodes", nodes.size)
    assert e <= tol
