"""Parity of the HIP path with the FP64 oracle at Prandtl numbers other than 1 (the
collision's quasi-equilibrium term, Sec. 3.1 update display), on every kernel that relaxes:
the single-pass 2D tile, the 3D tile and its relaxation launch (two nodes per lane in FP64,
one in FP32), the per-node gather kernel (also on the wall slabs of a tiled plan), the
two-launch 2D tile with one node per lane, and the curvilinear kernel with and without its
register stash.  Bars: FP64 1e-12 (1e-11 on curvilinear meshes), FP32 storage 1e-5 in
rho, u, T.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from harness import GpuRun, field_errors, oracle_moments, rel_err

pytestmark = pytest.mark.gpu

TOL64, TOL64_CURV, TOL32 = 1e-12, 1e-11, 1e-5
GATHER, TILED = 1, 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _vel(dim, vel, T0):
    if vel == "cub":
        return oracle.cubature_set(dim, T0)
    return oracle.velocity_set(dim, int(vel[2:] or 5), T0)


def _compare(mesh, phys, prec, fields, nsteps, tol, kernel=0, vel="gh", curv=False, compare_pops=True,
             mass_fix_every=0, expect_kernel=None):
    ov = _vel(mesh.dim if not curv else 2, vel, phys.T0)
    o = oracle.CurvOracle(mesh, phys, vel=ov) if curv else oracle.TensorOracle(mesh, phys, vel=ov)
    g = GpuRun(mesh, phys, prec, kernel, vel=vel)
    say("kernel in use", g.kernel, "Q", g.Q, "N", g.N, "Pr", phys.Pr)
    if expect_kernel is not None:
        assert g.kernel == expect_kernel
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
    # the term acts: the same run at Pr = 1 differs
    if nsteps >= 10:
        o1 = (oracle.CurvOracle if curv else oracle.TensorOracle)(mesh, dataclasses.replace(phys, Pr=1.0), vel=ov)
        assert rel_err(o1.run(p0, nsteps), pr) > 1e-9


def _shear(x):
    return W.shear_wave_fields(x, noise=1e-3, seed=2)


def _thermal_shear(x):
    rho, u, T = W.shear_wave_fields(x, noise=1e-3, seed=3)
    T = T + 0.05 * np.sin(x[:, 1])
    return rho / T, u, T


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("relax_mode", [0, 1])
def test_2d_single_pass_tile(prec, tol, relax_mode):
    say("Pr 0.71 2D single-pass tile", prec, relax_mode)
    mesh, phys = W.shear_wave_case(ncell=16, p=4)
    phys = dataclasses.replace(phys, Pr=0.71, relax_mode=relax_mode, mu_ref=0.01, T_ref=1.0, mu_exp=0.7)
    _compare(mesh, phys, prec, _thermal_shear, 30, tol, kernel=TILED, compare_pops=(prec == "f64"),
             expect_kernel=2)


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_2d_single_pass_tile_d2q19(prec, tol):
    say("Pr 0.71 2D single-pass tile on D2Q19", prec)
    mesh, phys = W.shear_wave_case(ncell=16, p=4)
    phys = dataclasses.replace(phys, Pr=0.71)
    _compare(mesh, phys, prec, _thermal_shear, 30, tol, kernel=TILED, vel="cub", compare_pops=(prec == "f64"),
             expect_kernel=2)


def test_2d_gather_fp64():
    say("Pr 0.71 2D gather")
    mesh, phys = W.shear_wave_case(ncell=8, p=4)
    phys = dataclasses.replace(phys, Pr=0.71)
    _compare(mesh, phys, "f64", _thermal_shear, 30, TOL64, kernel=GATHER, expect_kernel=0)


def test_2d_two_launch_tile_one_node_per_lane_fp64():
    """D2V16 (4 points per axis) on an 11 x 5-cell p = 3 mesh: the 2D tile stores the streamed
    values and the relaxation launch runs one node per lane (N = 33 x 15 is odd)."""
    say("Pr 0.71 2D two-launch tile, D2V16, odd N")
    tm = W.TensorMesh(dim=2, p=3, nodes="gll", ncell=(11, 5),
                      edges=[W.uniform_edges(11, 0.0, 11.0), W.uniform_edges(5, 0.0, 5.0)], face_bc=[[-1, -1], [-1, -1]])
    phys = W.Physics(dt=0.1, relax_mode=0, tau_bar=0.9, Pr=0.71)
    _compare(tm, phys, "f64", lambda x: W.random_fields(x.shape[0], 2, seed=51, u_amp=0.1), 15, TOL64,
             kernel=TILED, vel="gh4", expect_kernel=2)


@pytest.mark.parametrize("kernel", [pytest.param(GATHER, id="gather"), pytest.param(TILED, id="tiled")])
@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_3d_tgv(prec, tol, kernel):
    say("Pr 0.71 TGV 6^3 p3", prec, kernel)
    mesh, phys = W.tgv_case(ncell=6, p=3, dt=W.TGV_DT)
    phys = dataclasses.replace(phys, Pr=0.71)
    _compare(mesh, phys, prec, W.tgv_fields, 20, tol, kernel=kernel, compare_pops=(prec == "f64"))


@pytest.mark.parametrize("vel", ["gh", "cub"])
@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_channel_walls_force_mass_fix(prec, tol, vel):
    """The channel sub-box at Pr 0.7 (the paper's channel): thermal walls in the gather
    kernel's slabs, the tile and its relaxation launch inside, force, mass rescaling."""
    say("Pr 0.7 channel sub-box", prec, vel)
    mesh, phys = W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.75, T_wall=0.9, Ma_b=0.5)
    phys = dataclasses.replace(phys, Pr=0.7)
    _compare(mesh, phys, prec, lambda x: W.channel_fields(x, box=(2.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0), 20, tol,
             kernel=TILED, vel=vel, compare_pops=(prec == "f64"), mass_fix_every=5, expect_kernel=2)


def _warped_box(p=3):
    tm = W.TensorMesh(dim=2, p=p, nodes="gll", ncell=(6, 4),
                      edges=[np.array([0.0, 0.3, 0.7, 1.0, 1.3, 1.6, 2.0]), np.array([0.0, 0.2, 0.5, 0.8, 1.0])],
                      face_bc=[[0, 1], [2, 2]],
                      bcs=[W.BC(kind=W.BC_INLET, rho=1.05, u=(0.4, 0.05, 0.0), T=1.0),
                           W.BC(kind=W.BC_OUTLET),
                           W.BC(kind=W.BC_WALL, T_wall=0.9)])
    return W.curv_box(tm, warp=1.0)


@pytest.mark.parametrize("vel", ["gh", "cub", "gh4"])
@pytest.mark.parametrize("prec,tol", [("f64", TOL64_CURV), ("f32", TOL32)])
def test_curvilinear_warped_box(prec, tol, vel):
    """D2V25 and D2Q19 keep the streamed values in registers; D2V16 runs the generic path,
    which streams a third time for the heat flux."""
    say("Pr 0.71 warped box", prec, vel)
    phys = W.Physics(dt=0.01, relax_mode=1, tau_bar=0.9, mu_ref=0.01, Pr=0.71)
    _compare(_warped_box(), phys, prec, lambda x: W.random_fields(x.shape[0], 2, seed=31, u_mean=(0.3, 0.0)), 30,
             tol, vel=vel, curv=True, expect_kernel=1)
