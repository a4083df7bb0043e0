"""The velocity-split 3D step (kernel choice 3): one velocity per workgroup on a column of
output nodes, the source planes walked once along z, then the moments and the relaxation from
a node's streamed values held in the registers of the waves of a workgroup.

It computes the tiled kernel's numbers up to the order of the moment sums (the relaxation
adds the sums of the waves' parts): FP64 populations after several steps agree with the tiled
kernel's to 1e-13 and with the FP64 oracle at the FP64 bar (1e-12); FP32 storage with the tiled
kernel to 1e-6 and with the oracle to 1e-5 in rho, u, T.  Meshes with ragged x-y tiles and z
chunks, mildly stretched cells along z, forcing, Pr != 1, the three relaxation modes, and
walls in y (the boundary layers stay on the gather kernel), on D3Q45 and D3V125.
"""
import dataclasses
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
TILED, SPLIT = 2, 3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def box_case(ncell, p, stretch=0.0, **phys_kw):
    """A periodic 2 pi box of ncell = (nx, ny, nz) cells, its z cells stretched by a factor
    up to 1 + stretch (smooth, periodic), at the Taylor-Green time step of its smallest cell."""
    L = 2.0 * math.pi
    edges = [W.uniform_edges(n, 0.0, L) for n in ncell]
    if stretch:
        s = np.arange(ncell[2] + 1) / ncell[2]
        z = s + stretch / (2 * math.pi) * np.sin(2 * math.pi * s) / (1 + stretch)
        edges[2] = L * (z - z[0]) / (z[-1] - z[0])
    mesh = W.TensorMesh(dim=3, p=p, nodes="gll", ncell=tuple(ncell), edges=edges,
                        face_bc=[[-1, -1], [-1, -1], [-1, -1]])
    hmin = min(float(np.min(np.diff(e))) for e in edges)
    _, tgv = W.tgv_case(ncell=8, p=p)
    phys = dataclasses.replace(tgv, dt=0.5 * hmin / W.ZETA_MAX_GH5, **phys_kw)
    return mesh, phys


def _run_pair(mesh, phys, prec, nsteps, fields=W.tgv_fields, vel="cub"):
    """The same initial state stepped by the tiled kernel and by the velocity-split step."""
    runs = {}
    for kernel in (TILED, SPLIT):
        g = GpuRun(mesh, phys, prec, kernel, vel=vel)
        assert g.kernel == kernel
        rho, u, T = fields(g.coords())
        g.init(rho, u, T)
        g.run(nsteps)
        runs[kernel] = g
    return runs[TILED], runs[SPLIT]


CASES = [
    pytest.param(2, (26, 15, 13), 0.0, id="p2-ragged"),
    pytest.param(3, (18, 11, 9), 0.0, id="p3-ragged"),
    pytest.param(3, (18, 10, 12), 0.3, id="p3-stretched-z"),
    pytest.param(4, (14, 9, 8), 0.0, id="p4-ragged"),
]


@pytest.mark.parametrize("p,ncell,stretch", CASES)
def test_split_matches_tiled_fp64(p, ncell, stretch):
    say("split vs tiled fp64", p, ncell, stretch)
    mesh, phys = box_case(ncell, p, stretch)
    t, s = _run_pair(mesh, phys, "f64", 6)
    e = rel_err(s.pop(), t.pop())
    say("rel err", e)
    assert e <= 1e-13


# FP32 plans whose y axis is long enough run two output columns per thread (24-node tiles in y),
# shorter ones one; D3Q45 at p = 3 always runs one (the p = 3 two-column kernel is covered by
# the D3V125 cases below)
CASES32 = CASES + [
    pytest.param(3, (18, 7, 9), 0.0, id="p3-short-y"),
    pytest.param(2, (26, 14, 13), 0.0, id="p2-two-columns"),
    pytest.param(3, (18, 10, 9), 0.3, id="p3-long-y-stretched-z"),
    pytest.param(4, (14, 8, 8), 0.0, id="p4-two-columns"),
]


@pytest.mark.parametrize("p,ncell,stretch", CASES32)
def test_split_matches_tiled_fp32(p, ncell, stretch):
    say("split vs tiled fp32", p, ncell, stretch)
    mesh, phys = box_case(ncell, p, stretch)
    t, s = _run_pair(mesh, phys, "f32", 6)
    e = rel_err(s.pop(), t.pop())
    say("rel err", e)
    assert e <= 1e-6


@pytest.mark.parametrize("variant", ["mode1", "force_pr", "mode0", "streaming"])
def test_split_matches_tiled_physics_variants_fp64(variant):
    """Constant forcing with Pr = 0.71 (the heat-flux term), constant tau_bar, and pure
    streaming: each term of the relaxation launch, against the tiled kernel's."""
    kw = {"mode1": {}, "force_pr": {"force": (0.02, -0.01, 0.005), "Pr": 0.71},
          "mode0": {"relax_mode": 0, "tau_bar": 0.8}, "streaming": {"relax_mode": 2}}[variant]
    say("split vs tiled fp64", variant)
    mesh, phys = box_case((18, 11, 9), 3, **kw)
    t, s = _run_pair(mesh, phys, "f64", 5)
    e = rel_err(s.pop(), t.pop())
    say("rel err", e)
    assert e <= (0.0 if variant == "streaming" else 1e-13)


# ------------------------------------------------------------------ bounded meshes

def _channel(prec_kw=None):
    """The channel sub-box long enough in x for the 48-node tiles: tanh walls in y,
    isothermal walls at 0.9, power-law viscosity, Kupershtokh force, Pr 0.7, D3Q45 at a CFL
    of 0.75 on the product rule's largest abscissa."""
    mesh, phys = W.channel_case(ncell=(26, 8, 14), p=2, box=(4.0, 2.0, 1.5), cfl=0.75, T_wall=0.9, Ma_b=0.5)
    return mesh, dataclasses.replace(phys, Pr=0.7)


def _channel_fields(x):
    return W.channel_fields(x, box=(4.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0)


def _mixing():
    """The mixing layer's moving equilibrium walls in y, 26 x 8 x 14 cells, p = 2."""
    return W.mixing_layer_case(ncell=(26, 8, 14), p=2, Ma_c=0.7, box=(26 * 2.5 * W.MIX_DTHETA0, 8 * 2.75 * W.MIX_DTHETA0,
                                                                    14 * 1.5 * W.MIX_DTHETA0))


def _mixing_fields(x):
    return W.mixing_layer_fields(x, Ma_c=0.7, box=(26 * 2.5 * W.MIX_DTHETA0, 8 * 2.75 * W.MIX_DTHETA0,
                                                  14 * 1.5 * W.MIX_DTHETA0))


def _run_pair_fix(mesh, phys, prec, nsteps, fields, fix_every, vel="cub"):
    runs = {}
    for kernel in (TILED, SPLIT):
        g = GpuRun(mesh, phys, prec, kernel, vel=vel)
        assert g.kernel == kernel
        rho, u, T = fields(g.coords())
        g.init(rho, u, T)
        mref = g.moments(totals=True)["totals"][0] if fix_every else None
        g.run(nsteps, mass_fix_every=fix_every, mass_ref=mref)
        runs[kernel] = g
    return runs[TILED], runs[SPLIT]


@pytest.mark.parametrize("case", ["channel", "mixing"])
def test_split_matches_tiled_bounded_fp64(case):
    """Walls in y (thermal walls and forcing with the mass rescaling; moving equilibrium
    walls): the boundary layers stay on the gather kernel, the interior on the split step."""
    say("split vs tiled fp64 bounded", case)
    mesh, phys = _channel() if case == "channel" else _mixing()
    fields = _channel_fields if case == "channel" else _mixing_fields
    t, s = _run_pair_fix(mesh, phys, "f64", 6, fields, 3 if case == "channel" else 0)
    e = rel_err(s.pop(), t.pop())
    say("rel err", e)
    assert e <= 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_split_oracle_parity_channel(prec, tol):
    say("split vs oracle, channel", prec)
    mesh, phys = _channel()
    o, g = _oracle_pair(mesh, phys, prec)
    xyz = o.coords()
    rho, u, T = _channel_fields(xyz)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    mref = o.totals(p0)[0]
    pr = o.run(p0, 20, mass_fix_every=5, mass_ref=mref)
    g.run(20, mass_fix_every=5, mass_ref=mref)
    errs = field_errors(g.moments(), oracle_moments(o, pr))
    say("errors", errs)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if prec == "f64":
        e = rel_err(g.pop(), pr)
        say("pop error", e)
        assert e <= tol


def _oracle_pair(mesh, phys, prec):
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(3, phys.T0))
    g = GpuRun(mesh, phys, prec, SPLIT, vel="cub")
    assert g.kernel == SPLIT
    return o, g


@pytest.mark.parametrize("prec,tol,nsteps,ncell", [("f64", TOL64, 20, (18, 11, 9)), ("f32", TOL32, 20, (18, 7, 9)),
                                                   ("f32", TOL32, 20, (18, 11, 9))])
def test_split_oracle_parity(prec, tol, nsteps, ncell):
    say("split vs oracle", prec, nsteps, ncell)
    mesh, phys = box_case(ncell, 3, stretch=0.3, force=(0.01, 0.0, -0.01), Pr=0.71)
    o, g = _oracle_pair(mesh, phys, prec)
    xyz = o.coords()
    assert np.max(np.abs(g.coords() - xyz)) < 1e-13
    rho, u, T = W.tgv_fields(xyz)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    pr = o.run(p0, nsteps)
    g.run(nsteps)
    errs = field_errors(g.moments(), oracle_moments(o, pr))
    say("errors", errs)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if prec == "f64":
        e = rel_err(g.pop(), pr)
        say("pop error", e)
        assert e <= tol


def test_split_full_size_taylor_green_sampled():
    """The headline mesh (96^3 nodes, p = 3, FP64, D3Q45, the 32^3-cell time step), as the
    benchmark runs it (automatic choice): one step from the oracle's initial state, checked
    at sampled nodes (tile and z-chunk edges among them) against the oracle node by node."""
    mesh, phys = W.tgv_case(ncell=32, p=3, dt=W.TGV_DT)
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(3, phys.T0))
    g = GpuRun(mesh, phys, "f64", 0, vel="cub")
    assert g.kernel == SPLIT
    rho, u, T = W.tgv_fields(g.coords())
    p0 = o.init(rho, u, T)
    g.load(p0)
    g.run(1)
    got = g.pop()
    rng = np.random.Generator(np.random.PCG64(11))
    n = 96
    edges = [0, 23, 24, 47, 48, 71, 72, 95]
    special = [x + n * (y + n * z) for x in edges[::3] for y in edges[1::3] for z in (0, 47, 48, 95)]
    nodes = np.unique(np.concatenate([rng.integers(0, o.N, 60), special]))
    ref = o.step_nodes(p0, nodes)
    gq = np.stack([got[nodes + q * o.N] for q in range(2 * o.Q)], axis=1)
    e = rel_err(gq, ref)
    say("sampled nodes", len(nodes), "pop error", e)
    assert e <= TOL64


# ------------------------------------------------------------------ D3V125 (125 velocities)

@pytest.mark.parametrize("p,ncell,stretch", [pytest.param(2, (26, 15, 13), 0.0, id="p2-ragged"),
                                             pytest.param(3, (18, 10, 9), 0.3, id="p3-stretched-z")])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_split_d3v125_matches_tiled(p, ncell, stretch, prec, tol):
    say("split vs tiled d3v125", p, ncell, prec)
    mesh, phys = box_case(ncell, p, stretch, force=(0.01, 0.0, -0.01), Pr=0.71)
    t, s = _run_pair(mesh, phys, prec, 6, vel="gh")
    e = rel_err(s.pop(), t.pop())
    say("rel err", e)
    assert e <= tol


def test_split_d3v125_channel_matches_tiled():
    say("split vs tiled d3v125 channel fp64")
    mesh, phys = _channel()
    t, s = _run_pair_fix(mesh, phys, "f64", 6, _channel_fields, 3, vel="gh")
    e = rel_err(s.pop(), t.pop())
    say("rel err", e)
    assert e <= 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_split_d3v125_oracle_parity(prec, tol):
    say("split vs oracle d3v125", prec)
    mesh, phys = box_case((18, 11, 9), 3, stretch=0.3, force=(0.01, 0.0, -0.01), Pr=0.71)
    o = oracle.TensorOracle(mesh, phys)
    g = GpuRun(mesh, phys, prec, SPLIT)
    assert g.kernel == SPLIT and g.Q == 125
    xyz = o.coords()
    rho, u, T = W.tgv_fields(xyz)
    p0 = o.init(rho, u, T)
    g.init(rho, u, T)
    pr = o.run(p0, 20)
    g.run(20)
    errs = field_errors(g.moments(), oracle_moments(o, pr))
    say("errors", errs)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if prec == "f64":
        e = rel_err(g.pop(), pr)
        say("pop error", e)
        assert e <= tol
