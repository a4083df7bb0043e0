"""Pins of the curvilinear (isoparametric quadrilateral) oracle and of the O-grid
generator, against things other than the oracle itself: the exact area of the annulus
around the airfoil, an independently written isoparametric map, an extended-precision
intersection of the departure path with the wall, the tensor-product oracle on the same
box (a separate code path: per-axis tracing, no point location), and uniform states that
every boundary condition must leave unchanged."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _lagrange_basis(xr, t):
    """Lagrange basis on nodes xr at points t, via the Vandermonde inverse (independent
    of the oracle's product formula)."""
    V = np.vander(np.asarray(xr), increasing=True)
    C = np.linalg.inv(V)                                   # column j: coefficients of l_j
    T = np.vander(np.atleast_1d(t), len(xr), increasing=True)
    return T @ C


def _cell_map(mesh, c, xi, eta):
    n1 = mesh.p + 1
    xr = oracle.support_points(mesh.p, mesh.nodes)
    P = mesh.node_xyz[mesh.cell_nodes[c]].reshape(n1, n1, 2)          # [jy, jx]
    lx, ly = _lagrange_basis(xr, xi)[0], _lagrange_basis(xr, eta)[0]
    return np.einsum("y,x,yxa->a", ly, lx, P)


def _airfoil_area():
    th = np.linspace(0.0, 2.0 * np.pi, 400001)
    S = W.naca0012_surface(th)
    return 0.5 * abs(np.sum(S[:-1, 0] * S[1:, 1] - S[1:, 0] * S[:-1, 1]))


@pytest.mark.parametrize("na,nr", [(48, 16), (128, 64)])
def test_ogrid_is_unfolded_and_covers_the_annulus(na, nr):
    """The isoparametric Jacobian keeps one sign in every cell (the trailing-edge point,
    a corner of two cells, is the one degenerate point), and the nodal volumes add up to
    the area between the R = 10 circle and the airfoil."""
    mesh, phys = W.naca_ogrid(n_around=na, n_radial=nr, p=4)
    n1 = mesh.p + 1
    xr = oracle.support_points(mesh.p, mesh.nodes)
    t = np.linspace(-0.98, 0.98, 7)
    L = _lagrange_basis(xr, t)
    V = np.vander(np.asarray(xr), increasing=True)
    C = np.linalg.inv(V)
    dT = np.vander(t, n1 - 1, increasing=True) * np.arange(1, n1)[None, :]
    dL = dT @ C[1:, :]
    X = mesh.node_xyz[mesh.cell_nodes].reshape(-1, n1, n1, 2)
    dxi = np.einsum("cyxa,gy,hx->cgha", X, L, dL)
    deta = np.einsum("cyxa,gy,hx->cgha", X, dL, L)
    det = dxi[..., 0] * deta[..., 1] - dxi[..., 1] * deta[..., 0]
    sgn = np.sign(np.median(det))
    assert np.all(det * sgn > 0)
    o = oracle.CurvOracle(mesh, phys, geometry=False)
    area = math.pi * 10.0 ** 2 - _airfoil_area()
    assert abs(o.node_vol.sum() - area) < 1e-8 * area


def test_ogrid_boundary_tags():
    """Wall on the airfoil; inlet on the upstream arc (polar angle beyond 100 deg about
    mid-chord), outlet downstream; junctions away from +-90 deg."""
    mesh, _ = W.naca_ogrid(n_around=64, n_radial=8, p=4)
    fb = mesh.cell_face_bc
    assert np.all(fb[:64, 2] == 0) and np.all(fb[-64:, 3] >= 1)
    n1 = mesh.p + 1
    for c in range(64 * 7, 64 * 8):
        mid = mesh.node_xyz[mesh.cell_nodes[c].reshape(n1, n1)[n1 - 1, n1 // 2]] - [0.5, 0.0]
        ang = math.degrees(math.atan2(mid[1], mid[0]))
        assert (fb[c, 3] == 1) == (abs(ang) > 100.0)
    assert mesh.bcs[0].kind == W.BC_WALL and mesh.bcs[1].kind == W.BC_INLET and mesh.bcs[2].kind == W.BC_OUTLET


def test_point_location_inverts_the_isoparametric_map():
    """x = map_c(xi) for random cells and reference points (near the trailing edge and
    the wall too): the oracle finds a cell whose map sends its xi' back to x."""
    mesh, phys = W.naca_ogrid(n_around=48, n_radial=16, p=4)
    o = oracle.CurvOracle(mesh, phys, geometry=False)
    rng = np.random.Generator(np.random.PCG64(11))
    cells = np.concatenate([[0, 47, 1, 46, 24], rng.integers(0, len(mesh.cell_nodes), 60)])
    for c in cells:
        xi = rng.uniform(-1, 1, 2)
        x = _cell_map(mesh, c, *xi)
        c2, xi2 = o.locate(x)
        assert c2 >= 0
        x2 = _cell_map(mesh, c2, *xi2)
        assert np.max(np.abs(x2 - x)) < 1e-12 * max(1.0, np.max(np.abs(x)))
        if c2 == c:
            assert np.max(np.abs(xi2 - xi)) < 1e-8
    # outside: inside the airfoil and beyond the circle
    assert o.locate(np.array([0.5, 0.0]))[0] == -1
    assert o.locate(np.array([0.5, 10.5]))[0] == -1


def test_exit_point_matches_extended_precision_intersection():
    """The backward path of a node next to the wall meets the wall where the face curve
    and the segment intersect; solved here in long double by Newton on (t, s)."""
    mesh, phys = W.naca_ogrid(n_around=48, n_radial=16, p=4)
    o = oracle.CurvOracle(mesh, phys, geometry=False)
    n1 = mesh.p + 1
    xr = np.array(oracle.support_points(mesh.p, mesh.nodes), dtype=np.longdouble)
    LD = np.longdouble

    def basis(t):
        l = np.ones(n1, dtype=LD)
        dl = np.zeros(n1, dtype=LD)
        for j in range(n1):
            others = [q for q in range(n1) if q != j]
            for q in others:
                l[j] *= (t - xr[q]) / (xr[j] - xr[q])
            for k in others:
                term = LD(1) / (xr[j] - xr[k])
                for q in others:
                    if q != k:
                        term *= (t - xr[q]) / (xr[j] - xr[q])
                dl[j] += term
        return l, dl

    checked = 0
    for c in [3, 10, 20, 30, 40, 45]:
        cn = mesh.cell_nodes[c].reshape(n1, n1)
        edge = mesh.node_xyz[cn[0, :]].astype(LD)             # the wall face (eta = -1)
        k = cn[1, 2]                                          # first node off the wall
        for i in range(o.Q):
            d = phys.dt * o.zeta[i]
            if o.locate(o.xyz[k] - d)[0] >= 0:
                continue
            s, bc = o.exit(o.xyz[k], -d)
            assert bc == 0
            x = o.xyz[k].astype(LD)
            dd = d.astype(LD)
            t, sl = LD(0), LD(s)
            for _ in range(60):
                l, dl = basis(t)
                F = l @ edge - (x - sl * dd)
                J = np.array([[dl @ edge[:, 0], dd[0]], [dl @ edge[:, 1], dd[1]]], dtype=LD)
                det = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
                t -= (J[1, 1] * F[0] - J[0, 1] * F[1]) / det
                sl -= (J[0, 0] * F[1] - J[1, 0] * F[0]) / det
            assert abs(float(sl) - s) < 1e-11
            checked += 1
    assert checked >= 10


def _box_tensor(p=3, ncell=(5, 4)):
    """A wall-bounded box: inlet at x = 0, outlet at x = L, thermal walls at y = 0, H.
    Tags follow the axis order so that a path through a corner resolves identically in
    both oracles (the tensor oracle takes the x face first, the curvilinear one the
    smaller tag)."""
    ex = np.array([0.0, 0.3, 0.7, 1.2, 1.5, 2.0])[: ncell[0] + 1]
    ey = np.array([0.0, 0.25, 0.6, 0.8, 1.0])[: ncell[1] + 1]
    bcs = [W.BC(kind=W.BC_INLET, rho=1.05, u=(0.4, 0.05, 0.0), T=1.0),
           W.BC(kind=W.BC_OUTLET),
           W.BC(kind=W.BC_WALL, T_wall=0.9)]
    return W.TensorMesh(dim=2, p=p, nodes="gll", ncell=ncell, edges=[ex, ey],
                        face_bc=[[0, 1], [2, 2]], bcs=bcs)


@pytest.mark.parametrize("relax_mode,Pr", [(0, 1.0), (1, 1.0), (1, 0.71)])
def test_axis_aligned_curvilinear_box_matches_tensor_oracle(relax_mode, Pr):
    """With straight cells the curvilinear oracle (point location, path-face crossing,
    reflection, outlet projection) and the tensor oracle (per-axis tracing) compute the
    same step; 6 steps from a seeded random state."""
    tm = _box_tensor()
    phys = W.Physics(dt=0.012, relax_mode=relax_mode, tau_bar=0.9, mu_ref=0.01, Pr=Pr)
    cm = W.curv_box(tm)
    ot = oracle.TensorOracle(tm, phys)
    oc = oracle.CurvOracle(cm, phys)
    xt, xc = ot.coords(), oc.coords()
    assert np.max(np.abs(xt - xc)) < 1e-15
    rho, u, T = W.random_fields(ot.N, 2, seed=21)
    pt = ot.init(rho, u, T)
    pc = oc.init(rho, u, T)
    assert np.max(np.abs(pt - pc)) < 1e-15
    for _ in range(6):
        pt = ot.step(pt)
        pc = oc.step(pc)
    assert np.max(np.abs(pt - pc)) < 1e-12 * np.max(np.abs(pt))
    assert np.sum(oc.g_src != np.tile(np.arange(oc.Q), (oc.N, 1)).T.reshape(-1)) > 0    # walls were hit


def _uniform_box(kinds, warp, state):
    rho, u, T = state
    tm = W.TensorMesh(dim=2, p=4, nodes="gll", ncell=(4, 3),
                      edges=[np.array([0.0, 0.4, 0.9, 1.3, 2.0]), np.array([0.0, 0.3, 0.7, 1.0])],
                      face_bc=[[0, 1], [2, 3]],
                      bcs=[W.BC(kind=k, rho=rho, u=(u[0], u[1], 0.0), T=T,
                                T_wall=T if k == W.BC_WALL else float("nan")) for k in kinds])
    return W.curv_box(tm, warp=warp)


@pytest.mark.parametrize("case", ["rest_thermal_walls", "flow_all_inlets", "flow_outlet_right"])
def test_uniform_states_are_fixed_points_on_a_warped_mesh(case):
    """Interpolation reproduces constants on curved cells; bounce-back and the thermal
    wall (T_w = T) keep a fluid at rest; an inlet in the state of the fluid and the
    outlet keep a uniform flow.  One BGK step must change nothing (to rounding)."""
    if case == "rest_thermal_walls":
        state = (1.2, (0.0, 0.0), 0.95)
        kinds = [W.BC_WALL] * 4
    elif case == "flow_all_inlets":
        state = (0.9, (0.5, -0.2), 1.1)
        kinds = [W.BC_INLET] * 4
    else:
        state = (0.9, (0.5, -0.2), 1.1)
        kinds = [W.BC_INLET, W.BC_OUTLET, W.BC_INLET, W.BC_INLET]
    mesh = _uniform_box(kinds, warp=1.0, state=state)
    phys = W.Physics(dt=0.01, tau_bar=0.8)
    o = oracle.CurvOracle(mesh, phys)
    n = o.N
    rho = np.full(n, state[0])
    u = np.tile(state[1], (n, 1))
    T = np.full(n, state[2])
    p0 = o.init(rho, u, T)
    p1 = o.step(p0)
    assert np.max(np.abs(p1 - p0)) < 1e-13 * np.max(np.abs(p0))


def test_step_at_sampled_nodes_equals_full_step():
    mesh, phys = W.naca_ogrid(n_around=32, n_radial=8, p=3)
    o = oracle.CurvOracle(mesh, phys)
    rho, u, T = W.naca_fields(o.coords())
    pop = o.run(o.init(rho, u, T), 2)
    full = o.step(pop).reshape(2 * o.Q, o.N)
    nodes = np.array([0, 3, 17, o.N // 2, o.N - 1])
    assert np.array_equal(o.step_nodes(pop, nodes), full[:, nodes].T)
