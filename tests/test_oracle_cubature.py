"""Pins of the oracle's reduced velocity sets D2Q19 and D3Q45 (Sec. 3.2).

The paper gives the point counts and the quadrature degree (9) but no abscissae.  These
tests check the oracle's rules against what fixes them mathematically: every monomial of
total degree <= 9 integrated exactly against the Gaussian (moments from the closed form
(k-1)!! per axis, written here, not taken from the oracle), positive weights, central
symmetry, and then the method built on them: the equilibrium's Maxwellian moments to
order 4, the closed-form viscous decay of a shear wave, conservation on a periodic box.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def dfact(k):
    return 1 if k <= 0 else k * dfact(k - 2)


def gauss_moment(k, mean=0.0, var=1.0):
    s = 0.0
    for j in range(0, k + 1, 2):
        s += math.comb(k, j) * mean ** (k - j) * var ** (j / 2) * dfact(j - 1)
    return s


def monomial_errors(zeta, w, degree, T0=1.0):
    """Largest relative error of sum_i w_i prod_a zeta_ia^m_a against the Gaussian moment
    prod_a E[X^m_a], X ~ N(0, T0), over the monomials of total degree `degree`."""
    dim = zeta.shape[1]
    worst = 0.0
    for m in itertools.product(range(degree + 1), repeat=dim):
        if sum(m) != degree:
            continue
        ref = 1.0
        for a in range(dim):
            ref *= gauss_moment(m[a], 0.0, T0)
        got = float(np.sum(w * np.prod(zeta ** np.array(m), axis=1)))
        worst = max(worst, abs(got - ref) / max(1.0, abs(ref)))
    return worst


@pytest.mark.parametrize("dim", [2, 3])
def test_cubature_counts_match_paper(dim):
    zeta, w, opp = oracle.cubature_set(dim)
    assert zeta.shape == (GOLD["cubature_points_2d_3d_degree_9"]["value"][dim - 2], dim)
    assert len(w) > oracle.stroud_bound(9, dim)
    if dim == 3:
        assert math.floor(100 * (1 - len(w) / 343)) == GOLD["cubature_reduction_percent"]["value"]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("T0", [1.0, 1.3])
def test_cubature_degree_9_exact_and_10_not(dim, T0):
    zeta, w, _ = oracle.cubature_set(dim, T0)
    for deg in range(10):
        assert monomial_errors(zeta, w, deg, T0) < 1e-13, deg
    assert monomial_errors(zeta, w, 10, T0) > 1e-2


@pytest.mark.parametrize("dim", [2, 3])
def test_cubature_structure(dim):
    zeta, w, opp = oracle.cubature_set(dim)
    Q = len(w)
    assert np.all(w > 0) and abs(w.sum() - 1.0) < 1e-15
    assert np.all(zeta[0] == 0) and np.array_equal(opp[opp], np.arange(Q))
    assert np.array_equal(zeta[opp], -zeta)
    # orbit radii: 2D s = (48 -+ 8 sqrt 15)/7 and 8; 3D s = 3, 15, 9 (|zeta|^2 at T0 = 1)
    s = np.sum(zeta ** 2, axis=1)
    want = [(48 - 8 * math.sqrt(15)) / 7, (48 + 8 * math.sqrt(15)) / 7, 8.0] if dim == 2 else [3.0, 15.0, 9.0]
    n = 6 if dim == 2 else 12
    sizes = [n, n, 6 if dim == 2 else 20]
    k = 1
    for sz, sw in zip(sizes, want):
        assert np.allclose(s[k:k + sz], sw, rtol=1e-14), (k, sw)
        assert np.ptp(w[k:k + sz]) == 0
        k += sz
    if dim == 3:  # the rule's weights are rational: 28/135, 25/432, 1/2160, 1/216
        assert np.allclose([w[0], w[1], w[13], w[25]], [28 / 135, 25 / 432, 1 / 2160, 1 / 216], rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("state", [(1.0, (0.0, 0.0, 0.0), 1.0), (1.3, (0.7, -0.4, 0.25), 0.8)])
def test_cubature_equilibrium_maxwellian_moments_to_order_4(dim, state):
    rho, u, T = state
    vel = oracle.cubature_set(dim)
    zeta = vel[0]
    feq, geq = oracle.equilibrium(dim, rho, u[:dim], T, vel=vel)
    for m in itertools.product(range(5), repeat=dim):
        if sum(m) > 4:
            continue
        ref = rho
        for a in range(dim):
            ref *= gauss_moment(m[a], u[a], T)
        got = float(np.sum(feq * np.prod(zeta ** np.array(m), axis=1)))
        assert abs(got - ref) < 2e-14 * max(1.0, abs(ref)), (m, got, ref)
    assert np.allclose(geq, T * (2 / 0.4 - dim) * feq, rtol=1e-15, atol=0)


def test_d2q19_shear_wave_viscous_decay():
    """Closed form: u_y = A sin(x - U t) exp(-nu t), nu = (tau_bar - 1/2) T0 dt."""
    tau_bar = 1.3
    mesh, phys = W.shear_wave_case(ncell=16, p=4, tau_bar=tau_bar)
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(2, phys.T0))
    xyz = o.coords()
    rho, u, T = W.shear_wave_fields(xyz, noise=0.0)
    pop = o.init(rho, u, T)
    V = o.node_vol

    def amp(pp):
        _, uu, _ = o.moments(pp)
        s = np.sum(V * uu[:, 1] * np.sin(xyz[:, 0]))
        c = np.sum(V * uu[:, 1] * np.cos(xyz[:, 0]))
        return math.hypot(s, c) / np.sum(V * np.sin(xyz[:, 0]) ** 2)

    n = 100
    a0, a1 = amp(pop), amp(o.run(pop, n))
    nu = -math.log(a1 / a0) / (n * phys.dt)
    nu_ref = (tau_bar - 0.5) * phys.T0 * phys.dt
    assert abs(nu - nu_ref) < 0.02 * nu_ref


def _shear_decay_3d(axis_k, axis_u, nc=16, tau_bar=1.3, n=100):
    """3D box of nc cells along axis_k (2 along the others), p = 3: u = U e_k + A sin(x_k) e_u.
    Returns (nu / nu_ref - 1, relative drift of the mass) after n steps."""
    L = 2.0 * math.pi
    ncell = [2, 2, 2]
    ncell[axis_k] = nc
    mesh = W.TensorMesh(dim=3, p=3, nodes="gll", ncell=tuple(ncell),
                        edges=[W.uniform_edges(c, 0.0, L) for c in ncell], face_bc=[[-1, -1]] * 3)
    phys = W.Physics(gamma=1.4, dt=0.5 * (L / nc) / W.ZETA_MAX_GH5, relax_mode=0, tau_bar=tau_bar)
    o = oracle.TensorOracle(mesh, phys, vel=oracle.cubature_set(3, phys.T0))
    x = o.coords()
    u = np.zeros((o.N, 3))
    u[:, axis_k] = 0.5 * math.sqrt(1.4)
    u[:, axis_u] = 0.01 * np.sin(x[:, axis_k])
    pop = o.init(np.ones(o.N), u, np.ones(o.N))
    V = o.node_vol

    def amp(pp):
        uu = o.moments(pp)[1][:, axis_u]
        return math.hypot(np.sum(V * uu * np.sin(x[:, axis_k])), np.sum(V * uu * np.cos(x[:, axis_k])))

    m0 = o.totals(pop)[0]
    a0 = amp(pop)
    pop = o.run(pop, n)
    nu = -math.log(amp(pop) / a0) / (n * phys.dt)
    return nu / ((tau_bar - 0.5) * phys.T0 * phys.dt) - 1.0, o.totals(pop)[0] / m0 - 1.0


def test_d3q45_shear_wave_viscous_decay_and_isotropy():
    """The 3D set gives the closed-form shear viscosity, and the same decay for a wave along
    x (velocity along y) as along z (velocity along x): the set is invariant under the
    cyclic permutation of the axes that maps one case onto the other."""
    ex, mx = _shear_decay_3d(0, 1)
    ez, mz = _shear_decay_3d(2, 0)
    assert abs(ex) < 0.02 and abs(mx) < 1e-9
    assert abs(ex - ez) < 1e-9 and abs(mx - mz) < 1e-12
