"""Pins of the oracle's viscosity law, body force and mixing-layer diagnostic against
closed-form flows.

* tau = mu/p (Sec. 3.1) read as the dimensionless tau_bar = mu(T)/(rho T dt) + 1/2 with
  mu = mu_ref (T/T_ref)^omega (relax mode 1): a linear shear wave decays at the kinematic
  viscosity mu(T)/rho, on states with rho != 1, T != T_ref and omega != 0, and the
  Taylor-Green vortex loses kinetic energy at the initial rate 2 nu |k|^2 = 6 nu.
* Kupershtokh's exact difference (Sec. 4.3 forcing display, applied to g as well): a forced
  uniform equilibrium stays an equilibrium, moved to u + F dt / rho, in f and g alike; on
  any state the added populations carry no mass, the momentum F dt, and the kinetic-energy
  change rho (|u + du|^2 - |u|^2); a forced channel between bounce-back walls reaches the
  Poiseuille profile u = F y (2 - y) / (2 mu) (Sec. 3.3.2 walls).
* The momentum thickness of the initial tanh profile (Sec. 4.4) equals delta_theta0.

Each physical pin is also run on oracles with a plausible mistake planted in a copy of the
oracle's C source (compiled into a temporary directory): the pin must fail there.
"""
import contextlib
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

ORACLE_C = os.path.join(os.path.dirname(oracle.__file__), "sllbm_oracle.c")


def gauss_moment(k, mean, var):
    """E[X^k] for X ~ N(mean, var), closed form."""
    def dfact(n):
        return 1 if n <= 0 else n * dfact(n - 2)
    return sum(math.comb(k, j) * mean ** (k - j) * var ** (j / 2) * dfact(j - 1) for j in range(0, k + 1, 2))


# ---------------------------------------------------------------- planted mistakes

MUTANTS = {
    # relax mode 1 without the trapezoidal shift 1/2
    "no_half": ("tb = mu / (rho * T * m->dt) + 0.5;", "tb = mu / (rho * T * m->dt);"),
    # p = rho instead of p = rho T in tau = mu / p
    "p_without_T": ("tb = mu / (rho * T * m->dt) + 0.5;", "tb = mu / (rho * m->dt) + 0.5;"),
    # the viscosity law's exponent applied to T_ref / T
    "exponent_inverted": ("double mu = m->mu_ref * pow(T / m->T_ref, m->mu_exp);",
                          "double mu = m->mu_ref * pow(m->T_ref / T, m->mu_exp);"),
    # the force term on g built from f^eq instead of g^eq
    "g_force_from_feq": ("fo[i] += fe2[i] - fe[i];\n      go[i] += gfac * (fe2[i] - fe[i]);\n    }\n  }\n  return",
                         "fo[i] += fe2[i] - fe[i];\n      go[i] += fe2[i] - fe[i];\n    }\n  }\n  return"),
    # du = F dt instead of F dt / rho
    "du_without_rho": ("u2[a] += m->force[a] * m->dt / rho;", "u2[a] += m->force[a] * m->dt;"),
}


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    src = open(ORACLE_C).read()
    d = tmp_path_factory.mktemp("oracle_mutants")
    libs = {}
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, f"planted mistake {name}: its target is not unique in the oracle source"
        c = d / f"{name}.c"
        c.write_text(src.replace(old, new))
        so = d / f"lib{name}.so"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", "-o", str(so), str(c), "-lm"])
        libs[name] = ctypes.CDLL(str(so))
    return libs


@contextlib.contextmanager
def planted(libs, name):
    """Run the oracle's Python front end on the mutant C core `name`."""
    saved = oracle._LIB
    oracle._LIB = libs[name]
    try:
        yield
    finally:
        oracle._LIB = saved


def fails(pin, *args):
    """True if the pin raises (its assertion, or the run going non-finite)."""
    try:
        with np.errstate(all="ignore"):
            pin(*args)
    except (AssertionError, FloatingPointError, oracle.OracleError):
        return True
    return False


# ---------------------------------------------------------------- relax mode 1

def shear_wave_mode1(rho0, T0, omega):
    """Shear wave u_y = A sin(x - U t) on a uniform state (rho0, T0) in relax mode 1 with
    mu_ref chosen so that mu(T0) = 0.4 rho0 T0 dt: the measured decay rate of the wave
    amplitude must be nu k^2 with nu = mu(T0) / rho0 (k = 1), within 1.5 %."""
    mesh, phys = W.shear_wave_case(ncell=16, p=4)
    phys.relax_mode, phys.mu_exp, phys.T_ref = 1, omega, 1.25
    mu = 0.4 * rho0 * T0 * phys.dt
    phys.mu_ref = mu / (T0 / phys.T_ref) ** omega
    o = oracle.TensorOracle(mesh, phys)
    xyz = o.coords()
    rho, u, T = W.shear_wave_fields(xyz, noise=0.0)
    pop = o.init(rho * rho0, u, T * T0)
    V = o.node_vol

    def amp(pp):
        _, uu, _ = o.moments(pp)
        s = np.sum(V * uu[:, 1] * np.sin(xyz[:, 0]))
        c = np.sum(V * uu[:, 1] * np.cos(xyz[:, 0]))
        return math.hypot(s, c)

    n = 100
    a0, a1 = amp(pop), amp(o.run(pop, n))
    assert np.isfinite(a1) and a1 > 0
    nu = -math.log(a1 / a0) / (n * phys.dt)
    nu_ref = mu / rho0
    assert abs(nu - nu_ref) < 0.015 * nu_ref, (nu, nu_ref)


@pytest.mark.parametrize("rho0,T0,omega", [(1.0, 1.25, 0.0), (1.2, 1.6, 0.7), (0.8, 0.8, 0.5)])
def test_relax_mode1_shear_wave_decays_at_mu_over_rho(rho0, T0, omega):
    shear_wave_mode1(rho0, T0, omega)


def tgv_initial_decay():
    """Taylor-Green vortex at Ma 0.05 on a uniform temperature T = 1.3 T_ref, relax mode 1
    with omega = 0.7: the kinetic energy sum_k V_k rho_k |u_k|^2 / 2 falls at the initial
    rate d ln E_k / dt = -2 nu |k|^2 = -6 nu, nu = mu(T) / <rho> (the vortex is
    divergence-free, so the dissipation is 2 mu S:S), within 2 %.  The rate is measured
    over steps 3 to 12, after the non-equilibrium stress has formed."""
    mesh, phys = W.tgv_case(ncell=8, p=3, Ma=0.05)
    phys.relax_mode, phys.mu_ref, phys.mu_exp, phys.T_ref = 1, 0.03, 0.7, 1.0
    Tu = 1.3
    o = oracle.TensorOracle(mesh, phys)
    rho, u, T = W.tgv_fields(o.coords(), Ma=0.05)
    pop = o.init(rho / Tu, u, np.full_like(T, Tu))
    V = o.node_vol

    def ek(pp):
        r, uu, _ = o.moments(pp)
        return 0.5 * np.sum(V * r * np.sum(uu ** 2, axis=1))

    E = []
    for n in range(13):
        if n >= 3:
            E.append(ek(pop))
        pop = o.step(pop)
    assert np.all(np.isfinite(E))
    rate = math.log(E[-1] / E[0]) / ((len(E) - 1) * phys.dt)
    nu = phys.mu_ref * Tu ** 0.7 / (np.sum(V * rho / Tu) / np.sum(V))
    assert abs(rate + 6.0 * nu) < 0.02 * 6.0 * nu, (rate, -6.0 * nu)


def test_tgv_initial_energy_decay_is_six_nu():
    tgv_initial_decay()


# ---------------------------------------------------------------- Kupershtokh forcing

def _periodic_2d(force, relax_mode=1):
    mesh = W.TensorMesh(dim=2, p=3, nodes="gll", ncell=(3, 2), edges=[np.array([0.0, 0.4, 0.9, 1.2]),
                                                                      np.array([-0.5, 0.1, 0.6])],
                        face_bc=[[-1, -1], [-1, -1]], bcs=[])
    phys = W.Physics(dt=0.03, relax_mode=relax_mode, tau_bar=0.9, mu_ref=0.02, T_ref=1.0, mu_exp=0.7,
                     force=tuple(force) + (0.0,))
    return mesh, phys


def forced_uniform_equilibrium():
    """A uniform equilibrium (rho, u, T) is a fixed point of streaming and collision, so one
    forced step must return the equilibrium at (rho, u + F dt / rho, T) for f and for g:
    every population to round-off, and the raw moments sum_i zeta^m f_i (|m| <= 4) and
    sum_i zeta^m g_i (|m| <= 3) equal those of a Gaussian of mean u + F dt / rho and
    variance T, times rho and rho T (2 c_v - D)."""
    rho, u, T, F = 1.1, np.array([0.2, -0.1]), 0.9, np.array([0.3, 0.1])
    mesh, phys = _periodic_2d(F)
    o = oracle.TensorOracle(mesh, phys)
    N = o.N
    pop = o.init(np.full(N, rho), np.tile(u, (N, 1)), np.full(N, T))
    out = o.step(pop)
    u1 = u + F * phys.dt / rho
    want = o.init(np.full(N, rho), np.tile(u1, (N, 1)), np.full(N, T))
    assert np.max(np.abs(out - want)) < 1e-14
    Q = o.Q
    f, g = out[:Q * N].reshape(Q, N)[:, 0], out[Q * N:].reshape(Q, N)[:, 0]
    cv = 1.0 / (phys.gamma - 1.0)
    for a in range(5):
        for b in range(5 - a):
            zm = o.zeta[:, 0] ** a * o.zeta[:, 1] ** b
            gm = gauss_moment(a, u1[0], T) * gauss_moment(b, u1[1], T)
            assert abs(np.sum(zm * f) - rho * gm) < 1e-13, (a, b)
            if a + b <= 3:
                assert abs(np.sum(zm * g) - rho * T * (2 * cv - 2) * gm) < 1e-13, (a, b)


def test_forced_uniform_equilibrium_moves_to_u_plus_du():
    forced_uniform_equilibrium()


def test_force_term_mass_momentum_energy_on_a_random_state():
    """On a non-uniform state the forced and unforced steps differ by delta h = h^eq(u + du)
    - h^eq(u) at every node: sum delta f = 0, sum zeta delta f = F dt, sum delta g = 0 and
    sum (|zeta|^2 delta f + delta g) = rho (|u + du|^2 - |u|^2), with rho, u the moments of
    the streamed state (the collision keeps them)."""
    F = np.array([0.7, -0.4])
    mesh, phys = _periodic_2d(F)
    o_f = oracle.TensorOracle(mesh, phys)
    import copy
    ph0 = copy.copy(phys)
    ph0.force = (0.0, 0.0, 0.0)
    o_0 = oracle.TensorOracle(mesh, ph0)
    ph2 = copy.copy(ph0)
    ph2.relax_mode = 2
    o_s = oracle.TensorOracle(mesh, ph2)
    N, Q = o_f.N, o_f.Q
    rho, u, T = W.random_fields(N, 2, seed=21, rho_amp=0.1, u_amp=0.3, T_amp=0.1)
    rng = np.random.Generator(np.random.PCG64(22))
    pop = o_f.init(rho, u, T) * (1 + 0.02 * rng.uniform(-1, 1, 2 * Q * N))
    d = o_f.step(pop) - o_0.step(pop)
    r, us, _ = o_s.moments(o_s.step(pop))
    df, dg = d[:Q * N].reshape(Q, N), d[Q * N:].reshape(Q, N)
    z2 = np.sum(o_f.zeta ** 2, axis=1)[:, None]
    du = F[None, :] * phys.dt / r[:, None]
    assert np.max(np.abs(df.sum(0))) < 1e-14
    assert np.max(np.abs(dg.sum(0))) < 1e-14
    for a in range(2):
        assert np.max(np.abs((o_f.zeta[:, a:a + 1] * df).sum(0) - F[a] * phys.dt)) < 1e-14
    dE = r * (np.sum((us + du) ** 2, axis=1) - np.sum(us ** 2, axis=1))
    assert np.max(np.abs((z2 * df).sum(0) + dg.sum(0) - dE)) < 1e-14
    assert np.max(np.abs(dE)) > 1e-3


def poiseuille():
    """A channel between isothermal bounce-back walls at y = 0 and 2 (T_w = 1), periodic in
    x, rho = 1.3 at rest, driven by a uniform force F per unit volume: after 4000 steps
    (9.5 e-folds of the slowest mode) u_x = F y (2 - y) / (2 mu) within 1 % of its peak
    (Ma 0.04; relax mode 1 at tau_bar = 1)."""
    ny, p, rho0 = 8, 4, 1.3
    mesh = W.TensorMesh(dim=2, p=p, nodes="gll", ncell=(1, ny), edges=[W.uniform_edges(1, 0.0, 0.5),
                                                                       W.uniform_edges(ny, 0.0, 2.0)],
                        face_bc=[[-1, -1], [0, 0]], bcs=[W.BC(kind=W.BC_WALL, T_wall=1.0)])
    dt = 0.5 * (2.0 / ny) / W.ZETA_MAX_GH5
    mu = 0.5 * rho0 * dt
    F = 0.1 * mu
    phys = W.Physics(dt=dt, relax_mode=1, mu_ref=mu, T_ref=1.0, mu_exp=0.0, force=(F, 0.0, 0.0))
    o = oracle.TensorOracle(mesh, phys)
    y = o.coords()[:, 1]
    pop = o.init(np.full(o.N, rho0), np.zeros((o.N, 2)), np.ones(o.N))
    pop = o.run(pop, 4000)
    _, u, _ = o.moments(pop)
    exact = F * y * (2.0 - y) / (2.0 * mu)
    assert np.all(np.isfinite(u))
    assert np.max(np.abs(u[:, 0] - exact)) < 0.01 * np.max(exact), np.max(np.abs(u[:, 0] - exact)) / np.max(exact)
    assert np.max(np.abs(u[:, 1])) < 1e-3 * np.max(exact)


def test_poiseuille_profile_between_bounce_back_walls():
    poiseuille()


# ---------------------------------------------------------------- the pins have teeth

@pytest.mark.parametrize("mutant,pin,args", [
    ("no_half", shear_wave_mode1, (1.2, 1.6, 0.7)),
    ("p_without_T", shear_wave_mode1, (1.2, 1.6, 0.7)),
    ("exponent_inverted", shear_wave_mode1, (1.2, 1.6, 0.7)),
    ("p_without_T", tgv_initial_decay, ()),
    ("g_force_from_feq", forced_uniform_equilibrium, ()),
    ("du_without_rho", forced_uniform_equilibrium, ()),
    ("du_without_rho", poiseuille, ()),
])
def test_pin_fails_on_planted_mistake(mutant_libs, mutant, pin, args):
    with planted(mutant_libs, mutant):
        assert fails(pin, *args), f"{pin.__name__} passes with the planted mistake {mutant}"


# ---------------------------------------------------------------- mixing-layer diagnostic

def _layer_mesh(ny=128, half=20.0, rho_scale=1.0):
    d0 = W.MIX_DTHETA0
    mesh = W.TensorMesh(dim=3, p=2, nodes="gll", ncell=(2, ny, 2),
                        edges=[W.uniform_edges(2, 0.0, 4 * d0), W.uniform_edges(ny, -half * d0, half * d0),
                               W.uniform_edges(2, 0.0, 3 * d0)],
                        face_bc=[[-1, -1], [0, 0], [-1, -1]], bcs=[W.BC(kind=W.BC_INLET)])
    return mesh


def test_momentum_thickness_of_the_initial_profile():
    """u_x = (du/2) tanh(y / (2 delta_theta0)) on [-L, L]: delta_theta = delta_theta0
    tanh(L / (2 delta_theta0)) (closed form of the integral of sech^2 / 4); scaling rho by
    1.4 scales it by 1.4; a velocity perturbation with zero plane mean at rho = 1 leaves it
    unchanged up to its own second moment, which the Favre average keeps."""
    import torch
    from paper_2412_09051_amd import diagnostics as D
    import paper_2412_09051_amd as S
    d0, half = W.MIX_DTHETA0, 20.0
    mesh = _layer_mesh(half=half)
    m = S.sllbm_mesh_build(mesh)
    xyz, V = S.sllbm_mesh_nodes(m), S.sllbm_mesh_volumes(m)
    o = oracle.TensorOracle(mesh, W.Physics(dt=0.01))
    assert np.max(np.abs(V - o.node_vol)) < 1e-14
    shape = (mesh.axis_nodes(2), mesh.axis_nodes(1), mesh.axis_nodes(0))
    du = 2.0 * 0.7 * math.sqrt(1.4)
    area = (4 * d0) * (3 * d0)
    ux = 0.5 * du * np.tanh(xyz[:, 1] / (2.0 * d0))
    want = d0 * math.tanh(half / 2.0)
    Vt = torch.tensor(V).view(shape)
    got = D.momentum_thickness(torch.ones(shape, dtype=torch.float64), torch.tensor(ux).view(shape), Vt, du, area)
    assert abs(got - want) < 1e-5 * want, (got, want)
    got14 = D.momentum_thickness(torch.full(shape, 1.4, dtype=torch.float64), torch.tensor(ux).view(shape), Vt, du, area)
    assert abs(got14 - 1.4 * want) < 1e-5 * want
    # numpy arrays give the same number
    assert abs(D.momentum_thickness(np.ones(shape), ux.reshape(shape), V.reshape(shape), du, area) - got) < 1e-15
    # a perturbation u' = a cos(2 pi x / Lx) (zero mean on every node plane) leaves the plane means
    # and so delta_theta unchanged
    up = ux + 0.1 * du * np.cos(2 * math.pi * xyz[:, 0] / (4 * d0)) * np.exp(-(xyz[:, 1] / d0) ** 2)
    gotp = D.momentum_thickness(np.ones(shape), up.reshape(shape), V.reshape(shape), du, area)
    assert abs(gotp - got) < 1e-12 * want
    # growth rate over a window: least squares of a straight line is exact
    tau = np.arange(0.0, 1000.0, 25.0)
    th = 0.2 + 0.0155 * tau
    assert abs(D.window_rate(tau, th, (450.0, 700.0)) - 0.0155) < 1e-12
    assert D.window_rate(tau, th, (451.0, 460.0)) is None
