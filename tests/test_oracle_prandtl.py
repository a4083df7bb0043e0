"""Pins of the oracle's Prandtl-number term (Sec. 3.1 update display: h gains
(1/tau - 1/tau_Pr) h*, tau_Pr = (tau - 1/2)/Pr + 1/2; h* is a reading, since the paper
defers it to its references: the lowest-order Hermite terms carrying the heat flux).

What fixes it independently of that reading: the collision must conserve rho, j, E, relax
the non-equilibrium stress with tau and the heat flux with tau_Pr (moment by moment on one
step), and the flow must show the Prandtl number: a thermal wave at uniform pressure decays
at nu k^2 / Pr while a shear wave keeps nu k^2.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _moments(zeta, f, g):
    rho = f.sum(0)
    u = (zeta.T @ f) / rho
    return rho, u


def _flux_and_stress(zeta, f, g, u):
    """Per node: heat flux q = 1/2 sum c (|c|^2 f + g) and the central stress sum c c f."""
    c = zeta[:, :, None] - u[None, :, :]            # [Q][D][N]
    c2 = np.sum(c * c, axis=1)                      # [Q][N]
    q = 0.5 * np.sum(c * (c2 * f)[:, None, :] + c * g[:, None, :], axis=0)
    P = np.einsum("iak,ibk,ik->abk", c, c, f)
    return q, P


@pytest.mark.parametrize("Pr", [0.71, 2.0])
def test_collision_relaxes_heat_flux_with_tau_pr_and_stress_with_tau(Pr):
    mesh, phys = W.shear_wave_case(ncell=4, p=4)
    tb = 0.9
    streamed = dataclasses.replace(phys, relax_mode=2)
    collided = dataclasses.replace(phys, relax_mode=0, tau_bar=tb, Pr=Pr)
    o_s, o_c = oracle.TensorOracle(mesh, streamed), oracle.TensorOracle(mesh, collided)
    rng = np.random.Generator(np.random.PCG64(21))
    rho, u, T = W.random_fields(o_s.N, 2, seed=22)
    pop = o_s.init(rho, u, T) * (1 + 0.05 * rng.uniform(-1, 1, 2 * o_s.Q * o_s.N))
    a, b = o_s.step(pop).reshape(2, o_s.Q, o_s.N), o_c.step(pop).reshape(2, o_s.Q, o_s.N)
    zeta = o_s.zeta
    ra, ua = _moments(zeta, a[0], a[1])
    rb, ub = _moments(zeta, b[0], b[1])
    Ta, Tb = o_s.moments(a.ravel())[2], o_c.moments(b.ravel())[2]
    assert np.max(np.abs(ra - rb)) < 1e-14 and np.max(np.abs(ua - ub)) < 1e-13 and np.max(np.abs(Ta - Tb)) < 1e-13
    qa, Pa = _flux_and_stress(zeta, a[0], a[1], ua)
    qb, Pb = _flux_and_stress(zeta, b[0], b[1], ub)
    # the equilibria carry no heat flux and the stress rho T I
    Peq = ra * Ta
    tpr = (tb - 0.5) / Pr + 0.5
    assert np.max(np.abs(qb - (1 - 1 / tpr) * qa)) < 1e-12 * np.max(np.abs(qa))
    for al in range(2):
        for be in range(2):
            na = Pa[al, be] - (Peq if al == be else 0.0)
            nb = Pb[al, be] - (Peq if al == be else 0.0)
            assert np.max(np.abs(nb - (1 - 1 / tb) * na)) < 1e-11 * np.max(np.abs(Pa[al, be]))
    # teeth: the heat flux is not relaxed with tau
    assert np.max(np.abs(qb - (1 - 1 / tb) * qa)) > 1e-3 * np.max(np.abs(qa))


def _decay(Pr, wave, vel=None, tau=1.3, n=200):
    """Decay rate of a thermal wave (T = 1 + 0.01 sin x at uniform pressure) or of the
    shear wave, divided by nu k^2 with nu = (tau - 1/2) T0 dt and k = 1."""
    mesh, phys = W.shear_wave_case(ncell=16, p=4, tau_bar=tau)
    phys = dataclasses.replace(phys, Pr=Pr)
    o = oracle.TensorOracle(mesh, phys, vel=vel)
    x = o.coords()
    if wave == "thermal":
        T = 1 + 0.01 * np.sin(x[:, 0])
        pop = o.init(1 / T, np.zeros((o.N, 2)), T)
        field = lambda pp: o.moments(pp)[2] - 1
    else:
        rho, u, T = W.shear_wave_fields(x, noise=0.0)
        pop = o.init(rho, u, T)
        field = lambda pp: o.moments(pp)[1][:, 1]
    V = o.node_vol

    def amp(pp):
        q = field(pp)
        return math.hypot(np.sum(V * q * np.sin(x[:, 0])), np.sum(V * q * np.cos(x[:, 0])))

    a0 = amp(pop)
    a1 = amp(o.run(pop, n))
    return -math.log(a1 / a0) / (n * phys.dt) / ((tau - 0.5) * phys.T0 * phys.dt)


def test_thermal_wave_decays_at_nu_over_pr():
    r1 = _decay(1.0, "thermal")
    assert abs(r1 - 1.0) < 0.03          # Pr = 1: thermal diffusivity equals nu
    for Pr in (0.71, 2.0):
        r = _decay(Pr, "thermal")
        assert abs(r / r1 * Pr - 1.0) < 0.02, (Pr, r / r1)


def test_thermal_wave_decay_on_d2q19():
    vel = oracle.cubature_set(2)
    r1 = _decay(1.0, "thermal", vel=vel)
    r = _decay(0.71, "thermal", vel=vel)
    assert abs(r1 - 1.0) < 0.03 and abs(r / r1 * 0.71 - 1.0) < 0.02


def test_shear_wave_keeps_nu_at_other_pr():
    s1, s = _decay(1.0, "shear", n=100), _decay(0.71, "shear", n=100)
    assert abs(s1 - 1.0) < 0.02 and abs(s - s1) < 2e-3 * s1
