"""Pins of the oracle's channel force controller (Sec. 4.3: a PI controller adjusts the
streamwise force to hold the mean momentum) on states whose momentum is known exactly.

On a fully periodic mesh a uniform state stays uniform, the collision keeps its momentum
and Kupershtokh's exact difference adds rho du = F dt per step, so the mean momentum
obeys m(n+1) = m(n) + F(n) dt exactly; the controller's law is then a scalar recursion
written out here on its own."""
import numpy as np
import pytest

import oracle
import workloads as W


def _periodic_box(p=2, n=2):
    mesh = W.TensorMesh(dim=3, p=p, nodes="gll", ncell=(n, n, n), edges=[np.array([0.0, 0.5, 1.3]),
                                                                          np.array([0.0, 0.7, 1.0]),
                                                                          np.array([-0.2, 0.3, 0.9])],
                        face_bc=[[-1, -1]] * 3, bcs=[])
    phys = W.Physics(dt=0.02, relax_mode=0, tau_bar=0.9)
    return mesh, phys


def _uniform(o, rho, u, T):
    return o.init(np.full(o.N, rho), np.tile(np.asarray(u, dtype=float), (o.N, 1)), np.full(o.N, T))


def test_update_on_a_uniform_state_is_the_closed_form():
    mesh, phys = _periodic_box()
    o = oracle.TensorOracle(mesh, phys)
    pop = _uniform(o, 1.1, (0.3, -0.1, 0.05), 0.9)
    c = oracle.ForceController(o, (0.01, 0.0, 0.002), axis=0, target=0.5, kp=2.0, ki=3.0)
    F = c.update(pop, dt=0.25)
    e = 0.5 - 1.1 * 0.3
    assert abs(c.mean - 0.33) < 1e-14
    assert abs(F[0] - (0.01 + 2.0 * e + 3.0 * e * 0.25)) < 1e-14
    assert F[1] == 0.0 and F[2] == 0.002
    # second update integrates again
    F = c.update(pop, dt=0.5)
    assert abs(F[0] - (0.01 + 2.0 * e + 3.0 * e * 0.75)) < 1e-14
    # other axes
    c2 = oracle.ForceController(o, (0.0, 0.0, 0.0), axis=2, target=0.0, kp=1.0, ki=0.0)
    assert abs(c2.update(pop, 1.0)[2] - (-1.1 * 0.05)) < 1e-14


def test_closed_loop_on_a_uniform_state_follows_the_scalar_recursion():
    mesh, phys = _periodic_box()
    o = oracle.TensorOracle(mesh, phys)
    rho, dt = 1.05, phys.dt
    pop = _uniform(o, rho, (0.1, 0.02, -0.03), 1.0)
    F0, target, kp, ki, every = 0.3, 0.4, 5.0, 20.0, 2
    c = oracle.ForceController(o, (F0, 0.0, 0.0), axis=0, target=target, kp=kp, ki=ki)
    m, I, F = rho * 0.1, 0.0, F0
    for n in range(24):
        if n % every == 0:
            c.update(pop, every * dt)
            e = target - m
            I += e * every * dt
            F = F0 + kp * e + ki * I
            assert abs(c.force[0] - F) < 1e-13 * max(1.0, abs(F)), n
        pop = o.step(pop)
        m += F * dt
        _, mom, _ = o.totals(pop)
        assert abs(mom[0] / np.sum(o.node_vol) - m) < 1e-13, n
    # the transverse momentum is untouched
    _, mom, _ = o.totals(pop)
    assert abs(mom[1] / np.sum(o.node_vol) - rho * 0.02) < 1e-13


def test_proportional_control_halves_the_error_each_step():
    """F0 = 0, ki = 0, kp = 1 / (2 dt): m(n+1) = m(n) + (target - m(n)) / 2."""
    mesh, phys = _periodic_box()
    o = oracle.TensorOracle(mesh, phys)
    pop = _uniform(o, 1.0, (0.0, 0.0, 0.0), 1.0)
    c = oracle.ForceController(o, (0.0, 0.0, 0.0), axis=0, target=0.2, kp=1.0 / (2 * phys.dt), ki=0.0)
    for n in range(8):
        c.update(pop, phys.dt)
        assert abs(c.error - 0.2 / 2 ** n) < 1e-13, n
        pop = o.step(pop)
