"""The device-side force controller (Sec. 4.3) against the oracle's controller: the
closed form on a uniform state, and a controlled channel run with isothermal walls,
temperature-dependent viscosity and forcing, on both step kernels."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from harness import GpuRun, rel_err

pytestmark = pytest.mark.gpu

GATHER, TILED = 1, 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _periodic_box():
    mesh = W.TensorMesh(dim=3, p=2, nodes="gll", ncell=(2, 2, 2), edges=[np.array([0.0, 0.5, 1.3]),
                                                                          np.array([0.0, 0.7, 1.0]),
                                                                          np.array([-0.2, 0.3, 0.9])],
                        face_bc=[[-1, -1]] * 3, bcs=[])
    return mesh, W.Physics(dt=0.02, relax_mode=0, tau_bar=0.9)


def test_update_on_a_uniform_state_is_the_closed_form():
    say("case force update uniform")
    mesh, phys = _periodic_box()
    g = GpuRun(mesh, phys, "f64")
    S = g.S
    g.init(np.full(g.N, 1.1), np.tile([0.3, -0.1, 0.05], (g.N, 1)), np.full(g.N, 0.9))
    S.sllbm_force_reset(g.plan, (0.01, 0.0, 0.002))
    S.sllbm_force_update(g.plan, g.a, axis=0, target=0.5, kp=2.0, ki=3.0, dt=0.25)
    st = S.sllbm_force_read(g.plan)
    e = 0.5 - 1.1 * 0.3
    say(st)
    assert abs(st["mean_momentum"] - 0.33) < 1e-14
    assert abs(st["error"] - e) < 1e-14 and abs(st["integral"] - 0.25 * e) < 1e-14
    assert abs(st["force"][0] - (0.01 + 2.0 * e + 0.75 * e)) < 1e-14
    assert st["force"][1] == 0.0 and st["force"][2] == 0.002 and st["updates"] == 1
    S.sllbm_force_update(g.plan, g.a, axis=0, target=0.5, kp=2.0, ki=3.0, dt=0.5)
    st = S.sllbm_force_read(g.plan)
    assert abs(st["force"][0] - (0.01 + 2.0 * e + 3.0 * 0.75 * e)) < 1e-14 and st["updates"] == 2
    # a reset clears the integral
    S.sllbm_force_reset(g.plan, (0.0, 0.0, 0.0))
    st = S.sllbm_force_read(g.plan)
    assert st["integral"] == 0.0 and st["updates"] == 0 and not np.any(st["force"])


@pytest.mark.parametrize("kernel", [pytest.param(GATHER, id="gather"), pytest.param(TILED, id="tiled")])
def test_controlled_channel_matches_the_oracle(kernel):
    """12 steps of a small channel with the controller updated every 3 steps: the force
    history and the final populations agree to 1e-12 relative."""
    say("case controlled channel", kernel)
    mesh, phys = W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.9, T_wall=0.9, Ma_b=0.5)
    ctl = W.channel_controller(Ma_b=0.5, T_wall=0.9, tau_c=0.05)
    ctl["target"] *= 1.2          # away from the initial state, so the force moves
    o = oracle.TensorOracle(mesh, phys)
    g = GpuRun(mesh, phys, "f64", kernel)
    say("kernel in use", g.kernel)
    rho, u, T = W.channel_fields(o.coords(), box=(2.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0)
    pop = o.init(rho, u, T)
    g.init(rho, u, T)
    S = g.S
    c = oracle.ForceController(o, phys.force, **ctl)
    S.sllbm_force_reset(g.plan, phys.force)
    prm = dataclasses.replace(g.prm, force_device=1)
    every = 3
    for n in range(12):
        if n % every == 0:
            F = c.update(pop, every * phys.dt)
            S.sllbm_force_update(g.plan, g.a, dt=every * phys.dt, **ctl)
            st = S.sllbm_force_read(g.plan)
            say(n, "force", F[0], st["force"][0])
            # the controller multiplies the mean momentum's error (1e-12 relative) by its gains
            scale = abs(phys.force[0]) + ctl["kp"] * abs(ctl["target"]) + ctl["ki"] * abs(c.integral)
            assert abs(st["force"][0] - F[0]) <= 1e-12 * scale, (n, st["force"][0], F[0])
            assert abs(st["mean_momentum"] - c.mean) <= 1e-12 * abs(c.mean)
        pop = o.step(pop)
        S.sllbm_step(g.plan, prm, g.a, g.b)
        g.a, g.b = g.b, g.a
    g.torch.cuda.synchronize()
    assert abs(c.force[0] - phys.force[0]) > 1e-3 * abs(phys.force[0])     # the controller acted
    e = rel_err(g.pop(), pop)
    say("pop error", e)
    assert e <= 1e-12


def test_force_device_fp32_follows_the_fp64_force():
    """FP32 storage: the controlled force stays within 1e-5 (relative to the force scale)
    of the FP64 oracle's over 12 steps."""
    say("case controlled channel fp32")
    mesh, phys = W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.9, T_wall=0.9, Ma_b=0.5)
    ctl = W.channel_controller(Ma_b=0.5, T_wall=0.9, tau_c=0.05)
    ctl["target"] *= 1.2
    o = oracle.TensorOracle(mesh, phys)
    g = GpuRun(mesh, phys, "f32")
    rho, u, T = W.channel_fields(o.coords(), box=(2.0, 2.0, 1.5), Ma_b=0.5, T_wall=1.0)
    pop = o.init(rho, u, T)
    g.init(rho, u, T)
    S = g.S
    c = oracle.ForceController(o, phys.force, **ctl)
    S.sllbm_force_reset(g.plan, phys.force)
    prm = dataclasses.replace(g.prm, force_device=1)
    scale = abs(phys.force[0]) + ctl["kp"] * ctl["target"]
    for n in range(12):
        if n % 3 == 0:
            F = c.update(pop, 3 * phys.dt)
            S.sllbm_force_update(g.plan, g.a, dt=3 * phys.dt, **ctl)
            st = S.sllbm_force_read(g.plan)
            assert abs(st["force"][0] - F[0]) <= 1e-5 * scale, (n, st["force"][0], F[0])
        pop = o.step(pop)
        S.sllbm_step(g.plan, prm, g.a, g.b)
        g.a, g.b = g.b, g.a
    g.torch.cuda.synchronize()
