"""Pins of the learned-correction oracle (oracle/learned.py) against independent facts:
torch's own BF16 conversion, finite differences of the loss, closed forms of the
network and of Adam's first step, exact derivatives of polynomial fields, the algebra of
the projection, and the coordinates of nested meshes."""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.learned as L
import workloads as W


def test_bf16_rounding_matches_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.normal(0, 3, 20000), rng.uniform(-1e-3, 1e-3, 2000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0, 1.0 + 2 ** -9]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(L.bf16(x), ref)
    assert np.array_equal(L.from_bf16_bits(L.bf16_bits(x)), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert L.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert L.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def _random_params(n_in, n_out, seed, scale=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.uniform(-scale, scale, s) for s in L.param_shapes(n_in, n_out)]


def test_backward_matches_finite_differences():
    n_in, n_out, rows = 7, 9, 13
    params = _random_params(n_in, n_out, 2)
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.uniform(-1, 1, (rows, n_in))
    t = rng.uniform(-1, 1, (rows, n_out))
    loss, grads, _ = L.loss_and_grad(params, x, t, emulate=False)
    h = 1e-6
    for k, pk in enumerate(params):
        flat = pk.reshape(-1)
        for idx in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = L.loss_and_grad(params, x, t, emulate=False)[0]
            flat[idx] = old - h
            lm = L.loss_and_grad(params, x, t, emulate=False)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-7 + 1e-6 * abs(fd), (k, idx, fd, an)


def test_forward_closed_form():
    """A single path through the network: y_o = b4_o + W4[0, o] tanh(a3 tanh(a2 tanh(a1 x_0 + c1)))."""
    n_in, n_out = 5, 4
    params = [np.zeros(s) for s in L.param_shapes(n_in, n_out)]
    a1, a2, a3, c1 = 0.75, -1.25, 0.5, 0.125
    params[0][0, 0] = a1
    params[1][0] = c1
    params[2][0, 0] = a2
    params[4][0, 0] = a3
    params[6][0, :] = [1.0, -0.5, 0.25, 2.0]
    params[7][:] = [0.0, 0.5, -0.25, 1.0]
    x = np.array([[0.375, 9.0, 9.0, 9.0, 9.0], [-1.5, 0, 0, 0, 0]])
    y, _ = L.forward(params, x, emulate=False)
    for r in range(2):
        h = math.tanh(a3 * math.tanh(a2 * math.tanh(a1 * x[r, 0] + c1)))
        assert np.allclose(y[r], params[7] + params[6][0] * h, rtol=0, atol=1e-15)
    # rounding: BF16-representable inputs and weights give the same values with emulation
    y2, _ = L.forward(params, L.bf16(x), emulate=True)
    h = np.tanh(a3 * L.bf16(np.tanh(a2 * L.bf16(np.tanh(a1 * x[:, 0] + c1)))))
    assert np.allclose(y2, params[7][None, :] + L.bf16(h)[:, None] * params[6][0][None, :], atol=1e-15)


def test_adam_first_step_closed_form():
    """After one step m_hat = g, v_hat = g^2: theta moves by -lr g / (|g| + eps)."""
    g = [np.array([0.3, -2.0, 1e-3]), np.array([[5.0]])]
    th = [np.array([1.0, 2.0, 3.0]), np.array([[0.5]])]
    m = [np.zeros_like(a) for a in g]
    v = [np.zeros_like(a) for a in g]
    th0 = [a.copy() for a in th]
    L.adam_step(th, g, m, v, 1, lr=0.01)
    for a, a0, gg in zip(th, th0, g):
        assert np.allclose(a, a0 - 0.01 * gg / (np.abs(gg) + 1e-8), rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_projector_algebra(dim):
    zeta, w, _ = oracle.velocity_set(dim, 5, 1.0)
    P = L.projector(zeta, w)
    M = L.invariants(zeta)
    assert np.max(np.abs(M @ P)) < 1e-12                      # invariants untouched
    assert np.max(np.abs(P @ P - P)) < 1e-12                  # a projection
    Winv = 1.0 / np.concatenate([w, w])
    # orthogonal in <a, b> = sum a b / w: P is self-adjoint there
    S = P.T * Winv[None, :]
    assert np.max(np.abs(S - S.T)) / np.max(np.abs(S)) < 1e-10
    # what it removes is W M^T c
    c = np.arange(1.0, dim + 3)
    assert np.max(np.abs(P @ (np.concatenate([w, w]) * (M.T @ c)))) < 1e-12


def _poly_mesh(dim):
    edges = [np.array([0.0, 0.4, 1.1, 1.5]), np.array([-0.5, 0.1, 0.6]), np.array([0.0, 0.7, 1.2])]
    n = (3, 2, 2)[:dim]
    return W.TensorMesh(dim=dim, p=2, nodes="gll", ncell=n, edges=edges[:dim],
                        face_bc=[[0, 0]] * dim, bcs=[W.BC(kind=W.BC_WALL)])


@pytest.mark.parametrize("dim", [2, 3])
def test_features_are_exact_for_quadratic_fields(dim):
    """Fields quadratic per axis: the interpolant's derivative is exact, so the features
    are h times the analytic gradient (the two cells at an interface agree)."""
    mesh = _poly_mesh(dim)
    phys = W.Physics(dt=0.01)
    o = oracle.TensorOracle(mesh, phys)
    xyz = o.coords()
    X = [xyz[:, a] for a in range(dim)]
    rho = 1.0 + 0.05 * X[0] + 0.03 * X[1] ** 2
    u = np.stack([0.1 * X[1] - 0.02 * X[0] ** 2] + [0.05 * X[0] * X[1]] + ([0.04 * X[2]] if dim == 3 else []), axis=1)
    T = 1.0 + 0.02 * X[0] - 0.01 * X[dim - 1] ** 2
    pop = o.init(rho, u, T)
    F = L.features(mesh, o.zeta, phys.gamma, pop)
    assert F.shape == (o.N, 5 + 5 * dim if dim == 3 else 4 + 4 * dim)
    nf = dim + 2
    grads = {  # analytic gradient of each field, per axis
        0: [0.05 + 0 * X[0], 0.06 * X[1]] + ([0 * X[0]] if dim == 3 else []),
        1: [-0.04 * X[0], 0.1 + 0 * X[0]] + ([0 * X[0]] if dim == 3 else []),
        2: [0.05 * X[1], 0.05 * X[0]] + ([0 * X[0]] if dim == 3 else []),
    }
    if dim == 3:
        grads[3] = [0 * X[0], 0 * X[0], 0.04 + 0 * X[0]]
    grads[nf - 1] = [0.02 + 0 * X[0]] + [0 * X[0]] * (dim - 2) + [-0.02 * X[dim - 1]]
    if dim == 2:
        grads[nf - 1] = [0.02 - 0 * X[0], -0.02 * X[1]]
    # mean cell length per node and axis
    for q in range(nf):
        for a in range(dim):
            col = nf + q * dim + a
            e = np.asarray(mesh.edges[a])
            lens = np.diff(e)
            h = np.empty(o.N)
            for k in range(o.N):
                xa = X[a][k]
                inside = [lens[c] for c in range(len(lens)) if e[c] - 1e-12 <= xa <= e[c + 1] + 1e-12]
                h[k] = np.mean(inside)
            assert np.max(np.abs(F[:, col] - h * grads[q][a])) < 1e-12, (q, a)
    assert np.max(np.abs(F[:, 0] - (rho - 1))) < 1e-13
    assert np.max(np.abs(F[:, nf - 1] - (T - 1))) < 1e-13


def test_correction_keeps_invariants_and_targets_invert_it():
    """correct() changes no moment of a node; a network that outputs the target of a node
    reaches the true populations up to what the projection removes."""
    mesh, phys = W.mixing_layer_case(ncell=(3, 3, 3), box=(1.0, 1.2, 0.8))
    o = oracle.TensorOracle(mesh, phys)
    rho, u, T = W.mixing_layer_fields(o.coords(), box=(1.0, 1.2, 0.8), amp=0.2)
    pop = o.init(rho, u, T)
    n_in, n_out = 20, 2 * o.Q
    params = _random_params(n_in, n_out, 5, scale=0.3)
    out = L.correct(mesh, o.zeta, o.w, phys.gamma, pop, params)
    M = L.invariants(o.zeta)
    before = M @ pop.reshape(2 * o.Q, o.N)
    after = M @ out.reshape(2 * o.Q, o.N)
    assert np.max(np.abs(after - before)) < 1e-13 * np.max(np.abs(before))
    assert np.max(np.abs(out - pop)) > 1e-4
    # targets: y = t exactly gives plain + P (true - plain)
    pop_true = o.step(pop)
    import dataclasses
    o2 = oracle.TensorOracle(mesh, dataclasses.replace(phys, dt=1.3 * phys.dt))
    plain = o2.step(pop)
    assert np.max(np.abs(plain - pop_true)) > 1e-6
    t = L.targets(o.zeta, o.w, plain, pop_true)
    rho_p = plain[: o.Q * o.N].reshape(o.Q, o.N).sum(axis=0)
    scale = np.concatenate([o.w, o.w])[None, :] * rho_p[:, None]
    P = L.projector(o.zeta, o.w)
    fixed = plain + ((scale * t) @ P.T).T.reshape(-1)
    resid = (pop_true - fixed).reshape(2 * o.Q, o.N).T
    assert np.max(np.abs(resid @ P.T)) < 1e-13


def test_restriction_is_injection_on_nested_meshes():
    box = (1.0, 1.2, 0.8)
    mc, pc = W.mixing_layer_case(ncell=(3, 2, 2), box=box)
    mf, pf = W.mixing_layer_case(ncell=(3, 2, 2), refine=2, box=box)
    oc, of = oracle.TensorOracle(mc, pc), oracle.TensorOracle(mf, pf)
    # restricting the coordinates themselves (as a 2Q-population field) gives the coarse ones
    xf = of.coords()
    Q = 1
    for a in range(3):
        fld = np.concatenate([xf[:, a], xf[:, a]])
        got = L.restrict(mf, mc, 2, fld, Q)[: oc.N]
        assert np.max(np.abs(got - oc.coords()[:, a])) < 1e-14
    assert abs(pf.dt * 2 - pc.dt) < 1e-15
