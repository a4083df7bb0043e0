"""Oracle of the learned post-collision correction (plain numpy, FP64).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU baseline may
import this module.  It shares no code with the HIP library.

What it computes, in the order of the method:

* features of a node: its moments rho, u, T and their gradients, the derivative of
  the cell's Lagrange interpolant (eq:intf) along each axis at the node, averaged over
  the cells that share the node on that axis;
* the network: three tanh layers of width 64 and a linear output of 2Q values, with
  the matrix-product inputs rounded to BF16 (round to nearest even, through FP32) where
  the GPU rounds them, so that both sides multiply the same numbers;
* the correction of a node's post-collision populations: the network output times
  w_i rho, projected off the collision invariants (mass, momentum, total energy) in the
  inner product weighted by 1/w_i, and added;
* training: one-step targets (the restricted fine solution minus the plain coarse step,
  projected and divided by w_i rho), mean-square loss, its gradient by the chain rule,
  and one Adam step;
* restriction of a fine population field to a nested coarse mesh by injection.
"""
from __future__ import annotations

import numpy as np

from . import support_points

WIDTH = 64
DEPTH = 3


# --------------------------------------------------------------------------
# BF16 rounding (round to nearest even), reached through FP32 as on the GPU
# --------------------------------------------------------------------------

def bf16(x):
    """Round to the nearest BF16 value (ties to even), after rounding to FP32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def bf16_bits(x):
    """The 16-bit patterns of bf16(x)."""
    v = bf16(x).astype(np.float32)
    return (np.ascontiguousarray(v).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    b = np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------

def _diff_matrix(xr):
    """D[j, m] = l_m'(x_j): derivative of the m-th Lagrange basis function of the
    support points xr at support point j."""
    n = len(xr)
    D = np.zeros((n, n))
    for j in range(n):
        for m in range(n):
            if m == j:
                D[j, j] = sum(1.0 / (xr[j] - xr[q]) for q in range(n) if q != j)
            else:
                v = 1.0 / (xr[m] - xr[j])
                for q in range(n):
                    if q != m and q != j:
                        v *= (xr[j] - xr[q]) / (xr[m] - xr[q])
                D[j, m] = v
    return D


def _axis_derivative(mesh, a, q_line):
    """d/dx_a of a field along axis-a lines (q_line[..., n] over the axis's nodes): per
    cell the derivative of its interpolant at its support points, averaged over the
    cells that share a node.  Also returns the mean cell length h per node."""
    p = mesh.p
    nc = mesh.ncell[a]
    edges = np.asarray(mesh.edges[a], dtype=np.float64)
    periodic = mesh.face_bc[a][0] < 0
    Na = nc * p if periodic else nc * p + 1
    D = _diff_matrix(support_points(p, mesh.nodes))
    acc = np.zeros(q_line.shape)
    cnt = np.zeros(Na)
    hsum = np.zeros(Na)
    for c in range(nc):
        h = edges[c + 1] - edges[c]
        idx = [(c * p + j) % Na for j in range(p + 1)]
        vals = q_line[..., idx]                                   # [..., p+1]
        der = np.einsum("jm,...m->...j", D, vals) * (2.0 / h)
        for j in range(p + 1):
            acc[..., idx[j]] += der[..., j]
            cnt[idx[j]] += 1
            hsum[idx[j]] += h
    return acc / cnt, hsum / cnt


def features(mesh, zeta, gamma, pop, T0=1.0):
    """[N, 5 + 5 D] (3D: 20) node features of a population field on a tensor-product
    mesh, FP64 before rounding: rho - 1, u / sqrt(T0), T / T0 - 1, then for each of
    those five fields and each axis a, h_a d/dx_a of it (h_a the mean length of the cells
    along a that share the node)."""
    D = mesh.dim
    Q = zeta.shape[0]
    cv = 1.0 / (gamma - 1.0)
    N = pop.size // (2 * Q)
    f = pop[: Q * N].reshape(Q, N)
    g = pop[Q * N:].reshape(Q, N)
    rho = f.sum(axis=0)
    j = zeta.T @ f                                                # [D, N]
    E = (zeta ** 2).sum(axis=1) @ f + g.sum(axis=0)
    u = j / rho
    T = (E - rho * (u ** 2).sum(axis=0)) / (2.0 * rho * cv)
    sq = np.sqrt(T0)
    fields = [rho - 1.0] + [u[a] / sq for a in range(D)] + [T / T0 - 1.0]
    Nax = []
    for a in range(D):
        Nax.append(mesh.ncell[a] * mesh.p + (0 if mesh.face_bc[a][0] < 0 else 1))
    shape = tuple(reversed(Nax))                                  # [Nz, Ny, Nx]: x fastest
    out = [np.asarray(fv) for fv in fields]
    for fv in fields:
        grid = fv.reshape(shape)
        for a in range(D):
            ax = D - 1 - a                                        # numpy axis of mesh axis a
            moved = np.moveaxis(grid, ax, -1)
            der, h = _axis_derivative(mesh, a, moved)
            der = np.moveaxis(der * h, -1, ax)
            out.append(der.reshape(-1))
    return np.stack(out, axis=1)


# --------------------------------------------------------------------------
# Projection off the collision invariants
# --------------------------------------------------------------------------

def invariants(zeta):
    """M [D+2, 2Q]: rows 1 | 0, zeta_a | 0, |zeta|^2 | 1 acting on (f, g)."""
    Q, D = zeta.shape
    M = np.zeros((D + 2, 2 * Q))
    M[0, :Q] = 1.0
    for a in range(D):
        M[1 + a, :Q] = zeta[:, a]
    M[D + 1, :Q] = (zeta ** 2).sum(axis=1)
    M[D + 1, Q:] = 1.0
    return M


def projector(zeta, w):
    """P = I - W M^T (M W M^T)^-1 M with W = diag(w, w): the projection off the
    invariants that is orthogonal in the inner product <a, b> = sum a b / w."""
    M = invariants(zeta)
    W = np.concatenate([w, w])
    WMt = W[:, None] * M.T
    G = np.linalg.inv(M @ WMt)
    return np.eye(2 * zeta.shape[0]) - WMt @ G @ M


# --------------------------------------------------------------------------
# The network
# --------------------------------------------------------------------------

def param_shapes(n_in, n_out):
    return [(n_in, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, n_out), (n_out,)]


def unflatten(theta, n_in, n_out):
    out, o = [], 0
    for s in param_shapes(n_in, n_out):
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def forward(params, x, emulate=True):
    """y [rows, n_out] and the values the backward pass needs.  With emulate, every
    matrix-product input is rounded to BF16 (activations and weights), the tanh is
    applied to the unrounded sum, biases and sums stay unrounded."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    W = [params[0], params[2], params[4], params[6]]
    b = [params[1], params[3], params[5], params[7]]
    acts = [np.asarray(x, dtype=np.float64)]        # layer inputs before rounding
    h = acts[0]
    for l in range(DEPTH):
        z = r(h) @ r(W[l]) + b[l]
        h = np.tanh(z)
        acts.append(h)
    y = r(h) @ r(W[3]) + b[3]
    return y, acts


def backward(params, acts, dy, emulate=True):
    """Gradients of sum(dy * y) with respect to the parameters (the chain rule through
    the linear layers and tanh), rounding the matrix-product inputs as forward does."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    W = [params[0], params[2], params[4], params[6]]
    grads = [None] * 8
    d = np.asarray(dy, dtype=np.float64)
    for l in range(DEPTH, -1, -1):
        hin = acts[l]
        grads[2 * l] = r(hin).T @ r(d)
        grads[2 * l + 1] = d.sum(axis=0)
        if l > 0:
            dh = r(d) @ r(W[l]).T
            d = dh * (1.0 - acts[l] ** 2)
    return grads


def loss_and_grad(params, x, t, emulate=True):
    """Mean-square loss over all rows and outputs, and its parameter gradient."""
    y, acts = forward(params, x, emulate)
    n = y.size
    diff = y - t
    loss = float((diff ** 2).sum() / n)
    return loss, backward(params, acts, 2.0 * diff / n, emulate), y


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1), in place on params, m, v."""
    for k in range(len(params)):
        m[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] ** 2
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)


# --------------------------------------------------------------------------
# Correction, targets, restriction
# --------------------------------------------------------------------------

def correct(mesh, zeta, w, gamma, pop, params, T0=1.0):
    """Post-collision populations plus the projected, scaled network output."""
    Q = zeta.shape[0]
    N = pop.size // (2 * Q)
    x = bf16(features(mesh, zeta, gamma, pop, T0))
    y, _ = forward(params, x)
    rho = pop[: Q * N].reshape(Q, N).sum(axis=0)
    scale = np.concatenate([w, w])[None, :] * rho[:, None]          # [N, 2Q]
    P = projector(zeta, w)
    delta = (scale * y) @ P.T                                         # [N, 2Q]
    return pop + delta.T.reshape(-1)


def targets(zeta, w, pop_plain, pop_true):
    """t = P (true - plain) / (w_i rho), rho of the plain coarse step: [N, 2Q]."""
    Q = zeta.shape[0]
    N = pop_plain.size // (2 * Q)
    rho = pop_plain[: Q * N].reshape(Q, N).sum(axis=0)
    d = (pop_true - pop_plain).reshape(2 * Q, N).T                    # [N, 2Q]
    P = projector(zeta, w)
    scale = np.concatenate([w, w])[None, :] * rho[:, None]
    return (d @ P.T) / scale


def restrict(fine_mesh, coarse_mesh, ratio, pop_fine, Q):
    """Injection: the coarse node (jx, jy, jz) takes the fine node (r jx, r jy, r jz)."""
    D = coarse_mesh.dim
    Nc = [coarse_mesh.ncell[a] * coarse_mesh.p + (0 if coarse_mesh.face_bc[a][0] < 0 else 1) for a in range(D)]
    Nf = [fine_mesh.ncell[a] * fine_mesh.p + (0 if fine_mesh.face_bc[a][0] < 0 else 1) for a in range(D)]
    grids = np.meshgrid(*[ratio * np.arange(n) for n in Nc], indexing="ij")    # [Nx, Ny(, Nz)]
    kf = np.zeros(grids[0].shape, dtype=np.int64)
    stride = 1
    for a in range(D):
        kf += grids[a] * stride
        stride *= Nf[a]
    kf = np.transpose(kf).reshape(-1)                                # coarse order, x fastest
    Nfine = int(np.prod(Nf))
    return pop_fine.reshape(2 * Q, Nfine)[:, kf].reshape(-1)
