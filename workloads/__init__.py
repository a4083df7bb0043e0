"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method: it only describes meshes
(cell edges, boundary tags), physical parameters and initial nodal fields
(density, velocity, temperature) as plain numbers and numpy arrays.  Both the
oracle (tests) and the library (bench, smoke) receive exactly these arrays.

Random numbers come from numpy's PCG64 with fixed seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# Largest Gauss-Hermite abscissa of the 5-point rule, sqrt(5 + sqrt(10)); used
# only to pick time steps from a CFL number on the cell size.
ZETA_MAX_GH5 = 2.8569700138728056

BC_PERIODIC, BC_WALL, BC_INLET, BC_OUTLET = 0, 1, 2, 3
NODES = {"gll": 0, "glc": 1, "equi": 2}


@dataclass
class BC:
    kind: int
    rho: float = 1.0
    u: Sequence[float] = (0.0, 0.0, 0.0)
    T: float = 1.0
    T_wall: float = float("nan")   # NaN: plain bounce-back, no thermal condition


@dataclass
class TensorMesh:
    dim: int
    p: int
    nodes: str                     # "gll" | "glc" | "equi"
    ncell: Sequence[int]
    edges: List[np.ndarray]        # per axis, ncell+1 monotone coordinates
    face_bc: List[List[int]]       # per axis [low, high]: index into bcs or -1 (periodic)
    bcs: List[BC] = field(default_factory=list)

    def periodic(self, a: int) -> bool:
        return self.face_bc[a][0] < 0

    def axis_nodes(self, a: int) -> int:
        return self.ncell[a] * self.p + (0 if self.periodic(a) else 1)

    @property
    def num_nodes(self) -> int:
        n = 1
        for a in range(self.dim):
            n *= self.axis_nodes(a)
        return n


@dataclass
class Physics:
    gamma: float = 1.4
    dt: float = 0.01
    relax_mode: int = 0            # 0 constant tau_bar, 1 mu(T) law, 2 streaming only
    tau_bar: float = 1.0
    mu_ref: float = 0.0
    T_ref: float = 1.0
    mu_exp: float = 0.0
    force: Sequence[float] = (0.0, 0.0, 0.0)
    T0: float = 1.0
    Pr: float = 1.0


def uniform_edges(n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n


def tanh_edges(n: int, beta: float = 2.0) -> np.ndarray:
    """Wall-normal channel edges on [0, 2]: y = 1 + tanh(beta (2 eta - 1)) / tanh(beta)."""
    eta = np.arange(n + 1, dtype=np.float64) / n
    y = 1.0 + np.tanh(beta * (2.0 * eta - 1.0)) / np.tanh(beta)
    y[0], y[-1] = 0.0, 2.0
    return y


# --------------------------------------------------------------------------
# C1: 2D periodic shear wave (and isentropic vortex), D2V25, p=4 GLL
# --------------------------------------------------------------------------

def shear_wave_case(ncell: int = 16, p: int = 4, nodes: str = "gll", tau_bar: float = 1.3,
                    cfl: float = 0.5):
    L = 2.0 * math.pi
    mesh = TensorMesh(dim=2, p=p, nodes=nodes, ncell=(ncell, ncell),
                      edges=[uniform_edges(ncell, 0.0, L), uniform_edges(ncell, 0.0, L)],
                      face_bc=[[-1, -1], [-1, -1]])
    h = L / ncell
    phys = Physics(gamma=1.4, dt=cfl * h / ZETA_MAX_GH5, relax_mode=0, tau_bar=tau_bar)
    return mesh, phys


def shear_wave_fields(xyz: np.ndarray, amp: float = 0.01, U: Optional[float] = None,
                      noise: float = 1e-3, seed: int = 1):
    """u = (U, A sin x), rho = 1 + noise*U(-1,1), T = 1.  U defaults to Ma 0.5."""
    if U is None:
        U = 0.5 * math.sqrt(1.4)
    n = xyz.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = np.ones(n) + (noise * rng.uniform(-1.0, 1.0, n) if noise > 0 else 0.0)
    u = np.zeros((n, 2))
    u[:, 0] = U
    u[:, 1] = amp * np.sin(xyz[:, 0])
    T = np.ones(n)
    return rho, u, T


def vortex_case(ncell: int = 16, p: int = 4, nodes: str = "gll", tau_bar: float = 1.3, cfl: float = 0.5):
    L = 10.0
    mesh = TensorMesh(dim=2, p=p, nodes=nodes, ncell=(ncell, ncell),
                      edges=[uniform_edges(ncell, 0.0, L), uniform_edges(ncell, 0.0, L)],
                      face_bc=[[-1, -1], [-1, -1]])
    phys = Physics(gamma=1.4, dt=cfl * (L / ncell) / ZETA_MAX_GH5, relax_mode=0, tau_bar=tau_bar)
    return mesh, phys


def vortex_fields(xyz: np.ndarray, eps: float = 2.0, gamma: float = 1.4, noise: float = 1e-3, seed: int = 1):
    """Isentropic vortex of strength eps centred at (5, 5) on a Ma 0.5 stream in x."""
    U = 0.5 * math.sqrt(gamma)
    x = xyz[:, 0] - 5.0
    y = xyz[:, 1] - 5.0
    r2 = x * x + y * y
    f = np.exp(0.5 * (1.0 - r2))
    du = eps / (2.0 * math.pi) * f
    u = np.stack([U - du * y, du * x], axis=1)
    T = 1.0 - (gamma - 1.0) * eps ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    if noise > 0:
        rho = rho + noise * rng.uniform(-1.0, 1.0, rho.shape[0])
    return rho, u, T


# --------------------------------------------------------------------------
# C2: 3D periodic compressible Taylor-Green vortex, Ma 0.8, Re 400, p=3
# --------------------------------------------------------------------------

def tgv_case(ncell: int = 32, p: int = 3, nodes: str = "gll", cfl: float = 0.5, Re: float = 400.0,
             Ma: float = 0.8, dt: Optional[float] = None):
    L = 2.0 * math.pi
    mesh = TensorMesh(dim=3, p=p, nodes=nodes, ncell=(ncell, ncell, ncell),
                      edges=[uniform_edges(ncell, 0.0, L)] * 3,
                      face_bc=[[-1, -1], [-1, -1], [-1, -1]])
    U0 = Ma * math.sqrt(1.4)
    phys = Physics(gamma=1.4, dt=dt if dt is not None else cfl * (L / ncell) / ZETA_MAX_GH5, relax_mode=1,
                   mu_ref=U0 / Re, T_ref=1.0, mu_exp=0.0)
    return mesh, phys


# time step of the 32^3-cell configuration (CFL 0.5 on its cell size)
TGV_DT = 0.5 * (2.0 * math.pi / 32) / ZETA_MAX_GH5


def tgv_fields(xyz: np.ndarray, Ma: float = 0.8):
    U0 = Ma * math.sqrt(1.4)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    u = np.stack([U0 * np.sin(x) * np.cos(y) * np.cos(z),
                  -U0 * np.cos(x) * np.sin(y) * np.cos(z),
                  np.zeros_like(x)], axis=1)
    p = 1.0 + (U0 ** 2 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    T = np.ones_like(x)
    rho = p / T
    return rho, u, T


# --------------------------------------------------------------------------
# C4: 3D supersonic channel, isothermal walls at y = 0 and y = 2, tanh y-stretching
# --------------------------------------------------------------------------

def channel_case(ncell=(128, 96, 64), p: int = 2, nodes: str = "gll", Ma_b: float = 1.5, Re_b: float = 3000.0,
                 Re_tau: float = 220.6, cfl: float = 0.9, beta: float = 2.0, T_wall: float = 1.0,
                 box=(4.0 * math.pi, 2.0, 2.0 * math.pi)):
    ex = uniform_edges(ncell[0], 0.0, box[0])
    ey = tanh_edges(ncell[1], beta) * (box[1] / 2.0)
    ez = uniform_edges(ncell[2], 0.0, box[2])
    bcs = [BC(kind=BC_WALL, T_wall=T_wall)]
    mesh = TensorMesh(dim=3, p=p, nodes=nodes, ncell=tuple(ncell), edges=[ex, ey, ez],
                      face_bc=[[-1, -1], [0, 0], [-1, -1]], bcs=bcs)
    hmin = float(np.min(np.diff(ey)))
    u_b = Ma_b * math.sqrt(1.4 * T_wall)
    mu_w = 1.0 * u_b * 1.0 / Re_b
    F = 1.0 * Re_tau ** 2 * mu_w ** 2
    phys = Physics(gamma=1.4, dt=cfl * hmin / ZETA_MAX_GH5, relax_mode=1, mu_ref=mu_w, T_ref=T_wall,
                   mu_exp=0.7, force=(F, 0.0, 0.0))
    return mesh, phys


def channel_controller(Ma_b: float = 1.5, T_wall: float = 1.0, rho_b: float = 1.0, tau_c: float = 1.0):
    """Inputs of the channel's force controller: hold the mean streamwise momentum density
    at rho_b u_b; gains of a critically damped loop with time constant tau_c
    (kp = 2 / tau_c, ki = 1 / tau_c^2), since the paper gives none."""
    u_b = Ma_b * math.sqrt(1.4 * T_wall)
    return {"axis": 0, "target": rho_b * u_b, "kp": 2.0 / tau_c, "ki": 1.0 / tau_c ** 2}


def channel_fields(xyz: np.ndarray, Ma_b: float = 1.5, T_wall: float = 1.0, amp: float = 0.05,
                   kmax: int = 4, seed: int = 4, box=(4.0 * math.pi, 2.0, 2.0 * math.pi)):
    """Poiseuille profile 1.5 u_b (1 - (y-1)^2) plus random-phase modes scaled by a parabola."""
    u_b = Ma_b * math.sqrt(1.4 * T_wall)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    par = 1.0 - (y - 1.0) ** 2
    u = np.zeros((xyz.shape[0], 3))
    u[:, 0] = 1.5 * u_b * par
    rng = np.random.Generator(np.random.PCG64(seed))
    for comp in range(3):
        pert = np.zeros_like(x)
        for kx in range(1, kmax + 1):
            for kz in range(1, kmax + 1):
                ph = rng.uniform(0.0, 2.0 * math.pi, 2)
                pert += np.sin(2 * math.pi * kx * x / box[0] + ph[0]) * np.sin(2 * math.pi * kz * z / box[2] + ph[1])
        pert /= max(np.max(np.abs(pert)), 1e-30)
        u[:, comp] += amp * u_b * par * pert
    rho = np.ones(xyz.shape[0])
    T = np.full(xyz.shape[0], T_wall)
    return rho, u, T


def random_fields(n: int, dim: int, seed: int, rho_amp=0.05, u_amp=0.2, T_amp=0.05, u_mean=None):
    """Smooth-free random nodal state near rest: used by interpolation/BC unit tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = 1.0 + rho_amp * rng.uniform(-1.0, 1.0, n)
    u = u_amp * rng.uniform(-1.0, 1.0, (n, dim))
    if u_mean is not None:
        u = u + np.asarray(u_mean)[None, :dim]
    T = 1.0 + T_amp * rng.uniform(-1.0, 1.0, n)
    return rho, u, T


# --------------------------------------------------------------------------
# C5: temporal compressible mixing layer (Sec. 4.4), coarse and nested fine meshes
# --------------------------------------------------------------------------

MIX_DTHETA0 = 0.093


def mixing_layer_case(ncell=(64, 64, 64), p: int = 2, refine: int = 1, Ma_c: float = 0.7, box=None,
                      Re_theta: float = 160.0, cfl: float = 0.5, T_inf: float = 1.0):
    """Periodic in x and z, bounded in y by moving equilibrium walls u_x = +-du/2 (the
    temporal mixing layer of Sec. 4.4; du = 2 Ma_c sqrt(gamma T)).  The box defaults to
    160 x 176 x 98 initial momentum thicknesses (0.093).  refine = r gives the nested
    fine mesh with r times the cells per axis and the time step divided by r, whose
    every r-th node along each axis is a node of the coarse mesh (p = 2, GLL)."""
    if box is None:
        box = (160 * MIX_DTHETA0, 176 * MIX_DTHETA0, 98 * MIX_DTHETA0)
    n = tuple(c * refine for c in ncell)
    du = 2.0 * Ma_c * math.sqrt(1.4 * T_inf)
    edges = [uniform_edges(n[0], 0.0, box[0]), uniform_edges(n[1], -0.5 * box[1], 0.5 * box[1]),
             uniform_edges(n[2], 0.0, box[2])]
    bcs = [BC(kind=BC_INLET, rho=1.0, u=(-0.5 * du, 0.0, 0.0), T=T_inf),
           BC(kind=BC_INLET, rho=1.0, u=(0.5 * du, 0.0, 0.0), T=T_inf)]
    mesh = TensorMesh(dim=3, p=p, nodes="gll", ncell=n, edges=edges,
                      face_bc=[[-1, -1], [0, 1], [-1, -1]], bcs=bcs)
    h_coarse = min(box[a] / ncell[a] for a in range(3))
    dt = cfl * h_coarse / ZETA_MAX_GH5 / refine
    mu = du * MIX_DTHETA0 / Re_theta
    phys = Physics(gamma=1.4, dt=dt, relax_mode=1, mu_ref=mu, T_ref=T_inf, mu_exp=0.0)
    return mesh, phys


def mixing_layer_fields(xyz: np.ndarray, Ma_c: float = 0.7, amp: float = 0.05, seed: int = 5, T_inf: float = 1.0,
                        box=None, kmax: int = 4):
    """tanh profile u_x = du/2 tanh(y / (2 dtheta0)) plus broadband seeded perturbations
    (random-phase Fourier modes up to kmax per periodic axis, amplitude amp du, confined
    to the layer by a Gaussian in y); rho = 1, T = T_inf."""
    if box is None:
        box = (160 * MIX_DTHETA0, 176 * MIX_DTHETA0, 98 * MIX_DTHETA0)
    du = 2.0 * Ma_c * math.sqrt(1.4 * T_inf)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    rng = np.random.Generator(np.random.PCG64(seed))
    env = np.exp(-(y / (4.0 * MIX_DTHETA0)) ** 2)
    u = np.zeros((xyz.shape[0], 3))
    u[:, 0] = 0.5 * du * np.tanh(y / (2.0 * MIX_DTHETA0))
    for c in range(3):
        for kx in range(1, kmax + 1):
            for kz in range(0, kmax + 1):
                ph = rng.uniform(0.0, 2.0 * math.pi, 2)
                a = rng.uniform(-1.0, 1.0)
                u[:, c] += (amp * du / kmax) * a * env * np.cos(2 * math.pi * kx * x / box[0] + ph[0]) * \
                    np.cos(2 * math.pi * kz * z / box[2] + ph[1])
    return np.ones(xyz.shape[0]), u, np.full(xyz.shape[0], T_inf)


# --------------------------------------------------------------------------
# Curvilinear meshes (2D isoparametric quads of order p)
# --------------------------------------------------------------------------

@dataclass
class CurvMesh:
    """Unique nodes, cell -> node lists (reference order, xi fastest) and per-face
    boundary tags (xi-, xi+, eta-, eta+; -1 interior)."""
    p: int
    nodes: str
    node_xyz: np.ndarray
    cell_nodes: np.ndarray
    cell_face_bc: np.ndarray
    bcs: List[BC] = field(default_factory=list)
    dim: int = 2

    @property
    def num_nodes(self) -> int:
        return self.node_xyz.shape[0]


def _gll_positions(p: int, nodes: str) -> np.ndarray:
    """Where a mesh places the support points of a cell on [-1, 1] (mesh geometry)."""
    if nodes == "glc":
        return -np.cos(np.pi * np.arange(p + 1) / p)
    if nodes == "equi":
        return -1.0 + 2.0 * np.arange(p + 1) / p
    from numpy.polynomial import legendre
    inner = legendre.Legendre.basis(p).deriv().roots() if p > 1 else np.array([])
    return np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])


def _structured_cells(na: int, nr: int, p: int, periodic_a: bool):
    """Cell -> node lists of a structured (a, r) grid of na x nr cells; node index
    ia + Na ir with Na = na p (periodic in a) or na p + 1."""
    Na = na * p if periodic_a else na * p + 1
    cells = np.zeros((na * nr, (p + 1) ** 2), dtype=np.int64)
    for cr in range(nr):
        for ca in range(na):
            c = ca + na * cr
            for jy in range(p + 1):
                for jx in range(p + 1):
                    ia = ca * p + jx
                    if periodic_a:
                        ia %= Na
                    cells[c, jx + (p + 1) * jy] = ia + Na * (cr * p + jy)
    return Na, cells


def curv_box(mesh: TensorMesh, warp: float = 0.0) -> CurvMesh:
    """A 2D tensor-product box as an explicit curvilinear mesh (bounded on every face:
    face_bc of the tensor description gives the four sides' tags); warp > 0 bends the
    interior with a smooth map that fixes the boundary."""
    assert mesh.dim == 2
    p = mesh.p
    xr = _gll_positions(p, mesh.nodes)

    def axis_coords(a):
        e = mesh.edges[a]
        c = [e[0]]
        for k in range(mesh.ncell[a]):
            for b in range(1, p + 1):
                c.append(e[k] + 0.5 * (1 + xr[b]) * (e[k + 1] - e[k]))
        return np.array(c)

    cx, cy = axis_coords(0), axis_coords(1)
    X, Y = np.meshgrid(cx, cy)
    if warp > 0:
        Lx, Ly = cx[-1] - cx[0], cy[-1] - cy[0]
        sx = np.sin(np.pi * (X - cx[0]) / Lx) * np.sin(np.pi * (Y - cy[0]) / Ly)
        X, Y = X + warp * Lx * sx * 0.05, Y + warp * Ly * sx * 0.03
    xyz = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    na, nr = mesh.ncell
    _, cells = _structured_cells(na, nr, p, False)
    fb = -np.ones((na * nr, 4), dtype=np.int32)
    for cr in range(nr):
        for ca in range(na):
            c = ca + na * cr
            if ca == 0:
                fb[c, 0] = mesh.face_bc[0][0]
            if ca == na - 1:
                fb[c, 1] = mesh.face_bc[0][1]
            if cr == 0:
                fb[c, 2] = mesh.face_bc[1][0]
            if cr == nr - 1:
                fb[c, 3] = mesh.face_bc[1][1]
    return CurvMesh(p=p, nodes=mesh.nodes, node_xyz=xyz, cell_nodes=cells, cell_face_bc=fb, bcs=list(mesh.bcs))


def naca0012_surface(theta: np.ndarray) -> np.ndarray:
    """Closed-trailing-edge NACA 0012 (4-digit thickness law with -0.1036 x^4), chord
    [0, 1], parametrised by x = (1 + cos theta)/2: upper side for theta in [0, pi]."""
    x = 0.5 * (1.0 + np.cos(theta))
    yt = 0.6 * (0.2969 * np.sqrt(np.maximum(x, 0.0)) - 0.1260 * x - 0.3516 * x ** 2 + 0.2843 * x ** 3 - 0.1036 * x ** 4)
    y = np.where(np.sin(theta) >= 0.0, yt, -yt)
    return np.stack([x, y], axis=-1)


def naca_ogrid(n_around: int = 256, n_radial: int = 128, p: int = 4, nodes: str = "gll", R_out: float = 10.0,
               dr0: float = 2e-3, Ma: float = 1.5, Re: float = 1e4, T_inf: float = 1.0, gamma: float = 1.4,
               dt: float = 1.5e-4, smooth: int = 20):
    """Body-fitted O-grid around a NACA 0012 section: n_around cells around (cosine
    clustering at the leading and trailing edges through the x = (1+cos)/2 law) and
    n_radial cells out to a circle of radius R_out about mid-chord, geometric growth
    from a first cell of dr0.  Node layers are marched along smoothed layer normals
    (which spreads the trailing-edge fan) out to about one chord, then continued
    straight to uniformly spaced points of the circle.  Isoparametric cells of order p.
    Thermal wall on the airfoil at T_w = T_inf; equilibrium inlet on the upstream arc of
    the outer circle (polar angle about mid-chord beyond +-100 deg), outlet on the rest."""
    xr = _gll_positions(p, nodes)
    Na, cells = _structured_cells(n_around, n_radial, p, True)
    th_edges = 2.0 * np.pi * np.arange(n_around + 1) / n_around
    th = np.concatenate([th_edges[c] + 0.5 * (1 + xr[:-1]) * (th_edges[c + 1] - th_edges[c]) for c in range(n_around)])
    # geometric radial cell edges r_e (distance parameter from the wall), then node layers
    L = R_out - 0.5
    lo, hi = 1.0 + 1e-12, 10.0       # growth factor q: dr0 (q^n - 1)/(q - 1) = L, by bisection
    for _ in range(200):
        q = 0.5 * (lo + hi)
        if dr0 * (q ** n_radial - 1.0) / (q - 1.0) > L:
            hi = q
        else:
            lo = q
    re = L * (q ** np.arange(n_radial + 1) - 1.0) / (q ** n_radial - 1.0)
    rn = np.concatenate([re[c] + 0.5 * (1 + xr[:-1]) * (re[c + 1] - re[c]) for c in range(n_radial)] + [re[-1:]])
    A = naca0012_surface(th)
    # march node layers along smoothed normals out to about one chord (a cell edge) ...
    ms = int(np.argmin(np.abs(re - 1.0))) * p
    layers = [A]
    X = A.copy()
    for m in range(1, ms + 1):
        t = np.roll(X, -1, axis=0) - np.roll(X, 1, axis=0)
        n = np.stack([t[:, 1], -t[:, 0]], axis=1)
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        for _ in range(smooth):
            n = n + 0.5 * (np.roll(n, 1, axis=0) + np.roll(n, -1, axis=0))
            n /= np.linalg.norm(n, axis=1, keepdims=True)
        X = X + (rn[m] - rn[m - 1]) * n
        layers.append(X.copy())
    # ... then straight out to the circle of radius R_out about mid-chord, each grid line
    # ending at its own (uniformly spaced) angle parameter, spaced by the same layer
    # parameter
    O = np.stack([0.5 + R_out * np.cos(th), R_out * np.sin(th)], axis=-1)
    for m in range(ms + 1, len(rn)):
        a = (rn[m] - rn[ms]) / (rn[-1] - rn[ms])
        layers.append((1.0 - a) * X + a * O)
    layers = np.array(layers)                                      # [Nr, Na, 2]
    xyz = layers.reshape(-1, 2)
    fb = -np.ones((n_around * n_radial, 4), dtype=np.int32)
    u_inf = Ma * math.sqrt(gamma * T_inf)
    bcs = [BC(kind=BC_WALL, T_wall=T_inf), BC(kind=BC_INLET, rho=1.0, u=(u_inf, 0.0, 0.0), T=T_inf),
           BC(kind=BC_OUTLET)]
    outer = layers[-1]
    for ca in range(n_around):
        fb[ca, 2] = 0
        # inlet on the upstream arc, polar angle about mid-chord beyond +-100 deg: the
        # junctions with the outlet then sit where the circle's tangent is not a lattice
        # direction (at +-90 deg it is horizontal, and a horizontal velocity would graze
        # the boundary right at the junction)
        fm = outer[(ca * p + p // 2) % Na] - np.array([0.5, 0.0])
        fb[ca + n_around * (n_radial - 1), 3] = 1 if fm[0] / np.hypot(fm[0], fm[1]) < math.cos(math.radians(100.0)) else 2
    mesh = CurvMesh(p=p, nodes=nodes, node_xyz=np.ascontiguousarray(xyz), cell_nodes=cells, cell_face_bc=fb, bcs=bcs)
    mu = 1.0 * u_inf * 1.0 / Re
    phys = Physics(gamma=gamma, dt=dt, relax_mode=1, mu_ref=mu, T_ref=T_inf, mu_exp=0.0)
    return mesh, phys


def naca_fields(xyz: np.ndarray, Ma: float = 1.5, T_inf: float = 1.0, gamma: float = 1.4):
    """Free stream plus the vortex-street trigger u_y = 0.1 u_x sin(1.3 y + 0.1) (Sec. 4.1)."""
    u_inf = Ma * math.sqrt(gamma * T_inf)
    n = xyz.shape[0]
    u = np.zeros((n, 2))
    u[:, 0] = u_inf
    u[:, 1] = 0.1 * u_inf * np.sin(1.3 * xyz[:, 1] + 0.1)
    return np.ones(n), u, np.full(n, T_inf)
