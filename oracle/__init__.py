"""Oracle: plain, slow, FP64 CPU reference of the SLLBM time step (arXiv 2412.09051).

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU
baseline may import this package.  It shares no code with the HIP library:

* velocity set: 1D Gauss-Hermite rule from numpy (Sec. 3.2; 5 points give
  quadrature degree 9), tensor product over dimensions; or the reduced degree-9
  sets D2Q19 / D3Q45, solved from their moment conditions (cubature_set);
* support points: GLL from numpy's Legendre roots, GLC, equidistant (eq:intf);
* nodal volumes: integrals of the nodal Lagrange functions by Gauss-Legendre;
* the step itself: oracle/sllbm_oracle.c (tensor-product meshes),
  full tensor Lagrange product formula, explicit Hermite-tensor equilibrium.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
from numpy.polynomial import hermite_e, legendre

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = ctypes.CDLL(path)
    return _LIB


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


# --------------------------------------------------------------------------
# Velocity space (Sec. 3.2)
# --------------------------------------------------------------------------

def gauss_hermite_1d(n: int = 5):
    """Abscissae and weights of the n-point Gauss-Hermite rule for the weight
    exp(-x^2/2)/sqrt(2 pi) (roots of the n-th Hermite polynomial), ascending."""
    x, w = hermite_e.hermegauss(n)
    w = w / math.sqrt(2.0 * math.pi)
    o = np.argsort(x)
    return x[o].copy(), w[o].copy()


def velocity_set(dim: int, n: int = 5, T0: float = 1.0):
    """Product-rule velocity set D{dim}V{n^dim}: zeta_i = sqrt(T0) x_a, index
    i = a_x + n a_y + n^2 a_z over ascending abscissae; opposite reverses each a."""
    x, w = gauss_hermite_1d(n)
    Q = n ** dim
    zeta = np.zeros((Q, dim))
    wq = np.ones(Q)
    opp = np.zeros(Q, dtype=np.int32)
    for i in range(Q):
        r = i
        a = []
        for _ in range(dim):
            a.append(r % n)
            r //= n
        for d in range(dim):
            zeta[i, d] = math.sqrt(T0) * x[a[d]]
            wq[i] *= w[a[d]]
        j = 0
        for d in reversed(range(dim)):
            j = j * n + (n - 1 - a[d])
        opp[i] = j
    return zeta, wq, opp


def _orbit_unit_vectors(kind: str) -> np.ndarray:
    """Unit directions of one orbit, in a fixed order.

    hex0 / hex30: regular hexagon, vertex k at angle k pi/3 (hex0) or pi/6 + k pi/3 (hex30),
    k = 0..5.  ico: the 12 vertices of an icosahedron, the cyclic shifts of (0, +-1, +-phi)
    (shift c puts the 0 on axis c, +-1 on axis c+1, +-phi on axis c+2; c = 0, 1, 2 outer,
    then the sign of the 1, then the sign of phi, + before -).  dod: the dual dodecahedron,
    first the cube vertices (+-1, +-1, +-1) with x's sign changing fastest, then the cyclic
    shifts of (0, +-phi, +-1/phi) in the icosahedron's order."""
    if kind in ("hex0", "hex30"):
        # cos and sin of the six angles written out, so that zero components are exact
        h = math.sqrt(3.0) / 2.0
        if kind == "hex0":
            return np.array([(1.0, 0.0), (0.5, h), (-0.5, h), (-1.0, 0.0), (-0.5, -h), (0.5, -h)])
        return np.array([(h, 0.5), (0.0, 1.0), (-h, 0.5), (-h, -0.5), (0.0, -1.0), (h, -0.5)])
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    out = []
    if kind == "dod":
        for j in range(8):
            out.append([-1.0 if (j >> b) & 1 else 1.0 for b in range(3)])
        big, small = phi, 1.0 / phi
    else:
        big, small = 1.0, phi  # (0, 1, phi): the entry on axis c+1 is 1, on c+2 phi
    for c in range(3):
        for s1 in (1.0, -1.0):
            for s2 in (1.0, -1.0):
                v = [0.0, 0.0, 0.0]
                v[(c + 1) % 3] = s1 * big
                v[(c + 2) % 3] = s2 * small
                out.append(v)
    v = np.array(out)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def cubature_set(dim: int, T0: float = 1.0):
    """Reduced velocity sets D2Q19 and D3Q45 of quadrature degree 9 (Sec. 3.2).

    The paper names these point counts (the smallest known degree-9 cubatures for the
    Gaussian weight in 2D and 3D) but prints no abscissae, so the rules are fixed here
    from their defining conditions, for the weight exp(-|x|^2/2)/(2 pi)^(D/2):

    * 2D: the origin and three regular hexagons, two in the orientation hex0 and one in
      hex30; 3D: the origin, two icosahedra and the dual dodecahedron.  Each rule is
      invariant under the hexagon's (icosahedron's) symmetry group, which includes -1, so
      every odd moment vanishes, and every orbit reproduces the sphere's averages of the
      harmonics of degree 2 and 4 (and 8); what is left of exactness up to degree 9 is
      (i) the radial moments sum_k W_k s_k^m = E|x|^(2m), m = 0..4 (W_k: an orbit's total
      weight, s_k its squared radius) and (ii) the orbit averages y_k of the invariant
      harmonic of degree 6, alone and times |x|^2: sum_k W_k s_k^m y_k = 0, m = 3, 4.
    * The single orbit of the other orientation (hex30 / dod) follows from (ii) and the
      radial moments m = 3, 4; the two remaining orbits are then a two-node Gauss rule in s
      for the moments left over.
    * y_k is read off as the orbit's mean of x^6 minus the sphere's mean of x^6.

    Order: index 0 the origin, then the inner and the outer hex0 (ico) orbit, then the
    hex30 (dod) orbit, each in the order of _orbit_unit_vectors.  zeta = sqrt(T0) x.
    Returns (zeta [Q][dim], w [Q], opposite [Q])."""
    if dim == 2:
        main, other = _orbit_unit_vectors("hex0"), _orbit_unit_vectors("hex30")
    elif dim == 3:
        main, other = _orbit_unit_vectors("ico"), _orbit_unit_vectors("dod")
    else:
        raise ValueError("reduced cubature sets exist for dim 2 and 3")
    # E|x|^(2m) for the standard Gaussian in dim dimensions
    c = [float(np.prod([dim + 2 * j for j in range(m)])) for m in range(5)]
    # sphere mean of x^6: E[x^6] / E[|x|^6]
    sph6 = 15.0 / c[3]
    y_main = float(np.mean(main[:, 0] ** 6)) - sph6
    y_other = float(np.mean(other[:, 0] ** 6)) - sph6
    kappa = -y_other / y_main
    # (ii) with the radial moments 3 and 4: the other orbit's s and total weight
    B3, B4 = c[3] / (1.0 + kappa), c[4] / (1.0 + kappa)
    s_o = B4 / B3
    W_o = B3 / s_o ** 3
    # the main orbits carry the rest: moments A_m = sum W s^m, m = 1..4
    A = [None, c[1] - W_o * s_o, c[2] - W_o * s_o ** 2, kappa * B3, kappa * B4]
    # two-node Gauss rule for the measure s dW: nodes are the roots of s^2 + a s + b with
    # [A1 A2; A2 A3] [b; a] = -[A3; A4]
    b, a = np.linalg.solve(np.array([[A[1], A[2]], [A[2], A[3]]]), -np.array([A[3], A[4]]))
    # roots without cancellation: q = -(a + sign(a) sqrt(a^2 - 4b)) / 2, then q and b / q
    q = -0.5 * (a + math.copysign(math.sqrt(a * a - 4.0 * b), a))
    s_in, s_out = sorted((q, b / q))
    W_in, W_out = np.linalg.solve(np.array([[s_in, s_out], [s_in ** 2, s_out ** 2]]), np.array([A[1], A[2]]))
    W_0 = 1.0 - W_in - W_out - W_o
    pts = [np.zeros((1, dim)), main * math.sqrt(s_in), main * math.sqrt(s_out), other * math.sqrt(s_o)]
    ws = [np.array([W_0]), np.full(len(main), W_in / len(main)), np.full(len(main), W_out / len(main)),
          np.full(len(other), W_o / len(other))]
    zeta = math.sqrt(T0) * np.vstack(pts)
    w = np.concatenate(ws)
    Q = len(w)
    opp = np.zeros(Q, dtype=np.int32)
    for i in range(Q):
        d = np.max(np.abs(zeta + zeta[i]), axis=1)
        opp[i] = int(np.argmin(d))
        assert d[opp[i]] < 1e-12 * max(1.0, math.sqrt(T0))
    return zeta, w, opp


def stroud_bound(degree: int, dim: int) -> int:
    """Stroud's lower bound on the number of cubature points (Sec. 3.2 display)."""
    k = degree // 2
    return math.comb(k + dim, k)


# --------------------------------------------------------------------------
# Support points and nodal quadrature (eq:intf)
# --------------------------------------------------------------------------

def support_points(p: int, family: str = "gll") -> np.ndarray:
    if family == "gll":
        inner = legendre.Legendre.basis(p).deriv().roots() if p > 1 else np.array([])
        x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
        return x
    if family == "glc":
        return -np.cos(np.pi * np.arange(p + 1) / p)
    if family == "equi":
        return -1.0 + 2.0 * np.arange(p + 1) / p
    raise ValueError(family)


def lagrange_integrals(xref: np.ndarray) -> np.ndarray:
    """int_{-1}^{1} l_j(xi) d xi by Gauss-Legendre with enough points to be exact."""
    p = len(xref) - 1
    xq, wq = legendre.leggauss(p + 1)
    out = np.zeros(p + 1)
    for j in range(p + 1):
        v = np.ones_like(xq)
        for m in range(p + 1):
            if m != j:
                v *= (xq - xref[m]) / (xref[j] - xref[m])
        out[j] = np.sum(wq * v)
    return out


BC_CODES = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3}


class OrTensor(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("p", ctypes.c_int), ("Q", ctypes.c_int),
        ("zeta", _dp), ("w", _dp), ("opp", _ip), ("T0", ctypes.c_double),
        ("xref", _dp),
        ("ncell", ctypes.c_int * 3), ("edges", _dp * 3), ("periodic", ctypes.c_int * 3),
        ("face_bc", (ctypes.c_int * 2) * 3),
        ("n_bc", ctypes.c_int), ("bc_kind", _ip), ("bc_val", _dp),
        ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
        ("relax_mode", ctypes.c_int), ("tau_bar", ctypes.c_double), ("mu_ref", ctypes.c_double),
        ("T_ref", ctypes.c_double), ("mu_exp", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("mass_fix", ctypes.c_int), ("mass_ref", ctypes.c_double),
        ("node_vol", _dp), ("Pr", ctypes.c_double),
    ]


class OracleError(RuntimeError):
    pass


class TensorOracle:
    """FP64 reference of the SLLBM on a tensor-product (uniform or rectilinear) mesh.

    mesh / phys are workloads.TensorMesh / workloads.Physics instances."""

    def __init__(self, mesh, phys, n_gh: int = 5, vel=None):
        self.mesh, self.phys = mesh, phys
        self.dim = mesh.dim
        if vel is None:
            self.zeta, self.w, self.opp = velocity_set(mesh.dim, n_gh, phys.T0)
        else:  # explicit (zeta, w, opp), e.g. the integer set of the classic-LBM limit
            self.zeta = np.ascontiguousarray(vel[0], dtype=np.float64)
            self.w = np.ascontiguousarray(vel[1], dtype=np.float64)
            self.opp = np.ascontiguousarray(vel[2], dtype=np.int32)
        self.Q = self.zeta.shape[0]
        self.xref = support_points(mesh.p, mesh.nodes)
        self.N = mesh.num_nodes
        self._edges = [np.ascontiguousarray(e, dtype=np.float64) for e in mesh.edges]
        nb = max(len(mesh.bcs), 1)
        self._bc_kind = np.zeros(nb, dtype=np.int32)
        self._bc_val = np.zeros((nb, 6))
        for b, bc in enumerate(mesh.bcs):
            self._bc_kind[b] = bc.kind
            u = list(bc.u) + [0.0] * 3
            self._bc_val[b] = [bc.rho, u[0], u[1], u[2], bc.T, bc.T_wall]
        self.node_vol = self._node_volumes()
        s = OrTensor()
        s.dim, s.p, s.Q = mesh.dim, mesh.p, self.Q
        s.zeta, s.w, s.opp = _ptr(self.zeta), _ptr(self.w), _ptr(self.opp, _ip)
        s.T0 = phys.T0
        s.xref = _ptr(self.xref)
        for a in range(3):
            if a < mesh.dim:
                s.ncell[a] = mesh.ncell[a]
                s.edges[a] = _ptr(self._edges[a])
                s.periodic[a] = 1 if mesh.periodic(a) else 0
                s.face_bc[a][0], s.face_bc[a][1] = mesh.face_bc[a]
            else:
                s.ncell[a] = 1
                s.periodic[a] = 1
                s.face_bc[a][0] = s.face_bc[a][1] = -1
        s.n_bc = len(mesh.bcs)
        s.bc_kind, s.bc_val = _ptr(self._bc_kind, _ip), _ptr(self._bc_val)
        s.gamma, s.dt = phys.gamma, phys.dt
        s.relax_mode, s.tau_bar = phys.relax_mode, phys.tau_bar
        s.mu_ref, s.T_ref, s.mu_exp = phys.mu_ref, phys.T_ref, phys.mu_exp
        f = list(phys.force) + [0.0] * 3
        for a in range(3):
            s.force[a] = f[a] if a < mesh.dim else 0.0
        s.mass_fix, s.mass_ref = 0, 0.0
        s.node_vol = _ptr(self.node_vol)
        s.Pr = getattr(phys, "Pr", 1.0)
        self._s = s
        L = lib()
        L.or_tensor_num_nodes.restype = ctypes.c_size_t
        assert L.or_tensor_num_nodes(ctypes.byref(s)) == self.N

    # ---- geometry -------------------------------------------------------
    def _node_volumes(self):
        m = self.mesh
        li = lagrange_integrals(self.xref)
        vols = []
        for a in range(m.dim):
            Na = m.axis_nodes(a)
            v = np.zeros(Na)
            e = m.edges[a]
            for c in range(m.ncell[a]):
                h = e[c + 1] - e[c]
                for j in range(m.p + 1):
                    n = c * m.p + j
                    if m.periodic(a):
                        n %= Na
                    v[n] += 0.5 * h * li[j]
            vols.append(v)
        V = vols[0]
        for a in range(1, m.dim):
            V = np.multiply.outer(vols[a], V).reshape(-1)  # x fastest
        return np.ascontiguousarray(V.reshape(-1))

    def coords(self) -> np.ndarray:
        xyz = np.zeros((self.N, self.dim))
        lib().or_tensor_coords(ctypes.byref(self._s), _ptr(xyz))
        return xyz

    # ---- state ----------------------------------------------------------
    def init(self, rho, u, T) -> np.ndarray:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.N, self.dim)
        T = np.ascontiguousarray(T, dtype=np.float64)
        pop = np.zeros(2 * self.Q * self.N)
        lib().or_tensor_init(ctypes.byref(self._s), _ptr(rho), _ptr(u), _ptr(T), _ptr(pop))
        return pop

    def step(self, pop: np.ndarray, mass_ref: float | None = None) -> np.ndarray:
        out = np.empty_like(pop)
        s = self._s
        s.mass_fix = 1 if mass_ref is not None else 0
        s.mass_ref = float(mass_ref) if mass_ref is not None else 0.0
        err = np.zeros(2, dtype=np.int64)
        rc = lib().or_tensor_step(ctypes.byref(s), _ptr(np.ascontiguousarray(pop)), _ptr(out),
                                  err.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        s.mass_fix = 0
        if rc != 0:
            raise OracleError(f"oracle step failed rc={rc} at node {err[0]} velocity {err[1]}")
        return out

    def step_nodes(self, pop: np.ndarray, nodes, mass_ref: float | None = None) -> np.ndarray:
        """Post-collision populations at the listed nodes only: array [len(nodes)][2Q]."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        out = np.zeros((nodes.shape[0], 2 * self.Q))
        s = self._s
        s.mass_fix = 1 if mass_ref is not None else 0
        s.mass_ref = float(mass_ref) if mass_ref is not None else 0.0
        err = np.zeros(2, dtype=np.int64)
        rc = lib().or_tensor_step_nodes(ctypes.byref(s), _ptr(np.ascontiguousarray(pop)),
                                        nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        ctypes.c_int64(nodes.shape[0]), _ptr(out),
                                        err.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        s.mass_fix = 0
        if rc != 0:
            raise OracleError(f"oracle step failed rc={rc} at node {err[0]} velocity {err[1]}")
        return out

    def run(self, pop: np.ndarray, nsteps: int, mass_fix_every: int = 0, mass_ref: float | None = None):
        for n in range(nsteps):
            fix = mass_fix_every > 0 and n > 0 and n % mass_fix_every == 0
            pop = self.step(pop, mass_ref if fix else None)
        return pop

    def moments(self, pop: np.ndarray):
        rho = np.zeros(self.N)
        u = np.zeros((self.N, self.dim))
        T = np.zeros(self.N)
        lib().or_moments(ctypes.c_int(self.dim), ctypes.c_int(self.Q), _ptr(self.zeta),
                         ctypes.c_double(self.phys.gamma), ctypes.c_size_t(self.N),
                         _ptr(np.ascontiguousarray(pop)), _ptr(rho), _ptr(u), _ptr(T))
        return rho, u, T

    def totals(self, pop: np.ndarray):
        """Nodal-quadrature totals: mass, momentum[dim], total energy."""
        Q, N = self.Q, self.N
        f = pop[: Q * N].reshape(Q, N)
        g = pop[Q * N:].reshape(Q, N)
        V = self.node_vol
        mass = float(np.sum(V * f.sum(0)))
        mom = [float(np.sum(V * (self.zeta[:, a:a + 1] * f).sum(0))) for a in range(self.dim)]
        z2 = np.sum(self.zeta ** 2, axis=1)[:, None]
        energy = float(np.sum(V * ((z2 * f).sum(0) + g.sum(0))))
        return mass, mom, energy


    def set_force(self, force):
        """Body force of the following steps (Kupershtokh forcing, Sec. 4.3)."""
        f = list(force) + [0.0] * 3
        for a in range(3):
            self._s.force[a] = f[a] if a < self.dim else 0.0


class ForceController:
    """The driven channel's force controller (Sec. 4.3): the streamwise force starts at
    force0 and a PI law adjusts it to hold the mean momentum density at `target`.  Its
    discrete form (the paper gives none): at each update, with the mean momentum density
    m = sum_k V_k j_axis(k) / sum_k V_k over the nodal quadrature volumes,
        e = target - m,   I <- I + e dt,   F_axis = force0_axis + kp e + ki I.
    The new force is handed to the oracle for the steps that follow."""

    def __init__(self, oracle, force0, axis, target, kp, ki):
        self.o = oracle
        self.force0 = np.zeros(3)
        self.force0[:len(force0)] = force0
        self.force = self.force0.copy()
        self.axis, self.target, self.kp, self.ki = int(axis), float(target), float(kp), float(ki)
        self.integral = 0.0
        self.error = 0.0
        self.mean = 0.0
        oracle.set_force(self.force)

    def update(self, pop, dt):
        _, mom, _ = self.o.totals(pop)
        self.mean = mom[self.axis] / float(np.sum(self.o.node_vol))
        self.error = self.target - self.mean
        self.integral += self.error * dt
        self.force[self.axis] = self.force0[self.axis] + self.kp * self.error + self.ki * self.integral
        self.o.set_force(self.force)
        return self.force.copy()


def equilibrium(dim: int, rho: float, u, T: float, gamma: float = 1.4, T0: float = 1.0, n_gh: int = 5, vel=None):
    """f^eq and g^eq of one state for every velocity of the D{dim}V{n^dim} set, or of an
    explicit set vel = (zeta, w, opposite) built for the same T0."""
    zeta, w, _ = velocity_set(dim, n_gh, T0) if vel is None else vel
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    Q = zeta.shape[0]
    feq = np.zeros(Q)
    geq = np.zeros(Q)
    uu = np.zeros(3)
    uu[:dim] = u
    lib().or_equilibrium(ctypes.c_int(dim), ctypes.c_int(Q), _ptr(zeta), _ptr(w), ctypes.c_double(T0),
                         ctypes.c_double(gamma), ctypes.c_double(rho), _ptr(uu), ctypes.c_double(T),
                         _ptr(feq), _ptr(geq))
    return feq, geq


# --------------------------------------------------------------------------
# Curvilinear (isoparametric quadrilateral) meshes
# --------------------------------------------------------------------------

class OrCurv(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int), ("Q", ctypes.c_int), ("zeta", _dp), ("w", _dp), ("opp", _ip), ("T0", ctypes.c_double),
        ("xref", _dp), ("n_nodes", ctypes.c_int64), ("xyz", _dp), ("n_cells", ctypes.c_int64),
        ("cell_nodes", ctypes.POINTER(ctypes.c_int64)), ("face_bc", _ip), ("n_bc", ctypes.c_int), ("bc_kind", _ip),
        ("bc_val", _dp), ("gamma", ctypes.c_double), ("dt", ctypes.c_double), ("relax_mode", ctypes.c_int),
        ("tau_bar", ctypes.c_double), ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("mu_exp", ctypes.c_double), ("force", ctypes.c_double * 2), ("mass_fix", ctypes.c_int),
        ("mass_ref", ctypes.c_double), ("node_vol", _dp), ("Pr", ctypes.c_double),
        ("bx0", ctypes.c_double), ("by0", ctypes.c_double), ("bh", ctypes.c_double), ("bnx", ctypes.c_int),
        ("bny", ctypes.c_int), ("bstart", ctypes.POINTER(ctypes.c_int64)), ("bcells", ctypes.POINTER(ctypes.c_int64)),
    ]


def _lagrange_table(xref, pts):
    """l_j(pts) and l_j'(pts) by the product formula: arrays [len(pts), p+1]."""
    p = len(xref) - 1
    L = np.ones((len(pts), p + 1))
    dL = np.zeros((len(pts), p + 1))
    for j in range(p + 1):
        for m in range(p + 1):
            if m != j:
                L[:, j] *= (pts - xref[m]) / (xref[j] - xref[m])
        for k in range(p + 1):
            if k == j:
                continue
            t = np.full(len(pts), 1.0 / (xref[j] - xref[k]))
            for m in range(p + 1):
                if m != j and m != k:
                    t *= (pts - xref[m]) / (xref[j] - xref[m])
            dL[:, j] += t
    return L, dL


class CurvOracle:
    """FP64 reference of the SLLBM on a 2D curvilinear mesh (workloads.CurvMesh)."""

    def __init__(self, mesh, phys, n_gh: int = 5, geometry: bool = True, vel=None):
        """geometry=False skips the departure-point table (for tests of locate/exit);
        vel = (zeta, w, opposite) replaces the D2V{n_gh^2} set."""
        self.mesh, self.phys = mesh, phys
        self.dim = 2
        if vel is None:
            self.zeta, self.w, self.opp = velocity_set(2, n_gh, phys.T0)
        else:
            self.zeta = np.ascontiguousarray(vel[0], dtype=np.float64)
            self.w = np.ascontiguousarray(vel[1], dtype=np.float64)
            self.opp = np.ascontiguousarray(vel[2], dtype=np.int32)
        self.Q = self.zeta.shape[0]
        self.xref = support_points(mesh.p, mesh.nodes)
        self.xyz = np.ascontiguousarray(mesh.node_xyz, dtype=np.float64)
        self.N = self.xyz.shape[0]
        self.cells = np.ascontiguousarray(mesh.cell_nodes, dtype=np.int64)
        self.fb = np.ascontiguousarray(mesh.cell_face_bc, dtype=np.int32)
        nb = max(len(mesh.bcs), 1)
        self._bc_kind = np.zeros(nb, dtype=np.int32)
        self._bc_val = np.zeros((nb, 6))
        for b, bc in enumerate(mesh.bcs):
            self._bc_kind[b] = bc.kind
            u = list(bc.u) + [0.0] * 3
            self._bc_val[b] = [bc.rho, u[0], u[1], u[2], bc.T, bc.T_wall]
        self.node_vol = self._node_volumes()
        s = OrCurv()
        s.p, s.Q = mesh.p, self.Q
        s.zeta, s.w, s.opp, s.T0 = _ptr(self.zeta), _ptr(self.w), _ptr(self.opp, _ip), phys.T0
        s.xref = _ptr(self.xref)
        s.n_nodes, s.xyz = self.N, _ptr(self.xyz)
        s.n_cells, s.cell_nodes = self.cells.shape[0], self.cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        s.face_bc = _ptr(self.fb, _ip)
        s.n_bc, s.bc_kind, s.bc_val = len(mesh.bcs), _ptr(self._bc_kind, _ip), _ptr(self._bc_val)
        s.gamma, s.dt, s.relax_mode, s.tau_bar = phys.gamma, phys.dt, phys.relax_mode, phys.tau_bar
        s.mu_ref, s.T_ref, s.mu_exp = phys.mu_ref, phys.T_ref, phys.mu_exp
        f = list(phys.force) + [0.0, 0.0]
        s.force[0], s.force[1] = f[0], f[1]
        s.mass_fix, s.mass_ref, s.node_vol = 0, 0.0, _ptr(self.node_vol)
        s.Pr = getattr(phys, "Pr", 1.0)
        self._s = s
        # bucket width: the median cell extent, capped at ~4M buckets
        ext = np.ptp(self.xyz[self.cells], axis=1).max(axis=1)
        span = np.ptp(self.xyz, axis=0).max()
        h = max(float(np.median(ext)), span / 2000.0)
        lib().or_curv_prepare(ctypes.byref(s), ctypes.c_double(h))
        if geometry:
            self._geometry()

    def _geometry(self):
        s = self._s
        Qn = self.Q * self.N
        self.g_cell = np.zeros(Qn, dtype=np.int64)
        self.g_xi = np.zeros(2 * Qn)
        self.g_src = np.zeros(Qn, dtype=np.int32)
        self.g_kind = np.zeros(Qn, dtype=np.int32)
        self.g_th = np.zeros(self.N, dtype=np.int32)
        err = np.zeros(2, dtype=np.int64)
        rc = lib().or_curv_geometry(ctypes.byref(s), self.g_cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    _ptr(self.g_xi), _ptr(self.g_src, _ip), _ptr(self.g_kind, _ip),
                                    _ptr(self.g_th, _ip), err.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if rc != 0:
            raise OracleError(f"oracle geometry failed rc={rc} at node {err[0]} velocity {err[1]}")

    def __del__(self):
        if getattr(self, "_s", None) is not None:
            lib().or_curv_release(ctypes.byref(self._s))
            self._s = None

    def _node_volumes(self):
        """V_k = sum over cells of the integral of l_k |J| by a (p+2)^2 Gauss-Legendre rule."""
        xg, wg = legendre.leggauss(self.mesh.p + 2)
        L, dL = _lagrange_table(self.xref, xg)
        n1 = self.mesh.p + 1
        X = self.xyz[self.cells].reshape(-1, n1, n1, 2)           # [c, jy, jx, a]
        # basis at (gy, gx): L[gy, jy] L[gx, jx]
        dxi = np.einsum("cyxa,gy,hx->cgha", X, L, dL)
        deta = np.einsum("cyxa,gy,hx->cgha", X, dL, L)
        det = np.abs(dxi[..., 0] * deta[..., 1] - dxi[..., 1] * deta[..., 0])   # [c, gy, gx]
        wts = np.einsum("g,h,cgh->cgh", wg, wg, det)
        contrib = np.einsum("cgh,gy,hx->cyx", wts, L, L).reshape(len(self.cells), -1)
        V = np.zeros(self.N)
        np.add.at(V, self.cells.reshape(-1), contrib.reshape(-1))
        return V

    def coords(self):
        return self.xyz.copy()

    def init(self, rho, u, T):
        pop = np.zeros(2 * self.Q * self.N)
        lib().or_init_generic(ctypes.c_int(2), ctypes.c_int(self.Q), _ptr(self.zeta), _ptr(self.w),
                              ctypes.c_double(self.phys.T0), ctypes.c_double(self.phys.gamma),
                              ctypes.c_int64(self.N), _ptr(np.ascontiguousarray(rho, dtype=np.float64)),
                              _ptr(np.ascontiguousarray(u, dtype=np.float64).reshape(self.N, 2)),
                              _ptr(np.ascontiguousarray(T, dtype=np.float64)), _ptr(pop))
        return pop

    def step(self, pop, mass_ref=None):
        out = np.empty_like(pop)
        s = self._s
        s.mass_fix = 1 if mass_ref is not None else 0
        s.mass_ref = float(mass_ref) if mass_ref is not None else 0.0
        lib().or_curv_step(ctypes.byref(s), self.g_cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           _ptr(self.g_xi), _ptr(self.g_src, _ip), _ptr(self.g_kind, _ip), _ptr(self.g_th, _ip),
                           _ptr(np.ascontiguousarray(pop)), _ptr(out))
        s.mass_fix = 0
        return out

    def run(self, pop, nsteps, mass_fix_every=0, mass_ref=None):
        for n in range(nsteps):
            fix = mass_fix_every > 0 and n > 0 and n % mass_fix_every == 0
            pop = self.step(pop, mass_ref if fix else None)
        return pop

    def step_nodes(self, pop, nodes, mass_ref=None):
        """One step at the given nodes only (their geometry computed on the fly):
        returns [len(nodes), 2Q] = (f_0..f_{Q-1}, g_0..g_{Q-1}) per node."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        out = np.zeros((nodes.size, 2 * self.Q))
        err = np.zeros(2, dtype=np.int64)
        s = self._s
        s.mass_fix = 1 if mass_ref is not None else 0
        s.mass_ref = float(mass_ref) if mass_ref is not None else 0.0
        rc = lib().or_curv_step_nodes(ctypes.byref(s), _ptr(np.ascontiguousarray(pop)),
                                      nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      ctypes.c_int64(nodes.size), _ptr(out),
                                      err.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        s.mass_fix = 0
        if rc != 0:
            raise OracleError(f"oracle geometry failed rc={rc} at node {err[0]} velocity {err[1]}")
        return out

    def locate(self, x):
        """(cell, reference coordinates) of point x, cell -1 outside the mesh."""
        L = lib()
        L.or_curv_locate.restype = ctypes.c_int64
        xi = np.zeros(2)
        c = L.or_curv_locate(ctypes.byref(self._s), _ptr(np.ascontiguousarray(x, dtype=np.float64)), _ptr(xi))
        return int(c), xi

    def exit(self, x0, v):
        """(s, bc) where x0 + s v leaves the mesh, s in [0, 1], x0 inside."""
        L = lib()
        L.or_curv_exit.restype = ctypes.c_double
        bc = ctypes.c_int(-1)
        s = L.or_curv_exit(ctypes.byref(self._s), _ptr(np.ascontiguousarray(x0, dtype=np.float64)),
                           _ptr(np.ascontiguousarray(v, dtype=np.float64)), ctypes.byref(bc))
        return float(s), bc.value

    moments = TensorOracle.moments
    totals = TensorOracle.totals
