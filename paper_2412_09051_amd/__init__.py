"""Python binding of libsllbm, the MI355X SLLBM hot path (arXiv 2412.09051).

Argument marshalling only: every step of the method runs in the HIP library.
The functions carry the C-ABI names of include/sllbm.h.  PyTorch supplies device
memory and streams (tensor data pointers, torch.cuda.current_stream()).

Importing this module loads paper_2412_09051_amd/libsllbm.so and raises if it is
missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
# torch first: its bundled HIP runtime is then the one libsllbm.so binds to.  Loaded the
# other way round, the process would hold two HIP runtimes, and whichever initialises
# first keeps the GPU (the other reports no device).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
# SLLBM_LIB names another build of the library (e.g. a variant for an A/B timing)
LIB_PATH = os.environ.get("SLLBM_LIB") or os.path.join(HERE, "libsllbm.so")

SLLBM_OK, SLLBM_EINVAL, SLLBM_ENOMEM, SLLBM_EGEOM, SLLBM_EHIP, SLLBM_EUNSUPPORTED, SLLBM_EUNSTABLE = \
    0, -1, -2, -3, -4, -5, -6
ERR_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EGEOM", -4: "EHIP", -5: "EUNSUPPORTED", -6: "EUNSTABLE"}
SLLBM_NODES = {"gll": 0, "glc": 1, "equi": 2}
SLLBM_MESH_TENSOR, SLLBM_MESH_CURVILINEAR = 0, 1
SLLBM_F64, SLLBM_F32 = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2412_09051_amd/build.py` "
                      "(there is no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)


class SllbmError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.sllbm_last_error().decode()
        super().__init__(f"{where}: {ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class sllbm_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rho", ctypes.c_double), ("u", ctypes.c_double * 3),
                ("T", ctypes.c_double), ("T_wall", ctypes.c_double)]


class sllbm_mesh_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order_p", ctypes.c_int), ("nodes", ctypes.c_int), ("kind", ctypes.c_int),
                ("ncell", ctypes.c_int * 3), ("edges", _dp * 3), ("face_bc", (ctypes.c_int * 2) * 3),
                ("n_nodes", ctypes.c_int64), ("node_xyz", _dp),
                ("n_cells", ctypes.c_int64), ("cell_nodes", ctypes.POINTER(ctypes.c_int64)),
                ("cell_face_bc", ctypes.POINTER(ctypes.c_int32)),
                ("n_bc", ctypes.c_int), ("bcs", ctypes.POINTER(sllbm_bc))]


class sllbm_velset(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("Q", ctypes.c_int), ("zeta", _dp), ("w", _dp),
                ("opposite", ctypes.POINTER(ctypes.c_int32)), ("T0", ctypes.c_double)]


class sllbm_plan_info_t(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("Q", ctypes.c_int), ("dim", ctypes.c_int), ("order_p", ctypes.c_int),
                ("prec", ctypes.c_int), ("n_exceptions", ctypes.c_int64), ("n_thermal_nodes", ctypes.c_int64),
                ("table_bytes", ctypes.c_int64), ("has_device", ctypes.c_int), ("kernel", ctypes.c_int)]


class sllbm_params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("relax_mode", ctypes.c_int), ("tau_bar", ctypes.c_double),
                ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("mu_exp", ctypes.c_double),
                ("Pr", ctypes.c_double), ("force", ctypes.c_double * 3), ("mass_fix", ctypes.c_int),
                ("mass_ref", ctypes.c_double), ("force_device", ctypes.c_int)]


class sllbm_force_ctl(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int), ("target", ctypes.c_double), ("kp", ctypes.c_double),
                ("ki", ctypes.c_double), ("dt", ctypes.c_double)]


_lib.sllbm_last_error.restype = ctypes.c_char_p
for _name in ("sllbm_mesh_build", "sllbm_mesh_nodes", "sllbm_mesh_volumes", "sllbm_velset_gauss_hermite",
              "sllbm_velset_cubature",
              "sllbm_interp_plan", "sllbm_plan_info", "sllbm_plan_select_kernel", "sllbm_init_equilibrium",
              "sllbm_step", "sllbm_moments", "sllbm_moments_noalloc", "sllbm_plan_profile", "sllbm_plan_profile_read",
              "sllbm_force_reset", "sllbm_force_update", "sllbm_force_read", "sllbm_set_allocator"):
    getattr(_lib, _name).restype = ctypes.c_int
_lib.sllbm_mesh_destroy.restype = None
_lib.sllbm_plan_destroy.restype = None


def _check(rc, where):
    if rc != SLLBM_OK:
        raise SllbmError(rc, where)


def _np_ptr(a, t=_dp):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------------ handles

class Mesh:
    """Owner of an sllbm_mesh handle."""

    def __init__(self, handle, dim):
        self._lib = _lib
        self.handle = handle
        self.dim = dim

    def __del__(self):
        # the instance keeps the library alive: module globals may already be gone
        # when the interpreter shuts down
        lib = getattr(self, "_lib", None)
        if getattr(self, "handle", None) and lib is not None:
            lib.sllbm_mesh_destroy(self.handle)
            self.handle = None


class Plan:
    """Owner of an sllbm_plan handle (keeps its mesh alive)."""

    def __init__(self, handle, mesh, velset, dt, prec):
        self._lib = _lib
        self.handle = handle
        self.mesh = mesh
        self.velset = velset
        self.dt = dt
        self.prec = prec
        info = sllbm_plan_info(self)
        self.N = info["n_nodes"]
        self.Q = info["Q"]
        self.dim = info["dim"]

    def __del__(self):
        lib = getattr(self, "_lib", None)
        if getattr(self, "handle", None) and lib is not None:
            lib.sllbm_plan_destroy(self.handle)
            self.handle = None


@dataclass
class Params:
    gamma: float = 1.4
    relax_mode: int = 0
    tau_bar: float = 1.0
    mu_ref: float = 0.0
    T_ref: float = 1.0
    mu_exp: float = 0.0
    Pr: float = 1.0
    force: Sequence[float] = (0.0, 0.0, 0.0)
    mass_fix: int = 0
    mass_ref: float = 0.0
    force_device: int = 0

    def c(self):
        p = sllbm_params()
        p.gamma, p.relax_mode, p.tau_bar = self.gamma, self.relax_mode, self.tau_bar
        p.mu_ref, p.T_ref, p.mu_exp, p.Pr = self.mu_ref, self.T_ref, self.mu_exp, self.Pr
        f = list(self.force) + [0.0, 0.0, 0.0]
        for a in range(3):
            p.force[a] = f[a]
        p.mass_fix, p.mass_ref = int(self.mass_fix), float(self.mass_ref)
        p.force_device = int(self.force_device)
        return p

    @staticmethod
    def from_physics(phys, **kw):
        """Marshal a workloads.Physics description."""
        p = Params(gamma=phys.gamma, relax_mode=phys.relax_mode, tau_bar=phys.tau_bar, mu_ref=phys.mu_ref,
                   T_ref=phys.T_ref, mu_exp=phys.mu_exp, force=tuple(phys.force), Pr=getattr(phys, "Pr", 1.0))
        for k, v in kw.items():
            setattr(p, k, v)
        return p


# ------------------------------------------------------------------ C-ABI mirrors

def sllbm_velset_gauss_hermite(dim: int, n_per_dim: int = 5, T0: float = 1.0):
    Q = n_per_dim ** dim
    zeta = np.zeros(Q * dim)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    _check(_lib.sllbm_velset_gauss_hermite(dim, n_per_dim, ctypes.c_double(T0), _np_ptr(zeta), _np_ptr(w),
                                           _np_ptr(opp, ctypes.POINTER(ctypes.c_int32))), "sllbm_velset_gauss_hermite")
    return {"dim": dim, "Q": Q, "zeta": zeta.reshape(Q, dim), "w": w, "opposite": opp, "T0": T0}


def sllbm_velset_cubature(dim: int, T0: float = 1.0):
    """Reduced degree-9 set D2Q19 (dim 2) or D3Q45 (dim 3), same dict as the product rule's."""
    Q = ctypes.c_int(0)
    _check(_lib.sllbm_velset_cubature(dim, ctypes.c_double(T0), ctypes.byref(Q), None, None, None),
           "sllbm_velset_cubature")
    q = Q.value
    zeta = np.zeros(q * dim)
    w = np.zeros(q)
    opp = np.zeros(q, dtype=np.int32)
    _check(_lib.sllbm_velset_cubature(dim, ctypes.c_double(T0), ctypes.byref(Q), _np_ptr(zeta), _np_ptr(w),
                                      _np_ptr(opp, ctypes.POINTER(ctypes.c_int32))), "sllbm_velset_cubature")
    return {"dim": dim, "Q": q, "zeta": zeta.reshape(q, dim), "w": w, "opposite": opp, "T0": T0}


def _bcs_array(bcs):
    arr = (sllbm_bc * max(1, len(bcs)))()
    for b, bc in enumerate(bcs):
        arr[b].kind = bc.kind
        arr[b].rho = bc.rho
        u = list(bc.u) + [0.0, 0.0, 0.0]
        for a in range(3):
            arr[b].u[a] = u[a]
        arr[b].T = bc.T
        arr[b].T_wall = bc.T_wall
    return arr


def sllbm_mesh_build(mesh) -> Mesh:
    """mesh: a tensor description with attributes dim, p, nodes, ncell, edges, face_bc, bcs
    (workloads.TensorMesh), or a curvilinear one with node_xyz, cell_nodes, cell_face_bc."""
    d = sllbm_mesh_desc()
    d.dim, d.order_p, d.nodes = mesh.dim, mesh.p, SLLBM_NODES[mesh.nodes]
    keep = []
    if hasattr(mesh, "cell_nodes"):
        d.kind = SLLBM_MESH_CURVILINEAR
        xyz = np.ascontiguousarray(mesh.node_xyz, dtype=np.float64)
        cn = np.ascontiguousarray(mesh.cell_nodes, dtype=np.int64)
        fb = np.ascontiguousarray(mesh.cell_face_bc, dtype=np.int32)
        keep += [xyz, cn, fb]
        d.n_nodes = xyz.shape[0]
        d.node_xyz = _np_ptr(xyz)
        d.n_cells = cn.shape[0]
        d.cell_nodes = _np_ptr(cn, ctypes.POINTER(ctypes.c_int64))
        d.cell_face_bc = _np_ptr(fb, ctypes.POINTER(ctypes.c_int32))
    else:
        d.kind = SLLBM_MESH_TENSOR
        for a in range(mesh.dim):
            e = np.ascontiguousarray(mesh.edges[a], dtype=np.float64)
            keep.append(e)
            d.ncell[a] = mesh.ncell[a]
            d.edges[a] = _np_ptr(e)
            d.face_bc[a][0], d.face_bc[a][1] = mesh.face_bc[a]
    bcs = _bcs_array(mesh.bcs)
    d.n_bc = len(mesh.bcs)
    d.bcs = ctypes.cast(bcs, ctypes.POINTER(sllbm_bc))
    h = ctypes.c_void_p()
    _check(_lib.sllbm_mesh_build(ctypes.byref(d), ctypes.byref(h)), "sllbm_mesh_build")
    return Mesh(h, mesh.dim)


def sllbm_mesh_nodes(m: Mesh) -> np.ndarray:
    n = ctypes.c_int64()
    _check(_lib.sllbm_mesh_nodes(m.handle, ctypes.byref(n), None), "sllbm_mesh_nodes")
    xyz = np.zeros((n.value, m.dim))
    _check(_lib.sllbm_mesh_nodes(m.handle, ctypes.byref(n), _np_ptr(xyz)), "sllbm_mesh_nodes")
    return xyz


def sllbm_mesh_volumes(m: Mesh) -> np.ndarray:
    n = ctypes.c_int64()
    _check(_lib.sllbm_mesh_nodes(m.handle, ctypes.byref(n), None), "sllbm_mesh_nodes")
    v = np.zeros(n.value)
    _check(_lib.sllbm_mesh_volumes(m.handle, _np_ptr(v)), "sllbm_mesh_volumes")
    return v


def sllbm_interp_plan(m: Mesh, velset: dict, dt: float, prec: int = SLLBM_F64) -> Plan:
    zeta = np.ascontiguousarray(velset["zeta"], dtype=np.float64)
    w = np.ascontiguousarray(velset["w"], dtype=np.float64)
    opp = np.ascontiguousarray(velset["opposite"], dtype=np.int32)
    v = sllbm_velset(dim=velset["dim"], Q=velset["Q"], zeta=_np_ptr(zeta), w=_np_ptr(w),
                     opposite=_np_ptr(opp, ctypes.POINTER(ctypes.c_int32)), T0=velset["T0"])
    h = ctypes.c_void_p()
    _check(_lib.sllbm_interp_plan(m.handle, ctypes.byref(v), ctypes.c_double(dt), ctypes.c_int(prec),
                                  ctypes.byref(h)), "sllbm_interp_plan")
    return Plan(h, m, velset, dt, prec)


def sllbm_plan_select_kernel(plan: Plan, kernel: int) -> None:
    """0 automatic, 1 per-node gather kernel, 2 LDS-tiled kernel, 3 LDS-tiled kernel with
    velocity-split 3D steps (3D plans periodic along z on a 45- or 125-velocity set)."""
    _check(_lib.sllbm_plan_select_kernel(plan.handle, ctypes.c_int(kernel)), "sllbm_plan_select_kernel")


def sllbm_plan_profile(plan: Plan, enable: bool) -> None:
    """Start (clearing the counters) or stop per-kernel event timing of this plan."""
    _check(_lib.sllbm_plan_profile(plan.handle, ctypes.c_int(1 if enable else 0)), "sllbm_plan_profile")


def sllbm_plan_profile_read(plan: Plan) -> dict:
    """{kernel name: (total milliseconds, launches)} since profiling was enabled."""
    cap = 32
    names = (ctypes.c_char * 32 * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    n = _lib.sllbm_plan_profile_read(plan.handle, ctypes.c_int(cap), names, ms, cnt)
    if n < 0:
        raise SllbmError(n, "sllbm_plan_profile_read")
    return {bytes(names[k]).split(b"\0", 1)[0].decode(): (ms[k], cnt[k]) for k in range(min(n, cap))}


def sllbm_plan_info(plan: Plan) -> dict:
    info = sllbm_plan_info_t()
    _check(_lib.sllbm_plan_info(plan.handle, ctypes.byref(info)), "sllbm_plan_info")
    return {k: getattr(info, k) for k, _ in sllbm_plan_info_t._fields_}


def _dev_ptr(t, dtype=None, numel=None, what="tensor"):
    """Data pointer of a contiguous CUDA (HIP) tensor, checked for dtype and size."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _pop_dtype(plan):
    import torch
    return torch.float32 if plan.prec == SLLBM_F32 else torch.float64


def sllbm_init_equilibrium(plan: Plan, params: Params, rho, u, T, pop, stream=None):
    import torch
    N, D = plan.N, plan.dim
    _check(_lib.sllbm_init_equilibrium(plan.handle, ctypes.byref(params.c()),
                                       _dev_ptr(rho, torch.float64, N, "rho"), _dev_ptr(u, torch.float64, D * N, "u"),
                                       _dev_ptr(T, torch.float64, N, "T"),
                                       _dev_ptr(pop, _pop_dtype(plan), 2 * plan.Q * N, "pop"), _stream(stream)),
           "sllbm_init_equilibrium")


def sllbm_step(plan: Plan, params: Params, pop_in, pop_out, stream=None):
    n = 2 * plan.Q * plan.N
    dt = _pop_dtype(plan)
    _check(_lib.sllbm_step(plan.handle, ctypes.byref(params.c()), _dev_ptr(pop_in, dt, n, "pop_in"),
                           _dev_ptr(pop_out, dt, n, "pop_out"), _stream(stream)), "sllbm_step")


def sllbm_moments(plan: Plan, params: Params, pop, rho=None, u=None, T=None, totals: bool = False, stream=None):
    """Writes rho [N], u [dim][N], T [N] (each optional); returns the totals
    [mass, momentum..., energy] as a numpy array when totals=True (synchronising)."""
    import torch
    N, D = plan.N, plan.dim
    tot = np.zeros(2 + D) if totals else None
    _check(_lib.sllbm_moments(plan.handle, ctypes.byref(params.c()),
                              _dev_ptr(pop, _pop_dtype(plan), 2 * plan.Q * N, "pop"),
                              _dev_ptr(rho, torch.float64, N, "rho"), _dev_ptr(u, torch.float64, D * N, "u"),
                              _dev_ptr(T, torch.float64, N, "T"),
                              _np_ptr(tot) if totals else None, _stream(stream)), "sllbm_moments")
    return tot


def sllbm_moments_noalloc(plan: Plan, params: Params, pop, rho=None, u=None, T=None, totals: bool = False,
                          stream=None):
    """sllbm_moments with its reduction scratch in the library's fixed per-GPU array (no
    device allocation; plans of at most 2^25 nodes; overlapping calls on one GPU race)."""
    import torch
    N, D = plan.N, plan.dim
    tot = np.zeros(2 + D) if totals else None
    _check(_lib.sllbm_moments_noalloc(plan.handle, ctypes.byref(params.c()),
                                      _dev_ptr(pop, _pop_dtype(plan), 2 * plan.Q * N, "pop"),
                                      _dev_ptr(rho, torch.float64, N, "rho"), _dev_ptr(u, torch.float64, D * N, "u"),
                                      _dev_ptr(T, torch.float64, N, "T"),
                                      _np_ptr(tot) if totals else None, _stream(stream)), "sllbm_moments_noalloc")
    return tot


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = []      # the callbacks must outlive every object created with them


def sllbm_set_allocator(alloc=None, release=None):
    """alloc(nbytes) -> int device pointer (0 on failure), release(ptr); both None restores
    hipMalloc / hipFree.  Objects created afterwards allocate through them."""
    if alloc is None and release is None:
        _check(_lib.sllbm_set_allocator(None, None, None), "sllbm_set_allocator")
        return
    a = _ALLOC_FN(lambda n, ctx: alloc(int(n)) or None)
    r = _RELEASE_FN(lambda p, ctx: release(int(p)))
    _allocator_refs.append((a, r))
    _check(_lib.sllbm_set_allocator(a, r, None), "sllbm_set_allocator")


def use_torch_allocator():
    """Device memory of objects created afterwards comes from torch's caching allocator."""
    import torch
    sllbm_set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n), torch.cuda.caching_allocator_delete)


def sllbm_force_reset(plan: Plan, force0, stream=None):
    f = np.zeros(3)
    f[:len(force0)] = force0
    _check(_lib.sllbm_force_reset(plan.handle, _np_ptr(f), _stream(stream)), "sllbm_force_reset")


def sllbm_force_update(plan: Plan, pop, axis: int, target: float, kp: float, ki: float, dt: float, stream=None):
    c = sllbm_force_ctl(axis=int(axis), target=float(target), kp=float(kp), ki=float(ki), dt=float(dt))
    _check(_lib.sllbm_force_update(plan.handle, ctypes.byref(c), _dev_ptr(pop, _pop_dtype(plan), 2 * plan.Q * plan.N,
                                                                         "pop"), _stream(stream)), "sllbm_force_update")


def sllbm_force_read(plan: Plan, stream=None) -> dict:
    h = np.zeros(7)
    _check(_lib.sllbm_force_read(plan.handle, _np_ptr(h), _stream(stream)), "sllbm_force_read")
    return {"force": h[:3].copy(), "integral": h[3], "error": h[4], "mean_momentum": h[5], "updates": int(h[6])}


# ------------------------------------------------------------------ learned correction

for _name in ("sllbm_mlp_create", "sllbm_mlp_num_params", "sllbm_mlp_get_params", "sllbm_mlp_set_params",
              "sllbm_features", "sllbm_mlp_forward", "sllbm_mlp_correct", "sllbm_step_learned", "sllbm_learned_targets", "sllbm_restrict",
              "sllbm_mlp_gradient", "sllbm_mlp_train_step"):
    getattr(_lib, _name).restype = ctypes.c_int
_lib.sllbm_mlp_destroy.restype = None


class Mlp:
    """Owner of an sllbm_mlp handle (a network of n_in -> 64 -> 64 -> 64 -> n_out)."""

    def __init__(self, handle, n_in, n_out):
        self._lib = _lib
        self.handle = handle
        self.n_in, self.n_out = n_in, n_out
        n = ctypes.c_int64(0)
        _check(_lib.sllbm_mlp_num_params(handle, ctypes.byref(n)), "sllbm_mlp_num_params")
        self.nparam = n.value

    def __del__(self):
        lib = getattr(self, "_lib", None)
        if getattr(self, "handle", None) and lib is not None:
            lib.sllbm_mlp_destroy(self.handle)
            self.handle = None


def sllbm_mlp_create(n_in: int, n_out: int, seed: int = 0, width: int = 64, depth: int = 3) -> Mlp:
    h = ctypes.c_void_p()
    _check(_lib.sllbm_mlp_create(ctypes.c_int(n_in), ctypes.c_int(width), ctypes.c_int(depth), ctypes.c_int(n_out),
                                 ctypes.c_uint64(seed), ctypes.byref(h)), "sllbm_mlp_create")
    return Mlp(h, n_in, n_out)


def sllbm_mlp_get_params(m: Mlp) -> np.ndarray:
    out = np.zeros(m.nparam, dtype=np.float32)
    _check(_lib.sllbm_mlp_get_params(m.handle, out.ctypes.data_as(ctypes.c_void_p)), "sllbm_mlp_get_params")
    return out


def sllbm_mlp_set_params(m: Mlp, theta) -> None:
    a = np.ascontiguousarray(theta, dtype=np.float32)
    if a.size != m.nparam:
        raise ValueError(f"need {m.nparam} parameters, got {a.size}")
    _check(_lib.sllbm_mlp_set_params(m.handle, a.ctypes.data_as(ctypes.c_void_p)), "sllbm_mlp_set_params")


def n_features(dim: int) -> int:
    return (dim + 2) * (dim + 1)


def sllbm_features(plan: Plan, params: Params, pop, feat, stream=None):
    """feat: torch.bfloat16 [N, n_features(dim)] on the GPU."""
    import torch
    _check(_lib.sllbm_features(plan.handle, ctypes.byref(params.c()),
                               _dev_ptr(pop, _pop_dtype(plan), 2 * plan.Q * plan.N, "pop"),
                               _dev_ptr(feat, torch.bfloat16, plan.N * n_features(plan.dim), "feat"), _stream(stream)),
           "sllbm_features")


def sllbm_mlp_forward(m: Mlp, x, y, stream=None):
    """x: torch.bfloat16 [rows, n_in]; y: torch.float32 [rows, n_out]."""
    import torch
    rows = x.shape[0]
    _check(_lib.sllbm_mlp_forward(m.handle, _dev_ptr(x, torch.bfloat16, rows * m.n_in, "x"), ctypes.c_int64(rows),
                                  _dev_ptr(y, torch.float32, rows * m.n_out, "y"), _stream(stream)), "sllbm_mlp_forward")


def sllbm_mlp_correct(plan: Plan, params: Params, m: Mlp, pop, stream=None):
    _check(_lib.sllbm_mlp_correct(plan.handle, ctypes.byref(params.c()), m.handle,
                                  _dev_ptr(pop, _pop_dtype(plan), 2 * plan.Q * plan.N, "pop"), _stream(stream)),
           "sllbm_mlp_correct")


def sllbm_step_learned(plan: Plan, params: Params, m: Mlp, pop_in, pop_out, stream=None):
    """One step with the learned correction (sllbm_step then sllbm_mlp_correct; on 3D tiled
    plans the relaxation and the correction in one pass)."""
    n = 2 * plan.Q * plan.N
    _check(_lib.sllbm_step_learned(plan.handle, ctypes.byref(params.c()), m.handle,
                                   _dev_ptr(pop_in, _pop_dtype(plan), n, "pop_in"),
                                   _dev_ptr(pop_out, _pop_dtype(plan), n, "pop_out"), _stream(stream)),
           "sllbm_step_learned")


def sllbm_learned_targets(plan: Plan, pop_plain, pop_true, t, stream=None):
    """t: torch.float32 [N, 2Q]."""
    import torch
    n = 2 * plan.Q * plan.N
    dt = _pop_dtype(plan)
    _check(_lib.sllbm_learned_targets(plan.handle, _dev_ptr(pop_plain, dt, n, "pop_plain"),
                                      _dev_ptr(pop_true, dt, n, "pop_true"), _dev_ptr(t, torch.float32, n, "t"),
                                      _stream(stream)), "sllbm_learned_targets")


def sllbm_restrict(fine: Plan, coarse: Plan, ratio: int, pop_fine, pop_coarse, stream=None):
    dt = _pop_dtype(coarse)
    _check(_lib.sllbm_restrict(fine.handle, coarse.handle, ctypes.c_int(ratio),
                               _dev_ptr(pop_fine, dt, 2 * fine.Q * fine.N, "pop_fine"),
                               _dev_ptr(pop_coarse, dt, 2 * coarse.Q * coarse.N, "pop_coarse"), _stream(stream)),
           "sllbm_restrict")


def sllbm_mlp_gradient(m: Mlp, x, t, stream=None):
    """(gradient as float32 numpy [nparam], mean-square loss) over the rows of x, t."""
    import torch
    rows = x.shape[0]
    g = np.zeros(m.nparam, dtype=np.float32)
    loss = ctypes.c_float(0)
    _check(_lib.sllbm_mlp_gradient(m.handle, _dev_ptr(x, torch.bfloat16, rows * m.n_in, "x"),
                                   _dev_ptr(t, torch.float32, rows * m.n_out, "t"), ctypes.c_int64(rows),
                                   g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss), _stream(stream)),
           "sllbm_mlp_gradient")
    return g, loss.value


def sllbm_mlp_train_step(m: Mlp, x, t, lr: float, want_loss: bool = True, stream=None):
    import torch
    rows = x.shape[0]
    loss = ctypes.c_float(0)
    _check(_lib.sllbm_mlp_train_step(m.handle, _dev_ptr(x, torch.bfloat16, rows * m.n_in, "x"),
                                     _dev_ptr(t, torch.float32, rows * m.n_out, "t"), ctypes.c_int64(rows),
                                     ctypes.c_float(lr), ctypes.byref(loss) if want_loss else None, _stream(stream)),
           "sllbm_mlp_train_step")
    return loss.value if want_loss else None


__all__ = ["sllbm_velset_gauss_hermite", "sllbm_velset_cubature", "sllbm_mesh_build", "sllbm_mesh_nodes", "sllbm_mesh_volumes",
           "sllbm_interp_plan", "sllbm_plan_info", "sllbm_plan_select_kernel", "sllbm_init_equilibrium", "sllbm_step", "sllbm_moments",
           "sllbm_moments_noalloc", "sllbm_force_reset", "sllbm_force_update", "sllbm_force_read", "sllbm_set_allocator", "use_torch_allocator",
           "Params", "Plan", "Mesh", "SllbmError", "SLLBM_F64", "SLLBM_F32", "LIB_PATH",
           "Mlp", "sllbm_mlp_create", "sllbm_mlp_get_params", "sllbm_mlp_set_params", "sllbm_features",
           "sllbm_mlp_forward", "sllbm_mlp_correct", "sllbm_step_learned", "sllbm_learned_targets", "sllbm_restrict", "sllbm_mlp_gradient",
           "sllbm_mlp_train_step", "n_features"]
