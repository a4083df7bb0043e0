"""C-ABI checks that need no GPU: the library loads, exports every function that
include/sllbm.h declares, validates its arguments before touching a device, and its
host-side geometry (velocity set, support points, node coordinates, nodal volumes,
boundary-layer classification) agrees with the oracle's independent setup."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
import paper_2412_09051_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "sllbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sllbm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(S.LIB_PATH)
    names = header_functions()
    assert "sllbm_step" in names and "sllbm_interp_plan" in names and "sllbm_moments" in names
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("dim", [2, 3])
def test_velocity_set_matches_oracle(dim):
    v = S.sllbm_velset_gauss_hermite(dim, 5, 1.3)
    z, w, o = oracle.velocity_set(dim, 5, 1.3)
    assert np.max(np.abs(v["zeta"] - z)) < 1e-14 and np.max(np.abs(v["w"] - w)) < 1e-15
    assert np.array_equal(v["opposite"], o)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("T0", [1.0, 1.3])
def test_cubature_set_matches_oracle(dim, T0):
    """The library's closed forms against the oracle's rule solved from the moment conditions,
    index by index (the oracle's solve carries ~1e-14 relative error in the outer radius: its
    degree-6 orbit averages are small differences of O(0.1) numbers)."""
    v = S.sllbm_velset_cubature(dim, T0)
    z, w, o = oracle.cubature_set(dim, T0)
    assert v["Q"] == len(w) == (19 if dim == 2 else 45)
    assert np.max(np.abs(v["zeta"] - z)) < 5e-14 and np.max(np.abs(v["w"] - w)) < 1e-15
    assert np.array_equal(v["opposite"], o)
    assert np.array_equal(v["zeta"][v["opposite"]], -v["zeta"])


def test_cubature_set_arguments():
    lib = ctypes.CDLL(S.LIB_PATH)
    q = ctypes.c_int(0)
    z = (ctypes.c_double * 135)()
    assert lib.sllbm_velset_cubature(3, ctypes.c_double(1.0), ctypes.byref(q), None, None, None) == 0 and q.value == 45
    assert lib.sllbm_velset_cubature(1, ctypes.c_double(1.0), ctypes.byref(q), None, None, None) == S.SLLBM_EINVAL
    assert lib.sllbm_velset_cubature(2, ctypes.c_double(0.0), ctypes.byref(q), None, None, None) == S.SLLBM_EINVAL
    assert lib.sllbm_velset_cubature(2, ctypes.c_double(1.0), None, None, None, None) == S.SLLBM_EINVAL
    assert lib.sllbm_velset_cubature(3, ctypes.c_double(1.0), ctypes.byref(q), z, None, None) == S.SLLBM_EINVAL


@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_gauss_hermite_roots_match_numpy_rule(n):
    v = S.sllbm_velset_gauss_hermite(1 + 1, n, 1.0)
    x = np.unique(np.round(v["zeta"][:, 0], 14))
    xs, ws = oracle.gauss_hermite_1d(n)
    assert np.allclose(np.sort(x), xs, atol=1e-13)


def _meshes():
    yield W.shear_wave_case(ncell=5, p=4, nodes="glc")[0]
    yield W.tgv_case(ncell=3, p=3)[0]
    yield W.channel_case(ncell=(3, 5, 2), p=2, box=(1.0, 2.0, 1.0))[0]
    yield W.TensorMesh(dim=2, p=3, nodes="equi", ncell=(4, 3), edges=[np.array([0, .2, .5, .9, 1.4]),
                                                                       np.array([-1, 0, .3, .4])],
                       face_bc=[[-1, -1], [0, 1]], bcs=[W.BC(kind=W.BC_INLET), W.BC(kind=W.BC_OUTLET)])


@pytest.mark.parametrize("idx", range(4))
def test_nodes_and_volumes_match_oracle(idx):
    mesh = list(_meshes())[idx]
    m = S.sllbm_mesh_build(mesh)
    o = oracle.TensorOracle(mesh, W.Physics(dt=0.01))
    assert np.max(np.abs(S.sllbm_mesh_nodes(m) - o.coords())) < 1e-13
    assert np.max(np.abs(S.sllbm_mesh_volumes(m) - o.node_vol)) < 1e-14


def test_mesh_validation_errors():
    good = W.shear_wave_case(ncell=4, p=2)[0]
    import copy
    bad = copy.deepcopy(good)
    bad.edges[0] = np.array([0.0, 1.0, 0.5, 2.0, 3.0])
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_mesh_build(bad)
    assert e.value.code == S.SLLBM_EINVAL and "increasing" in str(e.value)
    bad = copy.deepcopy(good)
    bad.face_bc = [[-1, 0], [-1, -1]]
    bad.bcs = [W.BC(kind=W.BC_WALL)]
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_mesh_build(bad)
    assert e.value.code == S.SLLBM_EINVAL
    bad = copy.deepcopy(good)
    bad.p = 9
    with pytest.raises(S.SllbmError):
        S.sllbm_mesh_build(bad)


def test_two_bounded_axes_are_unsupported_on_tensor_meshes():
    mesh = W.TensorMesh(dim=2, p=2, nodes="gll", ncell=(3, 3), edges=[W.uniform_edges(3, 0, 1)] * 2,
                        face_bc=[[0, 0], [0, 0]], bcs=[W.BC(kind=W.BC_WALL)])
    m = S.sllbm_mesh_build(mesh)
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(2), 0.01)
    assert e.value.code == S.SLLBM_EUNSUPPORTED


def test_reflected_departure_point_leaving_again_is_projected():
    """A channel thinner than the path: the reflected point leaves through the other wall
    and is taken at its nearest boundary point; the plan builds and counts every pair."""
    mesh = W.TensorMesh(dim=2, p=2, nodes="gll", ncell=(3, 1), edges=[W.uniform_edges(3, 0, 1), np.array([0.0, 0.05])],
                        face_bc=[[-1, -1], [0, 0]], bcs=[W.BC(kind=W.BC_WALL)])
    m = S.sllbm_mesh_build(mesh)
    plan = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(2), 0.1)
    info = S.sllbm_plan_info(plan)
    y = S.sllbm_mesh_nodes(m)[:, 1]
    zy = S.sllbm_velset_gauss_hermite(2)["zeta"][:, 1]
    leaves = sum(int(np.sum((y - 0.1 * z < 0) | (y - 0.1 * z > 0.05))) for z in zy)
    assert info["n_exceptions"] == leaves


def test_curvilinear_plan_on_the_airfoil_grid():
    """The CSR plan of a small O-grid builds without a GPU; its thermal-wall nodes are
    the oracle's."""
    mesh, phys = W.naca_ogrid(n_around=48, n_radial=16, p=4, Ma=1.5)
    m = S.sllbm_mesh_build(mesh)
    assert np.max(np.abs(S.sllbm_mesh_nodes(m) - mesh.node_xyz)) == 0.0
    plan = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(2), phys.dt)
    info = S.sllbm_plan_info(plan)
    assert info["kernel"] == 1 and info["n_nodes"] == mesh.node_xyz.shape[0]
    o = oracle.CurvOracle(mesh, phys)
    assert info["n_thermal_nodes"] == int(np.sum(o.g_th >= 0))
    assert np.max(np.abs(S.sllbm_mesh_volumes(m) - o.node_vol)) < 1e-13 * o.node_vol.max()


def test_curvilinear_mesh_validation_errors():
    mesh, _ = W.naca_ogrid(n_around=16, n_radial=4, p=2)
    import copy
    bad = copy.deepcopy(mesh)
    bad.cell_nodes = bad.cell_nodes.copy()
    bad.cell_nodes[3, 2] = mesh.node_xyz.shape[0] + 5
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_mesh_build(bad)
    assert e.value.code == S.SLLBM_EINVAL
    bad = copy.deepcopy(mesh)
    bad.cell_face_bc = bad.cell_face_bc.copy()
    bad.cell_face_bc[0, 2] = 7
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_mesh_build(bad)
    assert e.value.code == S.SLLBM_EINVAL


def test_plan_info_without_gpu_counts_boundary_pairs():
    mesh, phys = W.channel_case(ncell=(4, 6, 4), p=2, box=(1.0, 2.0, 1.0))
    m = S.sllbm_mesh_build(mesh)
    plan = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(3), phys.dt)
    info = S.sllbm_plan_info(plan)
    # count the boundary pairs independently: nodes whose departure point leaves [0, 2] in y
    o = oracle.TensorOracle(mesh, phys)
    xyz = o.coords()
    y = xyz[:, 1]
    n = 0
    nth = 0
    for i in range(o.Q):
        yd = y - phys.dt * o.zeta[i, 1]
        n += int(np.sum((yd < 0) | (yd > 2.0)))
    thermal = np.zeros(o.N, bool)
    for i in range(o.Q):
        yd = y - phys.dt * o.zeta[i, 1]
        thermal |= (yd < 0) | (yd > 2.0)
    assert info["n_exceptions"] == n
    assert info["n_thermal_nodes"] == int(thermal.sum())
    if not info["has_device"]:
        assert info["table_bytes"] == 0


def _fake_ptr(addr):
    return ctypes.c_void_p(addr)


def test_step_argument_validation_before_any_launch():
    mesh, phys = W.shear_wave_case(ncell=4, p=2)
    m = S.sllbm_mesh_build(mesh)
    plan = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(2), phys.dt)
    lib = S._lib
    prm = S.Params.from_physics(phys)
    n_bytes = 2 * plan.Q * plan.N * 8
    a, b = 1 << 20, (1 << 20) + 4 * n_bytes   # never dereferenced: validation fails first
    for pr in (0.0, -0.7, float("inf"), float("nan")):
        bad = S.Params.from_physics(phys, Pr=pr)
        assert lib.sllbm_step(plan.handle, ctypes.byref(bad.c()), _fake_ptr(a), _fake_ptr(b), None) == S.SLLBM_EINVAL
        assert "Pr" in lib.sllbm_last_error().decode()
    assert lib.sllbm_step(plan.handle, ctypes.byref(prm.c()), _fake_ptr(a), _fake_ptr(a + 64), None) == S.SLLBM_EINVAL
    assert "overlap" in lib.sllbm_last_error().decode()
    assert lib.sllbm_step(plan.handle, ctypes.byref(prm.c()), _fake_ptr(a + 4), _fake_ptr(b), None) == S.SLLBM_EINVAL
    assert lib.sllbm_step(plan.handle, ctypes.byref(prm.c()), None, _fake_ptr(b), None) == S.SLLBM_EINVAL
    tau = S.Params.from_physics(phys, tau_bar=0.4)
    assert lib.sllbm_step(plan.handle, ctypes.byref(tau.c()), _fake_ptr(a), _fake_ptr(b), None) == S.SLLBM_EINVAL
    assert lib.sllbm_step(None, ctypes.byref(prm.c()), _fake_ptr(a), _fake_ptr(b), None) == S.SLLBM_EINVAL
    if not S.sllbm_plan_info(plan)["has_device"]:
        assert lib.sllbm_step(plan.handle, ctypes.byref(prm.c()), _fake_ptr(a), _fake_ptr(b), None) == S.SLLBM_EHIP
    # the controlled force must be set before a step or an update uses it
    fd = S.Params.from_physics(phys, force_device=1)
    assert lib.sllbm_step(plan.handle, ctypes.byref(fd.c()), _fake_ptr(a), _fake_ptr(b), None) == S.SLLBM_EINVAL
    assert "sllbm_force_reset" in lib.sllbm_last_error().decode()
    ctl = S.sllbm_force_ctl(axis=0, target=1.0, kp=1.0, ki=0.0, dt=0.1)
    assert lib.sllbm_force_update(plan.handle, ctypes.byref(ctl), _fake_ptr(a), None) == S.SLLBM_EINVAL
    state = (ctypes.c_double * 7)()
    assert lib.sllbm_force_read(plan.handle, state, None) == S.SLLBM_EINVAL
    assert lib.sllbm_force_reset(plan.handle, None, None) == S.SLLBM_EINVAL
    bad_fd = S.Params.from_physics(phys, force_device=2)
    assert lib.sllbm_step(plan.handle, ctypes.byref(bad_fd.c()), _fake_ptr(a), _fake_ptr(b), None) == S.SLLBM_EINVAL


def test_tiled_kernel_eligibility_follows_the_halo_rule():
    """The LDS-tiled kernel applies when every departure stencil stays within one cell
    of its node (CFL <= 1 on the cell) and the periodic axes are longer than a tile; the
    automatic choice takes it from 256 tiles (one per compute unit) on."""
    mesh, phys = W.tgv_case(ncell=8, p=3)
    m = S.sllbm_mesh_build(mesh)
    vs = S.sllbm_velset_gauss_hermite(3)

    def tiled(plan):
        try:
            S.sllbm_plan_select_kernel(plan, 2)
        except S.SllbmError as e:
            assert e.code == S.SLLBM_EUNSUPPORTED
            return False
        return S.sllbm_plan_info(plan)["kernel"] == 2

    p8 = S.sllbm_interp_plan(m, vs, phys.dt)
    assert S.sllbm_plan_info(p8)["kernel"] == 0          # 24^3 nodes: 16 tiles, automatic -> gather
    assert tiled(p8)
    h = 2 * math.pi / 8
    big = 1.5 * h / W.ZETA_MAX_GH5            # CFL 1.5: stencils two cells away
    assert not tiled(S.sllbm_interp_plan(m, vs, big))
    small = W.tgv_case(ncell=5, p=3)[0]       # 15 nodes per axis < tile + halo
    assert not tiled(S.sllbm_interp_plan(S.sllbm_mesh_build(small), vs, phys.dt))
    large, physl = W.tgv_case(ncell=24, p=3)  # 72^3 nodes: 432 tiles (periodic: velocity-split steps)
    assert S.sllbm_plan_info(S.sllbm_interp_plan(S.sllbm_mesh_build(large), vs, physl.dt))["kernel"] == 3


def test_velocity_split_step_eligibility():
    """The velocity-split 3D step: 3D plans that the tiled kernel takes
    (the automatic choice from 256 tiles on), periodic along z, walls on x or y allowed, on the
    45- and 125-velocity sets; not D3Q27, not meshes shorter than a 48 x 12-node tile and its halo,
    not 2D."""
    mesh, phys = W.tgv_case(ncell=32, p=3, dt=W.TGV_DT)
    m = S.sllbm_mesh_build(mesh)
    q45 = S.sllbm_interp_plan(m, S.sllbm_velset_cubature(3, phys.T0), phys.dt)
    assert S.sllbm_plan_info(q45)["kernel"] == 3
    S.sllbm_plan_select_kernel(q45, 2)
    assert S.sllbm_plan_info(q45)["kernel"] == 2
    S.sllbm_plan_select_kernel(q45, 3)
    assert S.sllbm_plan_info(q45)["kernel"] == 3
    q32 = S.sllbm_interp_plan(m, S.sllbm_velset_cubature(3, phys.T0), phys.dt, S.SLLBM_F32)
    assert S.sllbm_plan_info(q32)["kernel"] == 3
    v125 = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(3), phys.dt)
    assert S.sllbm_plan_info(v125)["kernel"] == 3
    v27 = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(3, 3), phys.dt)
    assert S.sllbm_plan_info(v27)["kernel"] == 2
    cmesh, cphys = W.channel_case(ncell=(6, 8, 6), p=2, box=(2.0, 2.0, 1.5), cfl=0.75, T_wall=0.9, Ma_b=0.5)
    walls = S.sllbm_interp_plan(S.sllbm_mesh_build(cmesh), S.sllbm_velset_cubature(3, cphys.T0), cphys.dt)
    smesh, sphys = W.shear_wave_case(ncell=16, p=4)
    flat = S.sllbm_interp_plan(S.sllbm_mesh_build(smesh), S.sllbm_velset_cubature(2, sphys.T0), sphys.dt)
    lmesh, lphys = W.channel_case(ncell=(26, 8, 14), p=2, box=(4.0, 2.0, 1.5), cfl=0.75, T_wall=0.9, Ma_b=0.5)
    long_walls = S.sllbm_interp_plan(S.sllbm_mesh_build(lmesh), S.sllbm_velset_cubature(3, lphys.T0), lphys.dt)
    S.sllbm_plan_select_kernel(long_walls, 3)
    assert S.sllbm_plan_info(long_walls)["kernel"] == 3
    for plan in (v27, walls, flat):
        with pytest.raises(S.SllbmError) as e:
            S.sllbm_plan_select_kernel(plan, 3)
        assert e.value.code == S.SLLBM_EUNSUPPORTED
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_plan_select_kernel(q45, 4)
    assert e.value.code == S.SLLBM_EINVAL


def test_profiling_needs_a_device_plan():
    mesh, phys = W.shear_wave_case(ncell=4, p=2)
    plan = S.sllbm_interp_plan(S.sllbm_mesh_build(mesh), S.sllbm_velset_gauss_hermite(2), phys.dt)
    if S.sllbm_plan_info(plan)["has_device"]:
        pytest.skip("a GPU is present")
    with pytest.raises(S.SllbmError) as e:
        S.sllbm_plan_profile(plan, True)
    assert e.value.code == S.SLLBM_EHIP
    assert S.sllbm_plan_profile_read(plan) == {}


def test_header_compiles_as_c(tmp_path):
    """include/sllbm.h is a C header: it compiles on its own with a C compiler."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "sllbm.h"\nint main(void) { return sllbm_last_error() == 0; }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([gcc, "-std=c11", "-Wall", "-Werror", "-I", inc, "-c", str(src), "-o", str(tmp_path / "use.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_set_allocator_needs_both_functions():
    lib = S._lib
    fn = S._ALLOC_FN(lambda n, ctx: None)
    assert lib.sllbm_set_allocator(fn, None, None) == S.SLLBM_EINVAL
    assert "both" in lib.sllbm_last_error().decode()
    assert lib.sllbm_set_allocator(None, None, None) == S.SLLBM_OK
