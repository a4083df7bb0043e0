"""sllbm_moments_noalloc (the allocation-free variant of sllbm_moments) through the C-ABI
against sllbm_moments: two calls in a row on one GPU, the second on a smaller plan, each
checked field by field and on the totals.  Both entry points run the same kernels in the
same reduction order, so the results must agree bit for bit."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(mesh, phys, prec, fields):
    import torch
    import paper_2412_09051_amd as S
    m = S.sllbm_mesh_build(mesh)
    plan = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(mesh.dim, 5, phys.T0), phys.dt, prec)
    prm = S.Params.from_physics(phys)
    rho, u, T = fields(S.sllbm_mesh_nodes(m))
    dt = torch.float32 if prec == S.SLLBM_F32 else torch.float64
    pop = torch.empty(2 * plan.Q * plan.N, dtype=dt, device="cuda")
    S.sllbm_init_equilibrium(plan, prm, torch.tensor(rho, device="cuda"),
                             torch.tensor(np.ascontiguousarray(u.T), device="cuda"), torch.tensor(T, device="cuda"), pop)
    # one step, so that the fields are not exactly the initial ones
    out = torch.empty_like(pop)
    S.sllbm_step(plan, prm, pop, out)
    return m, plan, prm, out


def _both(plan, prm, pop):
    import torch
    import paper_2412_09051_amd as S
    N, D = plan.N, plan.dim
    res = []
    for fn in (S.sllbm_moments, S.sllbm_moments_noalloc):
        r = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        u = torch.full((D * N,), float("nan"), dtype=torch.float64, device="cuda")
        T = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        tot = fn(plan, prm, pop, r, u, T, totals=True)
        torch.cuda.synchronize()
        res.append((r.cpu().numpy(), u.cpu().numpy(), T.cpu().numpy(), tot))
    return res


def test_noalloc_moments_equal_moments_on_two_calls_in_a_row():
    import paper_2412_09051_amd as S
    big = _plan(*W.tgv_case(ncell=12, p=3), S.SLLBM_F64, W.tgv_fields)                # 46,656 nodes, 183 blocks
    small = _plan(*W.shear_wave_case(ncell=5, p=3), S.SLLBM_F32,
                  lambda x: W.shear_wave_fields(x, noise=1e-3, seed=3))               # 225 nodes, 1 block
    for name, (_, plan, prm, pop) in (("tgv 36^3 f64", big), ("shear 15^2 f32", small)):
        ref, got = _both(plan, prm, pop)
        say(name, "nodes", plan.N, "totals", ref[3], got[3])
        for a, b in zip(ref[:3], got[:3]):
            assert np.all(np.isfinite(a)) and np.array_equal(a, b)
        assert np.array_equal(ref[3], got[3])
    # fields only (no totals): the reduction is skipped, the fields are the same
    _, plan, prm, pop = big
    import torch
    r = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    S.sllbm_moments_noalloc(plan, prm, pop, r)
    r2 = torch.zeros_like(r)
    S.sllbm_moments(plan, prm, pop, r2)
    torch.cuda.synchronize()
    assert torch.equal(r, r2)


def test_noalloc_moments_reports_bad_nodes_like_moments():
    """A population set with a negative density at one node: both entry points return
    SLLBM_EUNSTABLE, after writing the same totals."""
    import torch
    import paper_2412_09051_amd as S
    _, plan, prm, pop = _plan(*W.shear_wave_case(ncell=4, p=2), S.SLLBM_F64, lambda x: W.shear_wave_fields(x))
    bad = pop.clone()
    for i in range(plan.Q):
        bad[i * plan.N + 5] = -bad[i * plan.N + 5]
    codes = []
    for fn in (S.sllbm_moments, S.sllbm_moments_noalloc):
        with pytest.raises(S.SllbmError) as e:
            fn(plan, prm, bad, totals=True)
        codes.append(e.value.code)
    assert codes == [S.SLLBM_EUNSTABLE, S.SLLBM_EUNSTABLE]


def test_noalloc_moments_refuses_plans_beyond_its_scratch():
    """2^25 nodes is the limit; a 6000 x 6000-node plan is refused before any launch (the
    population pointer is never read)."""
    import torch
    import paper_2412_09051_amd as S
    mesh, phys = W.shear_wave_case(ncell=1500, p=4)
    m = S.sllbm_mesh_build(mesh)
    plan = S.sllbm_interp_plan(m, S.sllbm_velset_gauss_hermite(2, 5, phys.T0), phys.dt, S.SLLBM_F32)
    assert plan.N == 6000 * 6000 > (1 << 25)
    prm = S.Params.from_physics(phys)
    dummy = torch.zeros(64, dtype=torch.float32, device="cuda")
    tot = np.zeros(4)
    rc = S._lib.sllbm_moments_noalloc(plan.handle, ctypes.byref(prm.c()), ctypes.c_void_p(dummy.data_ptr()), None,
                                      None, None, tot.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    assert rc == S.SLLBM_EINVAL
    assert "exceed" in S._lib.sllbm_last_error().decode()
