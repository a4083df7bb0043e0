"""Plans and networks allocate their device memory through the caller's allocator (here
torch's caching allocator) when one is set, give every block back on destroy, and compute
the same step as with the library's own allocations."""
import gc
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from harness import GpuRun, rel_err

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_objects_allocate_through_the_callers_allocator():
    import torch
    import paper_2412_09051_amd as S
    live, counts = set(), {"alloc": 0, "release": 0}

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n)
        live.add(p)
        counts["alloc"] += 1
        return p

    def release(p):
        live.discard(p)
        counts["release"] += 1
        torch.cuda.caching_allocator_delete(p)

    say("case allocator: 2D tiled and 3D tiled plans, a network")
    S.sllbm_set_allocator(alloc, release)
    try:
        runs = []
        for mesh, phys, fields in ((*W.shear_wave_case(ncell=12, p=4), W.shear_wave_fields),
                                   (*W.tgv_case(ncell=6, p=3), W.tgv_fields)):
            o = oracle.TensorOracle(mesh, phys)
            g = GpuRun(mesh, phys, "f64")
            rho, u, T = fields(o.coords())
            g.init(rho, u, T)
            g.run(5)
            e = rel_err(g.pop(), o.run(o.init(rho, u, T), 5))
            say("pop error", e)
            assert e <= 1e-12
            runs.append(g)
        net = S.sllbm_mlp_create(S.n_features(3), 2 * 125, seed=3)
        assert counts["alloc"] > 0 and len(live) > 0
    finally:
        S.sllbm_set_allocator(None, None)
    del runs, g, net
    gc.collect()
    torch.cuda.synchronize()
    say("allocations", counts, "still live", len(live))
    assert not live and counts["release"] == counts["alloc"]
