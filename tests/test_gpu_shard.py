"""Sharded runs: a mesh cut into contiguous ranges of its Morton order, each stepped with its
halo, halos exchanged by the pack/unpack kernels and dt all-reduced by swe_shard_dt_combine,
must reproduce the single-domain run bit for bit (every owned cell computes exactly what it
computes unsharded, and the dt minimum is exact)."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def _single(swe, case, mesh, dtype, steps, **kw):
    s = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype,
                   inflow_q=case.inflow_q, **kw)
    rc, st = s.run(steps)
    return rc, st, s.numpy_state()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant,parts", [("tiled", 4), ("cell", 3), ("tiled", 7)])
def test_sharded_run_equals_single_domain_bitwise(gpu, dtype, variant, parts):
    swe = gpu
    case = gen.small(3)
    mesh = swe.Mesh(case.xy, case.tri)
    steps = 60
    rc0, st0, ref = _single(swe, case, mesh, dtype, steps, variant=variant)
    sh = swe.ShardedSolver(mesh, parts, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype,
                           variant=variant)
    sh.step(steps)
    rc1, st1 = sh.stats()
    got = sh.numpy_state()
    print(f"{dtype} {variant} {parts} shards: halos "
          f"{[m.n_cells - m.n_owned for m in sh.meshes]}, t {st1['t']} vs {st0['t']}")
    assert rc0 == rc1 == swe.SWE_OK
    assert st1["steps"] == st0["steps"] == steps and st1["t"] == st0["t"]
    assert st1["clamps"] == st0["clamps"]
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_exact_sharded_run_equals_single_domain_bitwise(gpu):
    """Correctly rounded FP64 (SWE_EXACT): five shards give the single-domain exact run."""
    swe = gpu
    case = gen.small(3)
    mesh = swe.Mesh(case.xy, case.tri)
    rc0, st0, ref = _single(swe, case, mesh, "f64", 60, variant="tiled", exact=True)
    sh = swe.ShardedSolver(mesh, 5, case.z, case.n, case.h, case.hu, case.hv, dtype="f64",
                           variant="tiled", exact=True)
    sh.step(60)
    rc1, st1 = sh.stats()
    assert rc0 == rc1 == swe.SWE_OK and st1["steps"] == st0["steps"] == 60
    assert st1["t"] == st0["t"]
    for a, b in zip(ref, sh.numpy_state()):
        assert np.array_equal(a, b)


def test_sharded_inflow_and_t_end_match_single_domain(gpu):
    swe = gpu
    case = gen.ensemble_scenario(3, t_min=8e3, t_max=9e3)
    mesh = swe.Mesh(case.xy, case.tri, case.edge_tag)
    t_end = 2.5
    rc0, st0, ref = _single(swe, case, mesh, "f64", 5000, t_end=t_end)
    sh = swe.ShardedSolver(mesh, 5, case.z, case.n, case.h, case.hu, case.hv, dtype="f64",
                           inflow_q=case.inflow_q, t_end=t_end)
    for _ in range(st0["steps"] + 3):   # steps past t_end change nothing
        sh.step()
    rc1, st1 = sh.stats()
    print(f"inflow scenario {mesh.n_cells} cells: {st0['steps']} steps to t_end")
    assert rc0 == rc1 == swe.SWE_OK and st0["done"] and st1["done"]
    assert st1["steps"] == st0["steps"] and st1["t"] == st0["t"] == t_end
    for a, b in zip(ref, sh.numpy_state()):
        assert np.array_equal(a, b)


def test_shard_state_refuses_replayed_dt(gpu):
    swe = gpu
    import torch
    case = gen.small(1)
    mesh = swe.Mesh(case.xy, case.tri)
    sh = swe.ShardedSolver(mesh, 2, case.z, case.n, case.h, case.hu, case.hv)
    dt = torch.full((4,), 1e-3, dtype=torch.float64, device=mesh.device)
    with pytest.raises(swe.SweError):
        sh.solvers[0].run(4, dt_seq=dt)
