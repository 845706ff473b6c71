"""Batched ensemble (scenarios of uneven size with their own inflow and roughness, each with
its own CFL dt): one launch per step must give every scenario exactly what its own run gives,
and match the oracle."""
import numpy as np
import pytest

import gen
import oracle
from parity import TOL_F64, errors, run_gpu

pytestmark = pytest.mark.gpu


def _batch(swe, cases, dtype, steps, t_end=0.0, variant="auto", xcd_remap=True, exact=False):
    meshes = [swe.Mesh(c.xy, c.tri, c.edge_tag) for c in cases]
    b = swe.Batch(meshes)
    bs = swe.BatchSolver(b, cases, dtype=dtype, t_end=t_end, variant=variant,
                         xcd_remap=xcd_remap, exact=exact)
    rc, st = bs.run(steps)
    return rc, st, bs


@pytest.mark.parametrize("variant,remap", [("cell", True), ("tiled", True), ("cell", False)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_equals_single_runs_bitwise(gpu, dtype, variant, remap):
    cases = [gen.ensemble_scenario(s) for s in range(6)]
    rc, st, bs = _batch(gpu, cases, dtype, 120, variant=variant, xcd_remap=remap)
    assert rc == 0
    for s, c in enumerate(cases):
        rc1, st1, h, hu, hv = run_gpu(c, dtype, steps=120)
        assert rc1 == 0 and st[s]["steps"] == st1["steps"] == 120
        assert st[s]["t"] == st1["t"]
        hb, hub, hvb = bs.numpy_state(s)
        assert np.array_equal(hb, h) and np.array_equal(hub, hu) and np.array_equal(hvb, hv)
    ts = [x["t"] for x in st]
    assert len(set(ts)) == len(ts)            # every scenario kept its own dt


@pytest.mark.parametrize("variant", ["tiled", "cell"])
def test_exact_batch_equals_single_exact_runs_bitwise(gpu, variant):
    """Correctly rounded FP64 (SWE_EXACT) in a batch: each scenario as its own exact run."""
    cases = [gen.ensemble_scenario(s) for s in (1, 4, 8)]
    rc, st, bs = _batch(gpu, cases, "f64", 80, variant=variant, exact=True)
    assert rc == 0
    for s, c in enumerate(cases):
        rc1, st1, h, hu, hv = run_gpu(c, "f64", steps=80, exact=True)
        assert rc1 == 0 and st[s]["steps"] == st1["steps"] == 80 and st[s]["t"] == st1["t"]
        hb, hub, hvb = bs.numpy_state(s)
        assert np.array_equal(hb, h) and np.array_equal(hub, hu) and np.array_equal(hvb, hv)


def test_batch_matches_oracle_and_stops_each_scenario_at_t_end(gpu):
    cases = [gen.ensemble_scenario(s) for s in (0, 7, 9)]
    rc, st, bs = _batch(gpu, cases, "f64", 3000, t_end=3.0)
    assert rc == 0
    for s, c in enumerate(cases):
        rc_o, h_o, hu_o, hv_o, dts, st_o = oracle.run_case(c, steps=10000, t_end=3.0)
        assert rc_o == 0 and st[s]["done"] == 1 and st[s]["t"] == 3.0
        assert st[s]["steps"] == st_o["steps"]
        e = errors(c, bs.numpy_state(s), (h_o, hu_o, hv_o))
        print(f"scenario {c.extra['scenario']}: {c.n_cells} cells, {st_o['steps']} steps, {e}")
        assert max(e) <= TOL_F64
