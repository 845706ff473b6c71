"""Checkpoint and resume: a run stopped after n steps, saved to host memory as (h, hu, hv, t,
steps) and restarted from that record in a new state gives the bits of the uninterrupted run.
The host loop of section 2.3 copies data only at the start and at the end, so such a restart is
the way a long simulation is split; the next dt of the restarted state is the CFL bound of the
saved state, computed by the same per-cell bound as the step's own epilogue."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", ["three_mounds", "inflow"])
def test_restart_from_a_saved_state_gives_the_uninterrupted_bits(gpu, dtype, name):
    case = (gen.three_mounds(nx=120, ny=48) if name == "three_mounds"
            else gen.ensemble_scenario(3, t_max=2e4))
    print(f"# resume {name} {dtype}: {case.n_cells} cells", flush=True)
    mesh = gpu.Mesh(case.xy, case.tri, case.edge_tag)
    kw = dict(dtype=dtype, inflow_q=case.inflow_q)
    n1, n2 = 137, 90
    full = gpu.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, **kw)
    rc, st_full = full.run(n1 + n2)
    assert rc == gpu.SWE_OK and st_full["steps"] == n1 + n2
    first = gpu.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, **kw)
    rc, st1 = first.run(n1)
    assert rc == gpu.SWE_OK
    # the checkpoint: host copies of the state in input order, its time and step count
    saved = {"h": None, "hu": None, "hv": None, "t": st1["t"], "steps": st1["steps"]}
    saved["h"], saved["hu"], saved["hv"] = (np.array(a) for a in first.numpy_state())
    del first
    resumed = gpu.Solver(mesh, case.z, case.n, saved["h"], saved["hu"], saved["hv"],
                         t0=saved["t"], **kw)
    rc, st2 = resumed.run(n2)
    assert rc == gpu.SWE_OK
    assert saved["steps"] + st2["steps"] == st_full["steps"]
    assert st2["t"] == st_full["t"] and st2["dt_next"] == st_full["dt_next"]
    assert st2["clamps"] + st1["clamps"] == st_full["clamps"]
    for a, b in zip(full.numpy_state(), resumed.numpy_state()):
        assert np.array_equal(a, b)


def test_restart_keeps_the_t_end_stop(gpu):
    """With t_end, the restarted state stops at the same step and at t_end exactly."""
    case = gen.three_mounds(nx=60, ny=24)
    mesh = gpu.Mesh(case.xy, case.tri)
    t_end = 1.0
    full = gpu.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, t_end=t_end)
    rc, st_full = full.run(10_000)
    assert rc == gpu.SWE_OK and st_full["done"] and st_full["t"] == t_end
    first = gpu.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, t_end=t_end)
    rc, st1 = first.run(st_full["steps"] // 2)
    h, hu, hv = first.numpy_state()
    resumed = gpu.Solver(mesh, case.z, case.n, h, hu, hv, t0=st1["t"], t_end=t_end)
    rc, st2 = resumed.run(10_000)
    assert rc == gpu.SWE_OK and st2["done"] and st2["t"] == t_end
    assert st1["steps"] + st2["steps"] == st_full["steps"]
    for a, b in zip(full.numpy_state(), resumed.numpy_state()):
        assert np.array_equal(a, b)
