"""swe_run_static (no workspace, no allocation) against swe_state_init + swe_run with a
workspace: the same kernels, so the same bits, on calls in a row whose later meshes are
smaller (the device array keeps the earlier calls' contents)."""
import ctypes as C

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def _solver_pair(swe, case, dtype):
    import torch
    mesh = swe.Mesh(case.xy, case.tri, case.edge_tag)
    ref = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype,
                     inflow_q=case.inflow_q)
    # the same state's buffers for the static call, but no workspace at all
    st = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype,
                    inflow_q=case.inflow_q)
    st.state.work = None
    st.ctrl.zero_()
    torch.cuda.synchronize()
    return mesh, ref, st


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_static_run_equals_the_workspace_run_twice_in_a_row(gpu, dtype):
    import torch
    from paper_1807_00672_amd import _abi as A
    from paper_1807_00672_amd.solver import _stream_handle
    # 40,000 cells in 157 tiles: the step merges its dt partials into atomic slots, which a fold
    # kernel reads and resets; up to 128 tiles the step folds them itself
    large = gen.dam_break(nx=200, ny=100, lx=40.0, ly=20.0)
    big = gen.three_mounds(nx=120, ny=48)                   # 11,520 cells, wet/dry, friction
    small = gen.dam_break(nx=40, ny=20, lx=8.0, ly=4.0)      # 1,600 cells
    for case, steps in ((large, 40), (big, 150), (small, 60)):
        mesh, ref, st = _solver_pair(gpu, case, dtype)
        print(f"# swe_run_static {dtype}: {case.name}, {mesh.n_cells} cells, {steps} steps",
              flush=True)
        rc_ref, s_ref = ref.run(steps)
        stats = A.swe_run_stats()
        rc = A.swe_run_static(mesh.handle, mesh.dev, st.params, st.state, steps, init=True,
                              t0=0.0, t_end=0.0, stats=stats, stream=_stream_handle())
        assert rc == rc_ref == gpu.SWE_OK, (rc, rc_ref, gpu.swe_last_error())
        s = stats.as_dict()
        for k in ("steps", "clamps", "t", "dt_next", "dt_min", "dt_max", "dt_sum", "cur"):
            assert s[k] == s_ref[k], (k, s[k], s_ref[k])
        a, b = ref.numpy_state(), st.numpy_state()
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        # a second static call continues the state (no init) like a second swe_run
        rc_ref, s_ref = ref.run(17)
        rc = A.swe_run_static(mesh.handle, mesh.dev, st.params, st.state, 17, stats=stats,
                              stream=_stream_handle())
        assert rc == rc_ref == gpu.SWE_OK
        assert stats.t == s_ref["t"] and stats.steps == s_ref["steps"]
        for x, y in zip(ref.numpy_state(), st.numpy_state()):
            assert np.array_equal(x, y)
        torch.cuda.synchronize()


def test_static_run_with_t_end_and_replayed_dt(gpu):
    import torch
    from paper_1807_00672_amd import _abi as A
    from paper_1807_00672_amd.solver import _stream_handle, _ptr
    case = gen.dam_break(nx=40, ny=20, lx=8.0, ly=4.0)
    mesh, ref, st = _solver_pair(gpu, case, "f64")
    dts = torch.full((40,), 2.5e-3, dtype=torch.float64, device=mesh.device)
    ref.init(0.0, 0.07)
    rc_ref, s_ref = ref.run(40, dt_seq=dts)
    stats = A.swe_run_stats()
    rc = A.swe_run_static(mesh.handle, mesh.dev, st.params, st.state, 40, init=True, t0=0.0,
                          t_end=0.07, dt_seq=_ptr(dts), stats=stats, stream=_stream_handle())
    assert rc == rc_ref == gpu.SWE_OK
    assert stats.steps == s_ref["steps"] and stats.t == s_ref["t"] == 0.07 and stats.done
    for x, y in zip(ref.numpy_state(), st.numpy_state()):
        assert np.array_equal(x, y)


def test_static_run_rejects_bad_arguments(gpu):
    from paper_1807_00672_amd import _abi as A
    case = gen.dam_break(nx=10, ny=5, lx=2.0, ly=1.0)
    mesh, ref, st = _solver_pair(gpu, case, "f64")
    assert A.lib.swe_run_static(mesh.handle, C.byref(mesh.dev), C.byref(st.params),
                                C.byref(st.state), 1, 0.0, float("nan"), 4, None, None,
                                None) == gpu.SWE_EINVAL
    assert A.lib.swe_run_static(mesh.handle, C.byref(mesh.dev), C.byref(st.params),
                                C.byref(st.state), 0, 0.0, 0.0, -1, None, None,
                                None) == gpu.SWE_EINVAL
