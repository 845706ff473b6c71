"""Full-size parity: configurations 2 (1,000,000 triangles, 1,000 steps) and 3 (10,000,000
triangles, 500 steps, the benchmark workload) in the launch configuration the benchmark
times.  Final states are compared on a seeded sample of cells against values the oracle wrote
(tests/golden/make_golden.py), a fixture that pins this host's oracle build too; the first
steps are compared on every cell against the oracle run here.  Every cell of the final states
is compared in test_gpu_configured.py."""
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle
from parity import TOL_F32, TOL_F64, errors, quarter_turn, run_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cases():
    return {}


def _case(cases, k):
    if k not in cases:
        cases[k] = gen.config(k)
    return cases[k]


def _golden(k):
    with open(os.path.join(GOLDEN, f"config{k}_final.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_final_state_matches_oracle_samples(gpu, cases, k, dtype):
    case = _case(cases, k)
    gd = _golden(k)
    rc, st, h, hu, hv = run_gpu(case, dtype)
    assert rc == 0 and st["steps"] == gd["steps"] == case.steps
    ids = np.asarray(gd["ids"])
    hmax = gd["max_h"]
    floor = 1e-3 * hmax * math.sqrt(case.g * hmax)
    e_h = np.abs(h[ids] - np.asarray(gd["h"])).max() / hmax
    e_hu = np.abs(hu[ids] - np.asarray(gd["hu"])).max() / max(gd["max_hu"], floor)
    e_hv = np.abs(hv[ids] - np.asarray(gd["hv"])).max() / max(gd["max_hv"], floor)
    wet = int((h > case.h_dry).sum())
    print(f"config {k} {dtype}: sampled errors h {e_h:.3e} hu {e_hu:.3e} hv {e_hv:.3e}; "
          f"t {st['t']!r} vs {gd['t']!r}; wet {wet} vs {gd['wet_cells']}")
    assert st["clamps"] == gd["clamps"]
    # both workloads are walled: with no depth clamped, the volume stays put up to rounding
    a, b, c = (case.xy[case.tri[:, j]] for j in range(3))
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    m0 = float(np.dot(case.h, area))
    drift = abs(float(np.dot(np.asarray(h, dtype=np.float64), area)) - m0) / m0
    print(f"   volume drift over {st['steps']} steps {drift:.3e}")
    assert gd["clamps"] > 0 or drift <= (1e-12 if dtype == "f64" else TOL_F32)
    if dtype == "f64":
        assert max(e_h, e_hu, e_hv) <= TOL_F64
        assert st["t"] == pytest.approx(gd["t"], rel=TOL_F64)
        assert wet == gd["wet_cells"]
        assert np.abs(h).max() == pytest.approx(hmax, rel=TOL_F64)
    else:
        # depth and volume here; the momentum of the FP32 run is compared on every cell with
        # the oracle of the float-rounded inputs (test_gpu_configured.py)
        assert e_h <= TOL_F32
        assert st["t"] == pytest.approx(gd["t"], rel=1e-5)
        band = TOL_F32 * hmax
        assert abs(wet - gd["wet_cells"]) <= int((np.abs(h - case.h_dry) <= band).sum())


@pytest.mark.parametrize("k,steps", [(2, 10), (3, 3)])
def test_first_steps_match_oracle_on_every_cell(gpu, cases, k, steps):
    case = _case(cases, k)
    rc_o, h_o, hu_o, hv_o, dts, st_o = oracle.run_case(case, steps=steps)
    rc_g, st_g, h, hu, hv = run_gpu(case, "f64", steps=steps)
    assert rc_o == 0 and rc_g == 0 and st_g["steps"] == steps
    e = errors(case, (h, hu, hv), (h_o, hu_o, hv_o))
    print(f"config {k}, {steps} steps, all {case.n_cells} cells: errors {e}")
    assert max(e) <= TOL_F64
    assert st_g["t"] == pytest.approx(st_o["t"], rel=TOL_F64)
    assert np.array_equal(h > case.h_dry, h_o > case.h_dry)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_quarter_turn_on_every_cell_at_full_size(gpu, cases, dtype):
    """The quarter-turn covariance of the step (a property that holds at any size) on the
    10,000,000-triangle benchmark workload, 100 steps, every cell: the turned mesh (its own
    Morton order, tiles and halos) gives h unchanged and (hu, hv) -> (-hv, hu) bit for bit."""
    case = _case(cases, 3)
    steps = 100
    rc, st, h, hu, hv = run_gpu(case, dtype, steps=steps)
    rc2, st2, h2, hu2, hv2 = run_gpu(quarter_turn(case), dtype, steps=steps)
    print(f"config 3 {dtype}, {steps} steps: t {st['t']!r} and {st2['t']!r}; differing cells "
          f"h {int((h2 != h).sum())}, hu {int((hu2 != -hv).sum())}, hv {int((hv2 != hu).sum())}")
    assert rc == rc2 == 0 and st["steps"] == st2["steps"] == steps and st["t"] == st2["t"]
    assert np.array_equal(h2, h) and np.array_equal(hu2, -hv) and np.array_equal(hv2, hu)
