"""Pins of the oracle's whole step against closed forms and invariants.

Eq. 4 (explicit Euler over the three edges), the CFL condition with Courant 0.7 (section 2.2),
hydrostatic reconstruction and semi-implicit friction (section 2.2), walls (section 3).
"""
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle
import riemann_exact

G = 9.81
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def mass(h, area):
    return float(np.dot(h, area))


# ------------------------------------------------------------------ mesh and geometry
def test_table2_grids_satisfy_euler_formula():
    """Table 2's five unstructured grids: V - E + T = 1 (one simply connected region) and the
    implied boundary-edge count B = 2E - 3T is positive."""
    with open(os.path.join(GOLDEN, "table2.json")) as f:
        tab = json.load(f)["tests"]
    for row in tab:
        assert row["nodes"] - row["edges"] + row["cells"] == 1
        assert 2 * row["edges"] - 3 * row["cells"] > 0
    assert [2 * r["edges"] - 3 * r["cells"] for r in tab] == [68, 224, 720, 2292, 7140]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_generated_meshes_match_euler_and_boundary_identities(k):
    c = gen.small(k)
    m = oracle.Mesh(c.xy, c.tri)
    assert m.n_nodes - m.n_edges + m.n_cells == 1
    assert 2 * m.n_edges == 3 * m.n_cells + m.n_boundary


def test_full_size_mesh_counts_of_config_1():
    c = gen.config(1)
    m = oracle.Mesh(c.xy, c.tri)
    assert (m.n_cells, m.n_nodes, m.n_edges, m.n_boundary) == (10000, 5151, 15150, 300)


def test_areas_inradii_and_closed_cells():
    c = gen.small(2)
    m = oracle.Mesh(c.xy, c.tri)
    cn, nb, area, r = m.arrays()
    assert (area > 0).all()
    assert area.sum() == pytest.approx(2000.0 * 1000.0, rel=1e-13)
    p = c.xy[cn]
    a = np.linalg.norm(p[:, 1] - p[:, 2], axis=1)
    b = np.linalg.norm(p[:, 2] - p[:, 0], axis=1)
    cc = np.linalg.norm(p[:, 0] - p[:, 1], axis=1)
    s = 0.5 * (a + b + cc)
    heron_r = np.sqrt((s - a) * (s - b) * (s - cc) / s)
    np.testing.assert_allclose(r, heron_r, rtol=1e-10)
    # every interior neighbour relation is mutual
    t = np.arange(m.n_cells)
    for k in range(3):
        j = nb[:, k]
        inner = j >= 0
        assert (np.any(nb[j[inner]] == t[inner, None], axis=1)).all()
    assert (nb < 0).sum() == m.n_boundary


def test_right_triangle_cfl_dt_by_hand():
    """Uniform state on an unjittered split-square mesh: every cell is a right isosceles
    triangle with legs d, inradius d (2 - sqrt 2) / 2, so dt = 0.7 r / (|u| + sqrt(g h))."""
    c = gen.dam_break(nx=20, ny=10, lx=20.0, ly=10.0, jitter=0.0)
    m = oracle.Mesh(c.xy, c.tri)
    t = m.n_cells
    h, u, v = 2.0, 0.5, -0.3
    dt = oracle.cfl_dt(m, np.full(t, h), np.full(t, h * u), np.full(t, h * v))
    r = 1.0 * (2.0 - math.sqrt(2.0)) / 2.0
    assert dt == pytest.approx(0.7 * r / (math.hypot(u, v) + math.sqrt(G * h)), rel=1e-14)


def test_inflow_cells_bound_the_cfl_dt_with_the_boundary_wave_speed():
    """Uniform still water on right isosceles triangles (one inradius r for every cell) with
    an inflow segment along x = 0: when the boundary wave speed of the inflow cells exceeds
    sqrt(g h), dt = 0.7 r / (|u_b| + sqrt(g h_b)) of that boundary state.  Shallow water takes
    the critical state (speed 2 sqrt(g h_c)), deep water the cell depth (q / h + sqrt(g h))."""
    from test_oracle_flux import critical_depth
    c = gen.dam_break(nx=20, ny=10, lx=20.0, ly=10.0, jitter=0.0)
    tag = np.zeros((c.n_cells, 3), dtype=np.int32)
    for k in range(3):
        a, b = c.xy[c.tri[:, k]], c.xy[c.tri[:, (k + 1) % 3]]
        tag[(a[:, 0] == 0.0) & (b[:, 0] == 0.0), k] = 1
    assert tag.sum() == 10
    m = oracle.Mesh(c.xy, c.tri, tag)
    t = m.n_cells
    r = 1.0 * (2.0 - math.sqrt(2.0)) / 2.0
    q = 10.0
    hc = float(critical_depth(q))
    for h, speed in ((0.5, 2.0 * math.sqrt(G * hc)), (4.0, q / 4.0 + math.sqrt(G * 4.0))):
        assert speed > math.sqrt(G * h)
        dt = oracle.cfl_dt(m, np.full(t, h), np.zeros(t), np.zeros(t), inflow_q=[q])
        assert dt == pytest.approx(0.7 * r / speed, rel=1e-13)
        dt_walls = oracle.cfl_dt(oracle.Mesh(c.xy, c.tri), np.full(t, h), np.zeros(t),
                                 np.zeros(t))
        assert dt_walls == pytest.approx(0.7 * r / math.sqrt(G * h), rel=1e-14)


# --------------------------------------------------------------------- invariants
def test_lake_at_rest_with_dry_islands_is_held_to_round_off():
    c = gen.lake_at_rest()
    assert (c.h == 0).sum() > 100 and (c.h > 0).sum() > 1000    # islands and water
    m = oracle.Mesh(c.xy, c.tri)
    rc, h, hu, hv, dts, st = oracle.run_case(c, mesh=m)
    assert rc == 0 and st["steps"] == 1000 and st["clamps"] == 0
    hmax = c.h.max()
    assert np.abs(h - c.h).max() <= 1e-12 * hmax
    assert max(np.abs(hu).max(), np.abs(hv).max()) <= 1e-12 * hmax * math.sqrt(G * hmax)


@pytest.mark.parametrize("k", [1, 2])
def test_mass_is_conserved_in_a_walled_box(k):
    c = gen.small(k)
    m = oracle.Mesh(c.xy, c.tri)
    area = m.arrays()[2]
    rc, h, hu, hv, dts, st = oracle.run_case(c, mesh=m)
    assert rc == 0 and st["clamps"] == 0
    m0 = mass(c.h, area)
    assert abs(mass(h, area) - m0) / m0 <= 1e-12
    assert h.min() >= 0.0
    if k == 2:   # the wet/dry case really has both
        assert (h <= c.h_dry).sum() > 0 and (h > c.h_dry).sum() > 0


def test_positivity_and_dry_cells_carry_no_momentum():
    c = gen.small(2)
    rc, h, hu, hv, dts, st = oracle.run_case(c)
    assert rc == 0
    assert h.min() >= 0.0
    dry = h <= c.h_dry
    assert (hu[dry] == 0).all() and (hv[dry] == 0).all()


# --------------------------------------------------------------------- closed forms
def _riemann_l1(case, t_end, hl, hr, x0):
    m = oracle.Mesh(case.xy, case.tri)
    cn, _, area, _ = m.arrays()
    rc, h, hu, hv, dts, st = oracle.run_case(case, steps=100000, t_end=t_end, mesh=m)
    assert rc == 0 and st["t"] == t_end
    xc = case.xy[cn].mean(axis=1)[:, 0]
    h_ex, u_ex = riemann_exact.sample((xc - x0) / t_end, hl, 0.0, hr, 0.0)
    return float(np.dot(np.abs(h - h_ex), area) / area.sum()), h, hu, xc


def test_stoker_dam_break_on_config_1():
    """Config 1 (jittered, 10,000 cells) against Stoker's wet-bed solution before the waves
    reach the walls: the middle state is reached and the L1 error is small."""
    with open(os.path.join(GOLDEN, "stoker.json")) as f:
        st = json.load(f)
    c = gen.config(1)
    err, h, hu, xc = _riemann_l1(c, 1.0, st["h_left"], st["h_right"], 10.0)
    assert err < 0.012
    mid = (xc > 10.0 + 1.0 * st["rarefaction_tail"] + 0.4) & (xc < 10.0 + 1.0 * st["shock_speed"] - 0.6)
    assert mid.sum() > 50
    assert np.median(h[mid]) == pytest.approx(st["h_mid"], rel=0.02)
    assert np.median(hu[mid] / h[mid]) == pytest.approx(st["u_mid"], rel=0.02)


def test_stoker_converges_under_refinement_on_strips():
    errs = []
    for nx in (100, 200, 400):
        c = gen.strip(nx)
        errs.append(_riemann_l1(c, 1.0, 1.0, 0.1, 10.0)[0])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.6 * errs[0]


def test_ritter_dry_bed_converges_under_refinement():
    errs = []
    for nx in (100, 200, 400):
        c = gen.strip(nx, h_right=0.0)
        errs.append(_riemann_l1(c, 0.5, 1.0, 0.0, 10.0)[0])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.7 * errs[0]


def test_friction_decay_matches_closed_form_in_a_uniform_interior():
    """Uniform flow: with no flux divergence the semi-implicit step gives 1/u -> 1/u + k dt,
    the exact solution u(t) = u0 / (1 + k u0 t) of du/dt = -k u^2, k = g n^2 / h^(4/3)."""
    h0, n_man, u0 = 1.7, 0.05, 1.0
    c = gen.dam_break(nx=80, ny=40, lx=40.0, ly=20.0, jitter=0.2, h_left=h0, h_right=h0)
    t = c.n_cells
    m = oracle.Mesh(c.xy, c.tri)
    cn = m.arrays()[0]
    rc, h, hu, hv, dts, st = oracle.run(m, c.z, np.full(t, n_man), c.h, c.h * u0, c.hv, 40)
    assert rc == 0
    tt = st["t"]
    xc = c.xy[cn].mean(axis=1)
    # the first-order scheme smears the wall waves well past their physical reach
    reach = 3.0 * (u0 + math.sqrt(G * h0)) * tt + 3.0
    inner = ((xc[:, 0] > reach) & (xc[:, 0] < 40 - reach) & (xc[:, 1] > reach) &
             (xc[:, 1] < 20 - reach))
    assert inner.sum() > 100
    k = G * n_man ** 2 / h0 ** (4.0 / 3.0)
    np.testing.assert_allclose(hu[inner] / h[inner], u0 / (1 + k * u0 * tt), rtol=1e-12)
    np.testing.assert_allclose(h[inner], h0, rtol=1e-13)


def test_cells_at_or_below_the_dry_threshold_end_a_step_without_momentum():
    """Cells whose depth after the update is at most h_dry carry no momentum, whatever they
    held before; depths stay non-negative."""
    c = gen.small(2)
    m = oracle.Mesh(c.xy, c.tri)
    rng = np.random.default_rng(9)
    t = c.n_cells
    h = np.where(rng.random(t) < 0.4, 0.5 * c.h_dry, c.h + 0.3)
    hu = rng.uniform(-1, 1, t) * h
    hv = rng.uniform(-1, 1, t) * h
    rc, h1, hu1, hv1, dts, st = oracle.run(m, c.z, c.n, h, hu, hv, 1)
    assert rc == 0 and h1.min() >= 0.0
    dry = h1 <= c.h_dry
    assert dry.sum() > 100
    assert (hu1[dry] == 0).all() and (hv1[dry] == 0).all()
    assert (hu1[~dry] != 0).sum() > 100


def test_inflow_volume_grows_at_the_prescribed_discharge():
    c = gen.ensemble_scenario(3)
    tag = c.edge_tag
    m = oracle.Mesh(c.xy, c.tri, tag)
    area = m.arrays()[2]
    a = c.xy[c.tri]
    seg_len = 0.0
    for k in range(3):
        d = a[:, (k + 1) % 3] - a[:, k]
        seg_len += np.hypot(d[:, 0], d[:, 1])[tag[:, k] == 1].sum()
    assert abs(seg_len - 0.1 * c.xy[:, 1].max()) <= 1.01 * c.extra["delta"]
    rc, h, hu, hv, dts, st = oracle.run_case(c, steps=200, mesh=m)
    assert rc == 0 and st["clamps"] == 0
    expect = mass(c.h, area) + c.inflow_q[0] * seg_len * st["t"]
    assert mass(h, area) == pytest.approx(expect, rel=1e-12)


# --------------------------------------------------------------------- control flow
def test_t_end_shortens_only_the_last_step():
    c = gen.config(1)
    m = oracle.Mesh(c.xy, c.tri)
    _, _, _, _, dts_free, _ = oracle.run_case(c, steps=200, mesh=m)
    rc, h, hu, hv, dts, st = oracle.run_case(c, steps=10000, t_end=0.5, mesh=m)
    assert rc == 0 and st["t"] == 0.5 and st["last_reached"]
    k = st["steps"]
    assert np.array_equal(dts[:-1], dts_free[: k - 1])
    assert 0 < dts[-1] <= dts_free[k - 1]
    t_before = 0.0
    for d in dts[:-1]:
        t_before = t_before + d
    assert dts[-1] == 0.5 - t_before
    assert np.cumsum(dts_free)[k - 2] < 0.5 <= np.cumsum(dts_free)[k - 1]


def test_replaying_the_dt_sequence_is_bitwise():
    c = gen.small(2)
    m = oracle.Mesh(c.xy, c.tri)
    rc, h, hu, hv, dts, st = oracle.run_case(c, steps=50, mesh=m)
    rc2, h2, hu2, hv2, dts2, _ = oracle.run_case(c, steps=50, mesh=m, dt_seq=dts)
    assert rc2 == 0 and np.array_equal(h, h2) and np.array_equal(hu, hu2)


@pytest.mark.parametrize("which", ["wetdry", "inflow"])
def test_a_quarter_turn_of_the_mesh_turns_the_result_bit_for_bit(which):
    """(x, y) -> (-y, x) is exact, and the step (normals, rotation into the edge frame and
    back, lengths, areas, |u|) is covariant under it operation by operation: h unchanged and
    (hu, hv) -> (-hv, hu) exactly.  A sign or component slip in a normal or in a frame
    rotation breaks this; the inflow case turns an inflow segment too."""
    import copy
    case = gen.small(2) if which == "wetdry" else gen.ensemble_scenario(3, steps=60)
    turned = copy.copy(case)
    turned.xy = np.ascontiguousarray(np.stack([-case.xy[:, 1], case.xy[:, 0]], axis=1))
    turned.hu, turned.hv = -case.hv, case.hu.copy()
    rc, h, hu, hv, _, st = oracle.run_case(case, steps=60)
    rc2, h2, hu2, hv2, _, st2 = oracle.run_case(turned, steps=60)
    assert rc == rc2 == 0 and st["steps"] == st2["steps"] == 60 and st["t"] == st2["t"]
    assert np.abs(hu).max() > 0 and np.abs(hv).max() > 0
    assert np.array_equal(h2, h) and np.array_equal(hu2, -hv) and np.array_equal(hv2, hu)


def test_all_dry_and_nonfinite_states_are_reported():
    c = gen.small(1)
    m = oracle.Mesh(c.xy, c.tri)
    z = np.zeros(c.n_cells)
    rc, *_ = oracle.run(m, z, z, z, z, z, 5)
    assert rc == oracle.EDRY
    h = c.h.copy()
    h[17] = np.nan
    rc, *_ = oracle.run(m, z, z, h, z, z, 5)
    assert rc == oracle.ENONFINITE


def test_three_mound_wet_dry_run_keeps_its_invariants():
    """Dam break over a dry floor with mounds: mass conserved, depths non-negative, dry cells
    without momentum, the front advanced past the low mounds, the tall mound's top still dry."""
    c = gen.three_mounds()
    m = oracle.Mesh(c.xy, c.tri)
    cn, _, area, _ = m.arrays()
    rc, h, hu, hv, dts, st = oracle.run_case(c, mesh=m)
    assert rc == 0 and st["steps"] == c.steps
    m0 = mass(c.h, area)
    assert abs(mass(h, area) - m0) <= 1e-12 * m0 + st["clamped_mass"]
    assert h.min() >= 0.0
    dry = h <= c.h_dry
    assert (hu[dry] == 0).all() and (hv[dry] == 0).all()
    xc = c.xy[cn].mean(axis=1)
    wet0 = (c.h > c.h_dry)
    assert xc[h > 1e-3, 0].max() > 30.0 > xc[wet0, 0].max()
    top = np.hypot(xc[:, 0] - 40.0, xc[:, 1] - 12.0) < 1.0
    assert (h[top] <= c.h_dry).all()
