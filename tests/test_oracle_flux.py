"""Pins of the oracle's interface flux against what the mathematics fixes.

HLLC flux (section 2.2, ref. [6]), hydrostatic reconstruction (section 2.2) and the wall ghost
(section 3).  Nothing here re-derives the oracle's formulas: consistency is checked against the
physical flux of eq. 1 written with (u, v), wave speeds against the exact Riemann solution.
"""
import math

import numpy as np
import pytest

import oracle
import riemann_exact

G = 9.81
H_DRY = 1e-6


def physical_normal_flux(h, u, v, nx, ny, g=G):
    """G(U) nx + H(U) ny of eq. 1, with U = (h, hu, hv)."""
    gx = np.stack([h * u, h * u * u + 0.5 * g * h * h, h * u * v], -1)
    hy = np.stack([h * v, h * u * v, h * v * v + 0.5 * g * h * h], -1)
    return gx * nx[:, None] + hy * ny[:, None]


def random_states(rng, n, dry_frac=0.2, vmax=6.0):
    h = rng.uniform(0.0, 3.0, n)
    h[rng.random(n) < dry_frac] = 0.0
    u = rng.uniform(-vmax, vmax, n)
    v = rng.uniform(-vmax, vmax, n)
    return h, u, v


def unit_normals(rng, n):
    th = rng.uniform(0, 2 * math.pi, n)
    return np.cos(th), np.sin(th)


def test_consistency_subcritical_and_supercritical():
    rng = np.random.default_rng(1)
    n = 200000
    h = rng.uniform(1e-3, 3.0, n)
    u = rng.uniform(-8, 8, n)
    v = rng.uniform(-8, 8, n)
    nx, ny = unit_normals(rng, n)
    f = oracle.hllc(h, u, v, h, u, v, nx, ny)
    ref = physical_normal_flux(h, u, v, nx, ny)
    scale = np.abs(ref).max(axis=1) + 0.5 * G * h * h
    err = np.abs(f - ref).max(axis=1) / scale
    assert err.max() < 2e-13   # HLL averaging loses (|S_L|+|S_R|)/(S_R-S_L) ulps
    # in the supercritical branch the upwind physical flux is returned as is
    q = u * nx + v * ny
    sup = np.abs(q) > np.sqrt(G * h) * 2.5
    assert sup.sum() > 1000
    assert err[sup].max() < 1e-14     # only the frame rotation rounds here


def test_antisymmetry_is_bitwise_with_reconstruction_and_dry_sides():
    rng = np.random.default_rng(2)
    n = 1_000_000
    hl, ul, vl = random_states(rng, n)
    hr, ur, vr = random_states(rng, n)
    zl = rng.uniform(-1, 1, n)
    zr = np.where(rng.random(n) < 0.3, zl, rng.uniform(-1, 1, n))
    nx, ny = unit_normals(rng, n)
    f, pl, pr = oracle.interface(hl, hl * ul, hl * vl, zl, hr, hr * ur, hr * vr, zr, nx, ny)
    g_, ql_, qr_ = oracle.interface(hr, hr * ur, hr * vr, zr, hl, hl * ul, hl * vl, zl, -nx, -ny)
    assert np.array_equal(g_, -f)
    assert np.array_equal(ql_, pr) and np.array_equal(qr_, pl)
    # every branch of the solver was exercised
    hs_dry = (f[:, 0] == 0) & (f[:, 1] == 0)
    assert hs_dry.any() and (~hs_dry).any()


def test_rotational_invariance():
    rng = np.random.default_rng(3)
    n = 200000
    hl, ul, vl = random_states(rng, n, dry_frac=0.1)
    hr, ur, vr = random_states(rng, n, dry_frac=0.1)
    nx, ny = unit_normals(rng, n)
    th = rng.uniform(0, 2 * math.pi, n)
    c, s = np.cos(th), np.sin(th)
    rot = lambda x, y: (c * x - s * y, s * x + c * y)
    f = oracle.hllc(hl, ul, vl, hr, ur, vr, nx, ny)
    ul2, vl2 = rot(ul, vl)
    ur2, vr2 = rot(ur, vr)
    nx2, ny2 = rot(nx, ny)
    f2 = oracle.hllc(hl, ul2, vl2, hr, ur2, vr2, nx2, ny2)
    fx, fy = rot(f[:, 1], f[:, 2])
    scale = 1.0 + np.abs(f).max(axis=1)
    assert np.abs(f2[:, 0] - f[:, 0]).max() / scale.max() < 1e-13
    assert (np.abs(f2[:, 1] - fx) / scale).max() < 1e-13
    assert (np.abs(f2[:, 2] - fy) / scale).max() < 1e-13


def test_hllc_contact_carries_upwind_tangential_velocity():
    """Equal depth and normal velocity, different tangential velocity: an isolated contact.

    HLLC keeps it sharp (f_w = f_h * w_upwind); HLL would average the two sides."""
    rng = np.random.default_rng(4)
    n = 10000
    h = rng.uniform(0.1, 3, n)
    q = rng.uniform(-2, 2, n)
    wl = rng.uniform(-3, 3, n)
    wr = rng.uniform(-3, 3, n)
    one, zero = np.ones(n), np.zeros(n)
    f = oracle.hllc(h, q, wl, h, q, wr, one, zero)     # frame = (x, y): q = u, w = v
    wup = np.where(q > 0, wl, wr)
    assert np.array_equal(f[:, 2], f[:, 0] * wup)
    hll = f[:, 0] * 0.5 * (wl + wr)
    assert (np.abs(f[:, 2] - hll) > 1e-6).mean() > 0.9


def test_wall_has_exactly_zero_mass_flux_and_rest_pressure():
    rng = np.random.default_rng(5)
    n = 200000
    h, u, v = random_states(rng, n, dry_frac=0.1)
    h[rng.random(n) < 0.05] = 0.5 * H_DRY
    nx, ny = unit_normals(rng, n)
    f, p = oracle.wall(h, h * u, h * v, nx, ny)
    assert (f[:, 0] == 0.0).all()
    rest = h > H_DRY
    f0, p0 = oracle.wall(h, 0 * h, 0 * h, nx, ny)
    np.testing.assert_allclose(f0[rest, 1], 0.5 * G * h[rest] ** 2 * nx[rest], rtol=1e-13,
                               atol=1e-15)
    # wet cells: no bed correction; dry cells: the full cell pressure g h^2 / 2
    assert (p[rest] == 0).all()
    np.testing.assert_allclose(p[~rest], 0.5 * G * h[~rest] ** 2, rtol=1e-15)


def test_wave_speeds_bound_the_exact_riemann_solution():
    """S_L and S_R enclose every signal of the exact solution; for two rarefactions and for
    dry beds they equal the exact extreme speeds."""
    rng = np.random.default_rng(6)
    for _ in range(400):
        hl, hr = rng.uniform(0.05, 3, 2)
        if rng.random() < 0.2:
            hr = 0.0
        ql, qr = rng.uniform(-3, 3, 2)
        if hr == 0.0 or hl == 0.0:
            pass
        elif qr - ql >= 2 * (math.sqrt(G * hl) + math.sqrt(G * hr)):
            continue
        sl, sr = oracle.wave_speeds([hl], [ql], [hr], [qr])
        el, er = riemann_exact.wave_speeds(hl, ql, hr, qr)
        assert sl[0] <= el + 1e-12 and sr[0] >= er - 1e-12
        hs, _ = riemann_exact.star_state(hl, ql, hr, qr) if hr > 0 else (0.0, 0.0)
        if hr == 0.0 or (hs <= hl and hs <= hr):
            assert sl[0] == pytest.approx(el, rel=1e-13, abs=1e-13)
            assert sr[0] == pytest.approx(er, rel=1e-13, abs=1e-13)


def test_reconstruction_of_flat_bed_is_plain_hllc():
    rng = np.random.default_rng(7)
    n = 100000
    hl, ul, vl = random_states(rng, n)
    hr, ur, vr = random_states(rng, n)
    hl[hl <= H_DRY] = 0.0
    hr[hr <= H_DRY] = 0.0
    z = rng.uniform(-2, 2, n)
    nx, ny = unit_normals(rng, n)
    f, pl, pr = oracle.interface(hl, hl * ul, hl * vl, z, hr, hr * ur, hr * vr, z, nx, ny)
    ul2 = np.where(hl > H_DRY, (hl * ul) / np.where(hl > 0, hl, 1), 0)
    vl2 = np.where(hl > H_DRY, (hl * vl) / np.where(hl > 0, hl, 1), 0)
    ur2 = np.where(hr > H_DRY, (hr * ur) / np.where(hr > 0, hr, 1), 0)
    vr2 = np.where(hr > H_DRY, (hr * vr) / np.where(hr > 0, hr, 1), 0)
    f2 = oracle.hllc(hl, ul2, vl2, hr, ur2, vr2, nx, ny)
    assert np.array_equal(f, f2)
    assert (pl == 0).all() and (pr == 0).all()


def test_reconstruction_step_is_well_balanced_pointwise():
    """Lake at rest across a bed step (one side may be dry): the flux plus the bed correction
    equals the pressure of the side's own depth, g h^2 / 2 n, so a cell's contributions sum to
    g h^2/2 * sum(l n) = 0."""
    rng = np.random.default_rng(8)
    n = 100000
    eta = 1.0
    zl = rng.uniform(-1, 1.5, n)
    zr = rng.uniform(-1, 1.5, n)
    hl = np.maximum(eta - zl, 0)
    hr = np.maximum(eta - zr, 0)
    nx, ny = unit_normals(rng, n)
    f, pl, pr = oracle.interface(hl, 0 * hl, 0 * hl, zl, hr, 0 * hr, 0 * hr, zr, nx, ny)
    assert np.abs(f[:, 0]).max() < 1e-12
    tot_x = f[:, 1] + pl * nx
    np.testing.assert_allclose(tot_x, 0.5 * G * hl * hl * nx, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ inflow boundary
def critical_depth(q, g=G):
    """Depth at which the unit discharge q flows critically, Froude number one (q / h equal to
    sqrt(g h)), by bisection on that condition (q / h - sqrt(g h) falls as h grows)."""
    q = np.asarray(q, dtype=np.float64)
    lo = np.full(q.shape, 1e-6)
    hi = np.full(q.shape, 1e3)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        sub = q / mid - np.sqrt(g * mid) > 0.0
        lo = np.where(sub, mid, lo)
        hi = np.where(sub, hi, mid)
    return 0.5 * (lo + hi)


def test_inflow_flux_of_deep_water_is_the_physical_flux_of_the_boundary_state():
    """At depths h >= h_c the boundary state is the cell's depth carrying the discharge
    inwards, (h, -q n / h): the edge flux is eq. 1's physical normal flux of that state and the
    boundary wave speed is |u_b| + sqrt(g h)."""
    rng = np.random.default_rng(31)
    n = 100000
    q = rng.uniform(5.0, 50.0, n)
    hc = critical_depth(q)
    h = hc * rng.uniform(1.0 + 1e-9, 4.0, n)
    nx, ny = unit_normals(rng, n)
    f, speed = oracle.inflow(q, h, nx, ny)
    ub, vb = -q * nx / h, -q * ny / h
    ref = physical_normal_flux(h, ub, vb, nx, ny)
    scale = np.abs(ref).max(axis=1)
    assert (np.abs(f - ref).max(axis=1) / scale).max() < 1e-14
    ref_speed = np.hypot(ub, vb) + np.sqrt(G * h)
    np.testing.assert_allclose(speed, ref_speed, rtol=1e-14)


def test_inflow_into_shallow_or_dry_cells_runs_at_critical_depth():
    """Below the critical depth (dry cells included) the boundary carries the discharge at
    critical flow: h_b^3 = q^2 / g, so the normal momentum flux q^2 / h_b + g h_b^2 / 2 is
    exactly 3/2 g h_c^2, the mass flux is -q and the boundary wave speed q / h_b + sqrt(g h_b) is
    2 sqrt(g h_c)."""
    rng = np.random.default_rng(32)
    n = 100000
    q = rng.uniform(5.0, 50.0, n)
    hc = critical_depth(q)
    h = hc * rng.uniform(0.0, 1.0 - 1e-9, n)
    h[: n // 10] = 0.0
    nx, ny = unit_normals(rng, n)
    f, speed = oracle.inflow(q, h, nx, ny)
    mom = 1.5 * G * hc * hc
    np.testing.assert_array_equal(f[:, 0], -q)
    np.testing.assert_allclose(f[:, 1], mom * nx, rtol=1e-13, atol=1e-13 * mom.max())
    np.testing.assert_allclose(f[:, 2], mom * ny, rtol=1e-13, atol=1e-13 * mom.max())
    np.testing.assert_allclose(speed, 2.0 * np.sqrt(G * hc), rtol=1e-13)
