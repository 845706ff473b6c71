"""Pin of the oracle's tangent-linear model (the reference for the GPU adjoint) against
central finite differences of the plain oracle, on the calibration setup (gauge misfit every
10 steps, dt replayed)."""
import numpy as np
import pytest

import gen
import oracle


def tilted_calibration():
    """The calibration recipe with a 1e-4 bed slope added: far from its bumps the bed is
    exactly flat, where max(z_a, z_b) has no derivative and finite differences measure a mix
    of one-sided slopes; the tilt keeps neighbouring beds ~3e-3 m apart."""
    case = gen.small(5)
    case.z = case.z + 1e-4 * gen.centroids(case.xy, case.tri)[:, 0]
    case.h = case.h.copy()
    return case


@pytest.fixture(scope="module")
def setup():
    case = tilted_calibration()
    mesh = oracle.Mesh(case.xy, case.tri)
    dts, obs = oracle.observations(case, mesh, steps=100)
    return case, mesh, dts, obs


@pytest.mark.parametrize("which", ["n", "z", "h", "hu"])
def test_tangent_matches_central_differences(setup, which):
    case, mesh, dts, obs = setup
    g = case.extra["gauges"]
    rng = np.random.default_rng(["n", "z", "h", "hu"].index(which))
    t = case.n_cells
    scale = {"n": 1e-3, "z": 1e-2, "h": 1e-2, "hu": 1e-2}[which]
    v = rng.normal(size=t) * scale
    if which in ("h", "hu"):
        v *= case.h > 1e-3              # keep dry cells dry
    base = dict(z=case.z, n=case.n, h=case.h, hu=case.hu, hv=case.hv)
    J, dJ = oracle.run_tl(mesh, case.z, case.n, case.h, case.hu, case.hv, dts, g, 10, obs,
                          **{"d" + which: v})
    eps = 1e-6

    def loss(sign):
        args = dict(base)
        args[which] = base[which] + sign * eps * v
        return oracle.run_loss(mesh, args["z"], args["n"], args["h"], args["hu"], args["hv"],
                               dts, g, 10, obs)

    fd = (loss(1) - loss(-1)) / (2 * eps)
    assert J == pytest.approx(loss(0), rel=1e-15)
    assert dJ == pytest.approx(fd, rel=1e-5)


def supersonic_channel(nx=24, ny=12, h0=1.7, froude=2.0, dt=0.015, seed=3):
    """Right triangles (fixed diagonals, 1 m squares), flat bed, uniform depth h0 and velocity
    u0 = Froude * sqrt(g h0) along x, walls, Manning n random per cell.  Every edge that carries
    mass is then supersonic (|q| >= u0 / sqrt(2) > c), so each HLLC mass flux is the upwind
    side's h q; edges along the flow carry none.  Gauge: the lower triangle of the central square,
    observed after two steps of length dt (observation h0 - 0.1)."""
    g = 9.81
    xs, ys = np.meshgrid(np.arange(nx + 1.0), np.arange(ny + 1.0))
    xy = np.stack([xs.ravel(), ys.ravel()], 1)
    node = lambda i, j: j * (nx + 1) + i
    tri = []
    for j in range(ny):
        for i in range(nx):
            tri.append((node(i, j), node(i + 1, j), node(i + 1, j + 1)))   # lower
            tri.append((node(i, j), node(i + 1, j + 1), node(i, j + 1)))   # upper
    tri = np.array(tri, np.int32)
    t = tri.shape[0]
    u0 = froude * np.sqrt(g * h0)
    n = np.random.default_rng(seed).uniform(0.02, 0.05, t)
    gauge = 2 * ((ny // 2) * nx + nx // 2)
    state = dict(z=np.zeros(t), n=n, h=np.full(t, h0), hu=np.full(t, h0 * u0), hv=np.zeros(t))
    return xy, tri, state, gauge, np.array([dt, dt]), np.array([[h0 - 0.1]]), (g, h0, u0, dt)


def friction_closed_form_dn(xy, tri, n, gauge, consts):
    """dJ/dn of the two-step misfit J = (h2[gauge] - obs)^2 in supersonic_channel, by hand.

    Step 1 moves no mass in the uniform interior and its friction turns u0 into
    u1 = u0 / D(n), D = 1 + dt g n^2 |q| / (h0^2 h0^(1/3)) with |q| = h0 u0.  Step 2's mass flux
    through an edge of the gauge cell with outward normal (n_x, n_y) is h0 u1 n_x of the upwind
    cell, so h2 = h0 - dt / A sum_k l_k n_x,k h0 u1(upwind_k), with l_k n_x,k = dy_k.  Outflow
    edges (dy > 0) take the gauge's own n, inflow edges (dy < 0) the neighbour's; dt is not
    differentiated.  Returns (J, dJ/dn)."""
    g, h0, u0, dt = consts
    p = xy[tri[gauge]]
    area = 0.5 * ((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[1, 1] - p[0, 1]) * (p[2, 0] - p[0, 0]))
    k_fric = dt * g * h0 * u0 / (h0 ** 2 * np.cbrt(h0))

    def u1(nm):
        return u0 / (1.0 + k_fric * nm * nm)

    def du1(nm):   # d(u0 / D)/dn
        d = 1.0 + k_fric * nm * nm
        return -u0 * (2.0 * k_fric * nm) / d ** 2

    keys = {}
    for c, (a, b, e) in enumerate(tri):
        for u, v in ((a, b), (b, e), (e, a)):
            keys.setdefault((min(u, v), max(u, v)), []).append(c)
    h2, dh2 = h0, np.zeros(tri.shape[0])
    for k in range(3):
        a, b = tri[gauge][k], tri[gauge][(k + 1) % 3]
        dy = xy[b, 1] - xy[a, 1]
        if dy == 0.0:
            continue
        cell = gauge if dy > 0 else [c for c in keys[(min(a, b), max(a, b))] if c != gauge][0]
        h2 -= dt / area * h0 * dy * u1(n[cell])
        dh2[cell] += -dt / area * h0 * dy * du1(n[cell])
    r = h2 - (h0 - 0.1)
    return r * r, 2.0 * r * dh2


def test_tangent_matches_friction_closed_form():
    """The tangent model's dJ/dn on the supersonic channel, cell by cell, against the
    closed form: nonzero exactly at the gauge (outflow edge) and its upwind neighbour."""
    xy, tri, st, gauge, dts, obs, consts = supersonic_channel()
    mesh = oracle.Mesh(xy, tri)
    j_want, want = friction_closed_form_dn(xy, tri, st["n"], gauge, consts)
    nz = np.flatnonzero(want)
    assert nz.size == 2
    probe = list(nz) + [gauge + 5, gauge - 2 * 24]     # and two cells that must give zero
    for c in probe:
        e = np.zeros(tri.shape[0])
        e[c] = 1.0
        J, dJ = oracle.run_tl(mesh, st["z"], st["n"], st["h"], st["hu"], st["hv"], dts,
                              [gauge], 2, obs, dn=e)
        assert J == pytest.approx(j_want, rel=1e-12)
        print(f"cell {c}: tangent {dJ!r}, closed form {want[c]!r}")
        assert dJ == pytest.approx(want[c], rel=1e-10, abs=1e-12 * np.abs(want).max())


def test_branch_signature_marks_switches(setup):
    """The signature of run_loss_sig is the same for repeated runs and for a perturbation too
    small to flip any branch; it changes when a perturbation flips a branch (a dry cell raised
    above the dry threshold, the bed tilted by more than the neighbouring beds' differences),
    and it leaves the misfit of run_loss unchanged."""
    case, mesh, dts, obs = setup
    g = case.extra["gauges"]
    base = (case.z, case.n, case.h, case.hu, case.hv)
    j0, s0 = oracle.run_loss_sig(mesh, *base, dts, g, 10, obs)
    assert j0 == oracle.run_loss(mesh, *base, dts, g, 10, obs)
    assert oracle.run_loss_sig(mesh, *base, dts, g, 10, obs) == (j0, s0)
    # a smooth perturbation: a gauge cell's roughness by 1e-8
    n1 = case.n.copy()
    n1[g[0]] += 1e-8
    j1, s1 = oracle.run_loss_sig(mesh, case.z, n1, case.h, case.hu, case.hv, dts, g, 10, obs)
    assert s1 == s0 and j1 != j0
    # a dry cell made wet: its dry tests flip
    dry = int(np.flatnonzero(case.h == 0.0)[0])
    h2 = case.h.copy()
    h2[dry] = 1e-3
    assert oracle.run_loss_sig(mesh, case.z, case.n, h2, case.hu, case.hv, dts, g, 10, obs)[1] != s0
    # a bed turned by more than its local differences: which side's bed is the higher flips
    z3 = case.z - 2e-3 * gen.centroids(case.xy, case.tri)[:, 0]
    assert oracle.run_loss_sig(mesh, z3, case.n, case.h, case.hu, case.hv, dts, g, 10, obs)[1] != s0
