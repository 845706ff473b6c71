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
