"""Hand-written adjoint of the step against the oracle: the loss, a dot-product test against
the oracle's tangent-linear model in every input direction, every gradient entry of a small
mesh against the tangent-linear derivative along its basis direction, central finite
differences on 32 random cells (eps = 1e-6), independence of the checkpoint interval, and
torch.autograd."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

STEPS = 200


@pytest.fixture(scope="module")
def setup(gpu):
    from test_oracle_adjoint import tilted_calibration
    case = tilted_calibration()
    om = oracle.Mesh(case.xy, case.tri)
    dts, obs = oracle.observations(case, om, steps=STEPS)
    mesh = gpu.Mesh(case.xy, case.tri)
    calib = gpu.Calibration(mesh, dts, case.extra["gauges"], obs, every=10, ckpt_every=50)
    j, grads = calib.run(case.n, case.z, case.h, case.hu, case.hv)
    return case, om, dts, obs, calib, j, grads


def test_loss_matches_oracle(setup):
    case, om, dts, obs, calib, j, grads = setup
    jo = oracle.run_loss(om, case.z, case.n, case.h, case.hu, case.hv, dts,
                         case.extra["gauges"], 10, obs)
    assert j == pytest.approx(jo, rel=1e-12)
    assert j > 0


def test_loss_has_the_bits_of_a_plain_run(setup, gpu):
    """The adjoint's forward and recompute passes step with the replay instance of the step
    kernel (dt given, no CFL bound formed); a plain run with the same dt sequence must pass
    through the same states, so the misfit of its gauge depths, summed on the host in the
    kernels' order (squares in gauge order per observation, then the observations in order),
    has the loss's bits."""
    import torch
    case, om, dts, obs, calib, j, grads = setup
    mesh = gpu.Mesh(case.xy, case.tri)
    sv = gpu.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype="f64")
    dt = torch.as_tensor(np.asarray(dts, np.float64), device=mesh.device)
    gauges = np.asarray(case.extra["gauges"])
    jj = 0.0
    for m in range(STEPS // 10):
        rc, _ = sv.run(10, dt_seq=dt[10 * m:10 * m + 10])
        assert rc == 0
        h = sv.numpy_state()[0]
        acc = 0.0
        for g, o in zip(gauges, obs[m]):
            r = float(h[g]) - float(o)
            acc += r * r
        jj += acc
    assert jj == j


@pytest.mark.parametrize("which", ["n", "z", "h", "hu", "hv"])
def test_dot_product_with_oracle_tangent(setup, which):
    case, om, dts, obs, calib, j, grads = setup
    k = ["n", "z", "h", "hu", "hv"].index(which)
    rng = np.random.default_rng(100 + k)
    v = rng.normal(size=case.n_cells)
    jo, djo = oracle.run_tl(om, case.z, case.n, case.h, case.hu, case.hv, dts,
                            case.extra["gauges"], 10, obs, **{"d" + which: v})
    adj = float(np.dot(grads[k], v))
    print(f"d{which}: adjoint <grad, v> = {adj!r}, tangent dJ[v] = {djo!r}")
    assert adj == pytest.approx(djo, rel=1e-9, abs=1e-14 * abs(jo))


def test_central_differences_on_random_cells(setup):
    case, om, dts, obs, calib, j, grads = setup
    rng = np.random.default_rng(7)
    wet = np.flatnonzero(case.h > 1e-2)
    cells = rng.choice(wet, size=32, replace=False)
    dn = grads[0]
    eps = 1e-6
    bad = []
    for c in cells:
        n_p, n_m = case.n.copy(), case.n.copy()
        n_p[c] += eps
        n_m[c] -= eps
        jp, _ = calib.run(n_p, case.z, case.h, case.hu, case.hv)
        jm, _ = calib.run(n_m, case.z, case.h, case.hu, case.hv)
        fd = (jp - jm) / (2 * eps)
        if abs(fd - dn[c]) > 1e-6 * np.abs(dn).max() + 1e-4 * abs(dn[c]):
            bad.append((int(c), fd, dn[c]))
    print(f"max |dJ/dn| {np.abs(dn).max():.3e}; disagreements {bad}")
    assert len(bad) == 0


@pytest.mark.parametrize("ckpt_every", [7, 1])
def test_checkpoint_interval_does_not_change_gradients(setup, gpu, ckpt_every):
    """Other checkpoint intervals, and every state stored (no recompute), give the same bits."""
    case, om, dts, obs, calib, j, grads = setup
    c2 = gpu.Calibration(calib.mesh, dts, case.extra["gauges"], obs, every=10, ckpt_every=ckpt_every)
    j2, g2 = c2.run(case.n, case.z, case.h, case.hu, case.hv)
    assert j2 == j
    for a, b in zip(grads, g2):
        assert np.array_equal(a, b)


def test_tiled_and_per_cell_adjoints_agree(setup, gpu):
    """The tiled flux adjoint differentiates each interface once, the per-cell one once per
    side: the same quantities, summed in the same order, up to rounding."""
    case, om, dts, obs, calib, j, grads = setup
    jc, gc = calib.run(case.n, case.z, case.h, case.hu, case.hv, variant="cell")
    jt, gt = calib.run(case.n, case.z, case.h, case.hu, case.hv, variant="tiled")
    assert jc == jt == j
    for a, b in zip(gc, gt):
        scale = np.abs(a).max()
        print(f"max |grad| {scale:.3e}, max difference {np.abs(a - b).max():.3e}")
        assert np.abs(a - b).max() <= 1e-12 * scale


def test_autograd_function(setup, gpu):
    """AdjointLoss on host tensors and on device tensors: the same loss and gradients bit for
    bit as Calibration.run; device inputs get device gradients (permuted on the device)."""
    import torch
    case, om, dts, obs, calib, j, grads = setup
    ts = [torch.tensor(a, requires_grad=True) for a in (case.n, case.z, case.h, case.hu, case.hv)]
    loss = gpu.AdjointLoss.apply(calib, *ts)
    (2.0 * loss).backward()
    assert loss.item() == j
    for t, g in zip(ts, grads):
        assert np.array_equal(t.grad.numpy(), 2.0 * g)
    dev = calib.mesh.device
    td = [torch.tensor(a, device=dev, requires_grad=True)
          for a in (case.n, case.z, case.h, case.hu, case.hv)]
    loss = gpu.AdjointLoss.apply(calib, *td)
    loss.backward()
    assert loss.device == dev and loss.item() == j
    for t, g in zip(td, grads):
        assert t.grad.device == dev and np.array_equal(t.grad.cpu().numpy(), g)
    jd, gd = calib.run_device(*[t.detach() for t in td])
    assert jd == j and all(x.device == dev for x in gd)


@pytest.mark.parametrize("ckpt_every", [1, 2])
def test_roughness_gradient_matches_friction_closed_form(gpu, ckpt_every):
    """dJ/dn on the supersonic channel (two steps, one gauge) against the hand-derived closed
    form: nonzero only at the gauge and its upwind neighbour."""
    from test_oracle_adjoint import friction_closed_form_dn, supersonic_channel
    xy, tri, st, gauge, dts, obs, consts = supersonic_channel()
    mesh = gpu.Mesh(xy, tri)
    j_want, want = friction_closed_form_dn(xy, tri, st["n"], gauge, consts)
    calib = gpu.Calibration(mesh, dts, [gauge], obs, every=2, ckpt_every=ckpt_every)
    j, grads = calib.run(st["n"], st["z"], st["h"], st["hu"], st["hv"])
    dn = grads[0]
    print(f"J {j!r} (closed form {j_want!r}); dn at the gauge {dn[gauge]!r} "
          f"(closed form {want[gauge]!r}); max |dn - closed form| {np.abs(dn - want).max():.3e}")
    assert j == pytest.approx(j_want, rel=1e-12)
    assert np.abs(dn - want).max() <= 1e-10 * np.abs(want).max()


@pytest.fixture(scope="module")
def small_full_gradient():
    """A 400-cell calibration (one full tile and a ragged one, 60 steps, 8 gauges) and every
    entry of the oracle's gradient: the tangent-linear derivative along each entry's basis
    direction, one oracle run per entry."""
    case = gen.calibration(nx=20, ny=10, steps=60, n_gauges=8)
    case.z = case.z + 1e-4 * gen.centroids(case.xy, case.tri)[:, 0]
    om = oracle.Mesh(case.xy, case.tri)
    dts, obs = oracle.observations(case, om, steps=60)
    t = case.n_cells
    ref = np.empty((5, t))
    for k, which in enumerate(("n", "z", "h", "hu", "hv")):
        for c in range(t):
            e = np.zeros(t)
            e[c] = 1.0
            _, ref[k, c] = oracle.run_tl(om, case.z, case.n, case.h, case.hu, case.hv, dts,
                                         case.extra["gauges"], 10, obs, **{"d" + which: e})
    return case, dts, obs, ref


@pytest.mark.parametrize("ckpt_every", [7, 1])
def test_every_gradient_entry_matches_the_oracle(gpu, small_full_gradient, ckpt_every):
    case, dts, obs, ref = small_full_gradient
    mesh = gpu.Mesh(case.xy, case.tri)
    calib = gpu.Calibration(mesh, dts, case.extra["gauges"], obs, every=10, ckpt_every=ckpt_every)
    j, grads = calib.run(case.n, case.z, case.h, case.hu, case.hv)
    for k, which in enumerate(("n", "z", "h", "hu", "hv")):
        scale = np.abs(ref[k]).max()
        err = np.abs(np.asarray(grads[k]) - ref[k]).max()
        print(f"d{which}: {np.count_nonzero(ref[k])} nonzero entries, max |grad| {scale:.3e}, "
              f"max difference {err:.3e}")
        assert scale > 0
        assert err <= 1e-12 * scale


def test_adjoint_with_an_inflow_segment_matches_the_oracle_tangent(gpu):
    """An ensemble scenario with its inflow segment (discharge through the boundary, the depth
    there from max(h, critical depth)): the loss and the dot product of each gradient with a
    random direction against the oracle's tangent model, gauges near the inflow."""
    case = gen.ensemble_scenario(3, steps=60)
    om = oracle.Mesh(case.xy, case.tri, case.edge_tag)
    q = case.inflow_q
    rc, _, _, _, dts, _ = oracle.run(om, case.z, case.n, case.h, case.hu, case.hv, 60, inflow_q=q)
    assert rc == 0 and len(dts) == 60
    rng = np.random.default_rng(5)
    near = np.argsort(gen.centroids(case.xy, case.tri)[:, 0])[:200]
    gauges = np.sort(rng.choice(near, 12, replace=False)).astype(np.int32)
    h, hu, hv, obs = case.h.copy(), case.hu.copy(), case.hv.copy(), []
    for s in range(60):   # observations of a rougher run
        rc, h, hu, hv, _, _ = oracle.run(om, case.z, 1.3 * case.n, h, hu, hv, 1,
                                         dt_seq=dts[s:s + 1], inflow_q=q)
        if (s + 1) % 10 == 0:
            obs.append(h[gauges].copy())
    obs = np.array(obs)
    mesh = gpu.Mesh(case.xy, case.tri, case.edge_tag)
    calib = gpu.Calibration(mesh, dts, gauges, obs, every=10, ckpt_every=7, inflow_q=q)
    j, grads = calib.run(case.n, case.z, case.h, case.hu, case.hv)
    jo = oracle.run_loss(om, case.z, case.n, case.h, case.hu, case.hv, dts, gauges, 10, obs,
                         inflow_q=q)
    assert j == pytest.approx(jo, rel=1e-12) and j > 0
    for k, which in enumerate(("n", "z", "h", "hu", "hv")):
        v = rng.normal(size=case.n_cells)
        _, djo = oracle.run_tl(om, case.z, case.n, case.h, case.hu, case.hv, dts, gauges, 10,
                               obs, inflow_q=q, **{"d" + which: v})
        adj = float(np.dot(grads[k], v))
        print(f"inflow d{which}: adjoint {adj!r}, tangent {djo!r}")
        assert adj == pytest.approx(djo, rel=1e-9, abs=1e-14 * abs(jo))
