"""Meshes whose tiles are scattered: cells in a random order, no Morton renumbering, so a
256-cell tile has more than 512 interfaces and the tiled kernels take their plain LDS layout
with a third round of interfaces (the FP64 step and the flux adjoint).  The results must not
depend on the cell order or on the kernel."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def scattered(case, seed=11):
    """The case with its triangles (and per-cell fields) in a random order."""
    perm = np.random.default_rng(seed).permutation(case.n_cells)
    c = gen.Case(case.name + "-scattered", case.xy, case.tri[perm], case.z[perm], case.n[perm],
                 case.h[perm], case.hu[perm], case.hv[perm], case.steps)
    return c, perm


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scattered_tiles_match_the_morton_run(gpu, dtype):
    import paper_1807_00672_amd as swe
    case = gen.small(3)
    sc, perm = scattered(case)
    m = swe.Mesh(sc.xy, sc.tri, morton=False)
    print(f"scattered mesh: {m.info.n_tiles} tiles, max interfaces per tile "
          f"{m.info.max_tile_edges}, max halo {m.info.max_halo}")
    assert m.info.max_tile_edges > 512
    ref = swe.Solver(swe.Mesh(case.xy, case.tri), case.z, case.n, case.h, case.hu, case.hv,
                     dtype=dtype, variant="tiled")
    ref.run(60)
    want = [x[perm] for x in ref.numpy_state()]
    for variant in ("tiled", "cell"):
        s = swe.Solver(m, sc.z, sc.n, sc.h, sc.hu, sc.hv, dtype=dtype, variant=variant)
        rc, st = s.run(60)
        assert rc == swe.SWE_OK and st["steps"] == 60
        for x, y in zip(s.numpy_state(), want):
            assert np.array_equal(x, y)


def test_scattered_tiles_adjoint(gpu):
    """The tiled flux adjoint in its plain layout (and beyond 64 KiB of LDS) against the per-cell
    one, on a scattered mesh."""
    import paper_1807_00672_amd as swe
    case = gen.small(5)
    sc, perm = scattered(case, seed=12)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    m = swe.Mesh(sc.xy, sc.tri, morton=False)
    assert m.info.max_tile_edges > 512
    steps = 60
    sv = swe.Solver(m, sc.z, sc.n, sc.h, sc.hu, sc.hv, dtype="f64")
    dts = []
    for _ in range(steps):
        dts.append(sv.stats()[1]["dt_next"])
        sv.step()
    gauges = inv[case.extra["gauges"][:16]]
    obs = np.full((steps // 10, gauges.size), 0.5)
    calib = swe.Calibration(m, np.array(dts), gauges, obs, every=10, ckpt_every=20)
    jt, gt = calib.run(sc.n, sc.z, sc.h, sc.hu, sc.hv, variant="tiled")
    jc, gc = calib.run(sc.n, sc.z, sc.h, sc.hu, sc.hv, variant="cell")
    assert jt == jc and jt > 0
    for a, b in zip(gt, gc):
        scale = np.abs(a).max()
        print(f"max |grad| {scale:.3e}, max difference {np.abs(a - b).max():.3e}")
        assert scale > 0 and np.abs(a - b).max() <= 1e-12 * scale
