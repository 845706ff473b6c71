"""Tile size (cells per workgroup of the step kernels, a property of the mesh): every size of
64, 128, 256 and 512 gives the same bits in FP64 (both arithmetic modes) and FP32, with the
tiled and the per-cell kernels, batched and single, and adjoint gradients equal up to rounding;
the tuner's choice of size is recorded and Mesh(tile="auto") builds with it."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

TILES = (64, 128, 256, 512)


def _run(swe, mesh, case, dtype, variant="auto", exact=False, steps=80):
    s = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype,
                   variant=variant, exact=exact, inflow_q=case.inflow_q)
    rc, st = s.run(steps)
    assert rc == swe.SWE_OK, (rc, st)
    return st, s.numpy_state()


@pytest.mark.parametrize("dtype,exact", [("f64", False), ("f64", True), ("f32", False)])
@pytest.mark.parametrize("name", ["three_mounds", "inflow"])
def test_every_tile_size_gives_the_same_bits(gpu, dtype, exact, name):
    case = (gen.three_mounds(nx=120, ny=48) if name == "three_mounds"
            else gen.ensemble_scenario(3, t_max=2e4))
    ref = None
    for tile in TILES:
        mesh = gpu.Mesh(case.xy, case.tri, case.edge_tag, tile=tile)
        assert mesh.tile == tile
        for variant in ("tiled", "cell"):
            st, fields = _run(gpu, mesh, case, dtype, variant, exact)
            print(f"# {name} {dtype}{' exact' if exact else ''} tile {tile} {variant}: "
                  f"{mesh.n_cells} cells, t {st['t']!r}", flush=True)
            if ref is None:
                ref = (st, fields)
                continue
            assert st["t"] == ref[0]["t"] and st["steps"] == ref[0]["steps"]
            assert st["clamps"] == ref[0]["clamps"]
            for a, b in zip(fields, ref[1]):
                assert np.array_equal(a, b)


def test_batches_of_every_tile_size_give_the_separate_runs_bits(gpu):
    cases = [gen.ensemble_scenario(s, t_max=2e4) for s in range(4)]
    ref = None
    for tile in TILES:
        meshes = [gpu.Mesh(c.xy, c.tri, c.edge_tag, tile=tile) for c in cases]
        bs = gpu.BatchSolver(gpu.Batch(meshes), cases, dtype="f64")
        rc, st = bs.run(60)
        assert rc == 0
        states = [bs.numpy_state(k) for k in range(len(cases))]
        if ref is None:
            ref = (st, states)
            continue
        for k in range(len(cases)):
            assert st[k]["t"] == ref[0][k]["t"]
            for a, b in zip(states[k], ref[1][k]):
                assert np.array_equal(a, b)


def test_adjoint_gradients_do_not_depend_on_the_tile_size(gpu):
    from test_oracle_adjoint import tilted_calibration
    import oracle
    case = tilted_calibration()
    om = oracle.Mesh(case.xy, case.tri)
    dts, obs = oracle.observations(case, om, steps=40)
    ref = None
    for tile in TILES:
        mesh = gpu.Mesh(case.xy, case.tri, tile=tile)
        calib = gpu.Calibration(mesh, dts, case.extra["gauges"], obs, every=10, ckpt_every=7)
        j, grads = calib.run(case.n, case.z, case.h, case.hu, case.hv)
        if ref is None:
            ref = (j, grads)
            continue
        # the forward passes, and so J, are bitwise equal.  The tiled flux adjoint takes an
        # interface between two cells of one tile once, with the side-b cotangent coming out of
        # the same differentiation as side a's, and one that crosses tiles from each side; which
        # interfaces cross depends on the tile size, and the two ways agree up to rounding (the
        # bar of the tiled against the per-cell adjoint)
        assert j == ref[0]
        for which, a, b in zip(("n", "z", "h", "hu", "hv"), grads, ref[1]):
            scale = np.abs(b).max()
            print(f"tile {tile} d{which}: max |grad| {scale:.3e}, "
                  f"max difference {np.abs(a - b).max():.3e}", flush=True)
            assert np.abs(a - b).max() <= 1e-12 * scale


def test_tune_tiles_records_the_fastest_size_for_auto_meshes(gpu):
    case = gen.small(3)
    best, res = gpu.tune.tune_tiles(case.xy, case.tri, case.z, case.n, case.h, case.hu, case.hv,
                                    dtype="f64", steps=6)
    print(f"tile timings: { {t: r['ms_per_step'] for t, r in res.items()} }; best {best}")
    assert set(res) == set(TILES) and all(r["tile"] == t for t, r in res.items())
    best_ms = {t: min(v for v in r["ms_per_step"].values() if v > 0) for t, r in res.items()}
    assert best == min(best_ms, key=best_ms.get)
    got = gpu.tune.tuning("f64", case.n_cells)
    assert got["tile"] == best and got["variant"] == res[best]["variant"]
    auto = gpu.Mesh(case.xy, case.tri, tile="auto", dtype="f64")
    assert auto.tile == best
    # a recorded size another process saved is followed as well
    r = gpu.swe_tune_result()
    r.variant = gpu.SWE_TILED
    r.xcd_remap = 1
    r.tile_cells = 128 if best != 128 else 64
    gpu.swe_tune_set(auto.device.index, gpu.SWE_F64, case.n_cells, r)
    assert gpu.Mesh(case.xy, case.tri, tile="auto").tile == r.tile_cells
    gpu.tune.forget("f64", case.n_cells)
    assert gpu.Mesh(case.xy, case.tri, tile="auto").tile == gpu.SWE_TILE
