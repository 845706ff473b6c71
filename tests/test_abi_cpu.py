"""Host-side checks of libswe that need no GPU: the library loads, exports every function
include/swe.h declares, and its mesh builder agrees with the oracle's independent
connectivity (section 2.2 triangles; section 2.3 interfaces)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import gen
import oracle

swe = pytest.importorskip("paper_1807_00672_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert "swe_run" in names and "swe_mesh_create" in names and len(names) >= 11
    for n in names:
        assert hasattr(swe.lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", swe.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (swe_\w+)", out))
    assert set(names) <= exported
    assert set(names) == set(swe.EXPORTS)


def test_library_embeds_gfx950_code():
    with open(swe.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("morton", [True, False])
def test_mesh_builder_agrees_with_oracle_connectivity(k, morton):
    c = gen.small(k)
    m = swe.Mesh(c.xy, c.tri, morton=morton, device=None)
    om = oracle.Mesh(c.xy, c.tri)
    info = m.info
    assert (info.n_cells, info.n_nodes, info.n_edges, info.n_boundary_edges) == (
        om.n_cells, om.n_nodes, om.n_edges, om.n_boundary)
    assert info.n_nodes - info.n_edges + info.n_cells == 1
    assert 2 * info.n_edges == 3 * info.n_cells + info.n_boundary_edges
    t = m.n_cells
    perm = m.perm
    assert np.array_equal(np.sort(perm), np.arange(t))            # bijection
    if not morton:
        assert np.array_equal(perm, np.arange(t))
    ocn, onb, oarea, _ = om.arrays()
    # nodes: same counter-clockwise local order per cell, through both renumberings
    c2n = m.c2n.reshape(3, t).T
    assert np.array_equal(m.node_perm[c2n], ocn[perm])
    xy = m.xy.reshape(-1, 2)
    assert np.array_equal(xy, c.xy[m.node_perm])
    # neighbours: same cells across the same local edges, boundary codes kept
    nbr = m.nbr.reshape(3, t).T
    inner = nbr >= 0
    mapped = np.where(inner, perm[np.where(inner, nbr, 0)], nbr)
    assert np.array_equal(mapped, onb[perm])
    assert info.total_area == pytest.approx(oarea.sum(), rel=1e-13)
    # precomputed geometry: the oracle's areas and inradii bit for bit, and each edge-list
    # entry's vector from its owning cell's node k to node k+1
    _, _, _, oinr = om.arrays()
    assert np.array_equal(m.cell_geo[:t], oarea[perm])
    assert np.array_equal(m.cell_geo[t:], oinr[perm])
    ev = m.edge_vec.reshape(-1, 2)
    assert ev.shape[0] == info.n_tile_edges
    for tile in range(int(info.n_tiles)):
        e0, e1 = m.edge_off[tile], m.edge_off[tile + 1]
        w = m.edges[e0:e1].astype(np.int64)
        ca = tile * m.tile + (w & swe._abi.EDGE_A_MASK)
        k = (w >> swe._abi.EDGE_KA_SHIFT) & 3
        n0 = m.c2n.reshape(3, t)[k, ca]
        n1 = m.c2n.reshape(3, t)[(k + 1) % 3, ca]
        assert np.array_equal(ev[e0:e1], xy[n1] - xy[n0])
    # the float copies the FP32 step reads: rounded to nearest
    assert np.array_equal(m.edge_vec32, m.edge_vec.astype(np.float32))
    assert np.array_equal(m.cell_geo32, m.cell_geo.astype(np.float32))


def test_morton_order_brings_neighbours_closer():
    """Rows of 800 triangles: in input order a 256-cell tile holds a third of a row, so the
    neighbours above and below fall outside it; Morton tiles are compact."""
    c = gen.wetdry(nx=400, ny=200, steps=1)
    far, same = {}, {}
    for morton in (False, True):
        m = swe.Mesh(c.xy, c.tri, morton=morton, device=None)
        t = m.n_cells
        nbr = m.nbr.reshape(3, t).T
        i = np.repeat(np.arange(t)[:, None], 3, 1)
        ok = nbr >= 0
        far[morton] = np.percentile(np.abs(nbr[ok] - i[ok]), 90)
        same[morton] = (nbr[ok] // 256 == i[ok] // 256).mean()
    assert far[True] < far[False] / 8
    assert same[True] > 0.85 > 0.7 > same[False]


def test_hilbert_order_keeps_consecutive_cells_adjacent():
    """Along a Hilbert curve consecutive cells of the quantised grid are edge neighbours, so
    consecutive mesh cells stay close everywhere; a Morton curve jumps at every quadrant
    boundary.  Both keep tiles compact."""
    c = gen.wetdry(nx=128, ny=128, lx=1280.0, ly=1280.0, steps=1)   # 10 m squares
    jump, same = {}, {}
    for order in ("hilbert", "morton"):
        m = swe.Mesh(c.xy, c.tri, order=order, device=None)
        t = m.n_cells
        assert sorted(m.perm.tolist()) == list(range(t))
        xy = m.xy.reshape(-1, 2)[m.c2n.reshape(3, t)].mean(axis=0)   # centroids, mesh order
        jump[order] = np.linalg.norm(np.diff(xy, axis=0), axis=1).max()
        nbr = m.nbr.reshape(3, t).T
        i = np.repeat(np.arange(t)[:, None], 3, 1)
        ok = nbr >= 0
        same[order] = (nbr[ok] // 256 == i[ok] // 256).mean()
    assert jump["hilbert"] < 40.0 < 320.0 < jump["morton"]
    assert same["hilbert"] > 0.85 and same["morton"] > 0.85
    with pytest.raises(swe.SweError):
        swe.swe_mesh_create(c.xy, c.tri, None, swe.SWE_MORTON | swe.SWE_HILBERT)


def test_clockwise_input_and_edge_tags_are_reoriented():
    c = gen.ensemble_scenario(3)
    tri = c.tri.copy()
    tag = c.edge_tag.copy()
    flip = np.arange(len(tri)) % 3 == 0
    tri[flip] = tri[flip][:, [0, 2, 1]]        # clockwise: edges become (e2^-1, e1^-1, e0^-1)
    tag[flip] = tag[flip][:, [2, 1, 0]]
    a = swe.Mesh(c.xy, c.tri, c.edge_tag, device=None)
    b = swe.Mesh(c.xy, tri, tag, device=None)
    assert np.array_equal(a.nbr, b.nbr) and np.array_equal(a.c2n, b.c2n)
    assert a.info.n_inflow_edges == (c.edge_tag > 0).sum() == b.info.n_inflow_edges
    assert a.info.n_inflow_segments == 1
    assert (a.nbr == -2).sum() == a.info.n_inflow_edges


def test_bad_meshes_are_rejected_with_codes():
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 2]], float)
    ok = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    swe.Mesh(xy, ok, device=None)
    cases = {
        "node out of range": (np.array([[0, 1, 7]]), swe.SWE_EMESH),
        "repeated node": (np.array([[0, 1, 1]]), swe.SWE_EMESH),
        "zero area": (np.array([[0, 3, 4]]), swe.SWE_EMESH),
        "edge shared three times": (np.array([[0, 1, 2], [1, 3, 2], [1, 4, 2]]), swe.SWE_EMESH),
        "overlapping triangles": (np.array([[0, 1, 2], [0, 1, 3]]), swe.SWE_EMESH),
    }
    for name, (tri, code) in cases.items():
        with pytest.raises(swe.SweError) as e:
            swe.swe_mesh_create(xy, tri)
        assert e.value.code == code, name
        assert swe.swe_last_error()
    with pytest.raises(swe.SweError) as e:
        swe.swe_mesh_create(xy, np.zeros((0, 3), np.int32))
    assert e.value.code == swe.SWE_EINVAL
    bad = xy.copy()
    bad[4, 0] = np.nan
    with pytest.raises(swe.SweError) as e:
        swe.swe_mesh_create(bad, ok)
    assert e.value.code == swe.SWE_EINVAL
    out = C.c_void_p()
    assert swe.lib.swe_mesh_create(None, 5, None, 2, None, 0, C.byref(out)) == swe.SWE_EINVAL
    with pytest.raises(swe.SweError) as e:
        swe.swe_mesh_create(xy, ok, edge_tag=np.full((2, 3), 99))
    assert e.value.code == swe.SWE_EINVAL


def test_step_calls_reject_bad_arguments_without_touching_a_device():
    c = gen.small(1)
    m = swe.Mesh(c.xy, c.tri, device=None)
    dm = swe.swe_dev_mesh(m.n_cells, m.n_nodes, None, None, None)
    p = swe.swe_params(9.81, 0.7, 1e-6, swe.SWE_F64, 0, None)
    s = swe.swe_state()
    for bad in (swe.swe_params(0.0, 0.7, 1e-6, 0, 0, None), swe.swe_params(9.81, 1.5, 1e-6, 0, 0, None),
                swe.swe_params(9.81, 0.7, -1.0, 0, 0, None), swe.swe_params(9.81, 0.7, 1e-6, 7, 0, None)):
        assert swe.lib.swe_step(m.handle, C.byref(dm), C.byref(bad), C.byref(s), None) == swe.SWE_EINVAL
    assert swe.lib.swe_step(m.handle, C.byref(dm), C.byref(p), C.byref(s), None) == swe.SWE_EINVAL
    assert "null" in swe.swe_last_error()
    assert swe.lib.swe_run(None, None, None, None, 1, None, None, None) == swe.SWE_EINVAL
    assert swe.swe_workspace_bytes(10000) >= 40 * 16
    # the mesh geometry the kernels read: the cell areas and inradii for either kernel, the
    # edge vectors for the tiled one (stand-in addresses, never dereferenced on these paths)
    buf = np.zeros(1 << 16, np.uint8)
    a = (buf.ctypes.data + 255) // 256 * 256
    full = [a] * 8
    dm = swe.swe_dev_mesh(m.n_cells, m.n_nodes, *full, None, None, None, None)
    assert swe.lib.swe_step(m.handle, C.byref(dm), C.byref(p), C.byref(s), None) == swe.SWE_EINVAL
    assert "null device mesh array" in swe.swe_last_error()
    st = swe.swe_state()
    st.h[0] = st.h[1] = st.hu[0] = st.hu[1] = st.hv[0] = st.hv[1] = a
    st.z = st.n = st.ctrl = st.work = a
    tiled = swe.swe_params(9.81, 0.7, 1e-6, swe.SWE_F64, 0, None, swe.SWE_TILED, 0)
    dm = swe.swe_dev_mesh(m.n_cells, m.n_nodes, *full, None, a, None, None)
    assert swe.lib.swe_step(m.handle, C.byref(dm), C.byref(tiled), C.byref(st), None) == swe.SWE_EINVAL
    assert "tile arrays" in swe.swe_last_error()
    f32 = swe.swe_params(9.81, 0.7, 1e-6, swe.SWE_F32, 0, None, swe.SWE_TILED, 0)
    dm = swe.swe_dev_mesh(m.n_cells, m.n_nodes, *full, a, a, None, None)   # FP64 arrays only
    assert swe.lib.swe_step(m.handle, C.byref(dm), C.byref(f32), C.byref(st), None) == swe.SWE_EINVAL


@pytest.mark.parametrize("k,morton,tile", [(1, True, 256), (2, True, 256), (3, False, 256),
                                            (1, True, 64), (2, True, 128), (3, True, 512),
                                            (3, False, 512)])
def test_tile_lists_cover_every_interface_exactly_once_per_tile(k, morton, tile):
    """The tiled step evaluates, per tile of `tile` mesh-order cells, each interface between
    two tile cells once, each interface to a halo cell or to the boundary once, and each cell
    finds its three local edges through its slots."""
    c = gen.small(k)
    m = swe.Mesh(c.xy, c.tri, morton=morton, device=None, tile=tile)
    t = m.n_cells
    assert m.tile == m.info.tile_cells == tile
    nbr = m.nbr.reshape(3, t)
    slot = m.slot.reshape(3, t)
    info = m.info
    assert info.n_tiles == (t + tile - 1) // tile
    seen = set()
    for tt in range(info.n_tiles):
        s0, s1 = tt * tile, min(t, (tt + 1) * tile)
        halo = m.halo[m.halo_off[tt]:m.halo_off[tt + 1]]
        cells = np.arange(s0, s1)
        nb = nbr[:, s0:s1].ravel()
        expect = np.unique(nb[(nb >= 0) & ((nb < s0) | (nb >= s1))])
        assert np.array_equal(halo, expect)
        ent = m.edges[m.edge_off[tt]:m.edge_off[tt + 1]]
        a = (ent & swe._abi.EDGE_A_MASK).astype(np.int64)
        kk = ((ent >> swe._abi.EDGE_KA_SHIFT) & 3).astype(np.int64)
        b = (ent >> 16).astype(np.uint16).view(np.int16).astype(np.int64)
        assert (a < s1 - s0).all() and (kk < 3).all()
        # side b's local edge (bits 11-12) for interfaces between two tile cells: b's
        # neighbour across it is a; 0 for the others
        kb = ((ent >> swe._abi.EDGE_KB_SHIFT) & 3).astype(np.int64)
        assert ((ent >> 13) & 7 == 0).all()
        inner = (b >= 0) & (b < tile)
        assert (kb[~inner] == 0).all() and (kb < 3).all()
        assert (nbr[kb[inner], s0 + b[inner]] == s0 + a[inner]).all()
        bnd = b < 0
        assert not (bnd[:-1] & ~bnd[1:]).any()          # boundary entries last
        for e in range(len(ent)):
            ia = s0 + a[e]
            j = nbr[kk[e], ia]
            if b[e] < 0:
                assert j == b[e]
            elif b[e] < tile:
                assert j == s0 + b[e] and ia < j
            else:
                assert j == halo[b[e] - tile]
            key = (tt, min(ia, j) if j >= 0 else ia, max(ia, j) if j >= 0 else (kk[e], j))
            assert key not in seen
            seen.add(key)
        for i in cells:
            for q in range(3):
                sl = int(slot[q, i])
                e, side_b = sl & 0x7FFF, bool(sl & 0x8000)
                assert e < len(ent)
                if side_b:
                    assert b[e] == i - s0 and nbr[kk[e], s0 + a[e]] == i and nbr[q, i] == s0 + a[e]
                else:
                    assert a[e] == i - s0 and kk[e] == q
    assert info.n_tile_edges == len(m.edges) and info.max_halo == max(
        m.halo_off[1:] - m.halo_off[:-1])
    assert len(seen) == info.n_tile_edges


@pytest.mark.parametrize("k,order,tile", [(1, "morton", 256), (3, "hilbert", 256),
                                          (5, "morton", 256), (1, "morton", 128),
                                          (5, "morton", 64)])
def test_tile_node_lists_reproduce_the_edge_vectors_bitwise(k, order, tile):
    """Each tile's node list holds the distinct nodes of its cells, with their coordinates;
    each edge-list entry's two node ids give back its edge vector, bit for bit.  Lists are
    kept where every tile has at most min(256, tile) nodes (one per work-item)."""
    c = gen.small(k)
    m = swe.Mesh(c.xy, c.tri, order=order, device=None, tile=tile)
    t = m.n_cells
    info = m.info
    assert info.n_tile_nodes > 0 and 0 < info.max_tile_nodes <= min(256, tile)
    off, nodes, en = m.tile_node_off, m.tile_nodes.reshape(-1, 2), m.edge_nodes.astype(np.int64)
    assert off[0] == 0 and off[-1] == info.n_tile_nodes and (np.diff(off) > 0).all()
    assert np.diff(off).max() == info.max_tile_nodes
    xy, c2n = m.xy.reshape(-1, 2), m.c2n.reshape(3, t)
    ev = m.edge_vec.reshape(-1, 2)
    for tt in range(info.n_tiles):
        s0, s1 = tt * tile, min(t, (tt + 1) * tile)
        want = np.unique(c2n[:, s0:s1])
        tn = nodes[off[tt]:off[tt + 1]]
        assert len(tn) == len(want)
        assert np.array_equal(np.unique(tn, axis=0), np.unique(xy[want], axis=0))
        e0, e1 = m.edge_off[tt], m.edge_off[tt + 1]
        p0, p1 = tn[en[e0:e1] & 0xFF], tn[en[e0:e1] >> 8]
        assert np.array_equal(p1 - p0, ev[e0:e1])


def test_scattered_tiles_get_no_node_lists_and_batches_concatenate_them():
    """Tiles of 256 cells in random order touch far more than 256 nodes: no node lists (the
    FP64 tiled step then reads the edge vectors).  A batch keeps the lists of its scenarios,
    with their tile-local ids, when every scenario has them."""
    c = gen.small(5)
    perm = np.random.default_rng(3).permutation(c.n_cells)
    sc = swe.Mesh(c.xy, c.tri[perm], morton=False, device="cpu")
    assert sc.info.n_tile_nodes == 0 and sc.info.max_tile_nodes > 256
    assert sc.tile_nodes is None and sc.dev.tile_nodes is None
    cases = [gen.ensemble_scenario(s) for s in range(3)]
    meshes = [swe.Mesh(x.xy, x.tri, x.edge_tag, device=None) for x in cases]
    b = swe.Batch(meshes, device="cpu")
    i = b.info
    assert i.n_tile_nodes == sum(m.info.n_tile_nodes for m in meshes)
    assert i.max_tile_nodes == max(m.info.max_tile_nodes for m in meshes)
    off = swe.swe_batch_export(b.handle, swe._abi.SWE_ARR_TILE_NODE_OFF, int(i.n_tiles) + 1, np.int32)
    nodes = swe.swe_batch_export(b.handle, swe._abi.SWE_ARR_TILE_NODES, 2 * int(i.n_tile_nodes),
                                 np.float64).reshape(-1, 2)
    en = swe.swe_batch_export(b.handle, swe._abi.SWE_ARR_EDGE_NODES, int(i.n_tile_edges),
                              np.uint16).astype(np.int64)
    eoff = swe.swe_batch_export(b.handle, swe._abi.SWE_ARR_EDGE_OFF, int(i.n_tiles) + 1, np.int32)
    ev = swe.swe_batch_export(b.handle, swe._abi.SWE_ARR_EDGE_VEC, 2 * int(i.n_tile_edges),
                              np.float64).reshape(-1, 2)
    for tt in range(int(i.n_tiles)):
        tn = nodes[off[tt]:off[tt + 1]]
        e = slice(eoff[tt], eoff[tt + 1])
        assert np.array_equal(tn[en[e] >> 8] - tn[en[e] & 0xFF], ev[e])
    mixed = swe.Batch([meshes[0], sc], device="cpu")
    assert mixed.info.n_tile_nodes == 0 and "tile_nodes" not in mixed.d


def test_batch_concatenates_scenarios_without_straddling_tiles():
    cases = [gen.ensemble_scenario(s) for s in range(5)]
    meshes = [swe.Mesh(c.xy, c.tri, c.edge_tag, device=None) for c in cases]
    b = swe.swe_batch_create([m.handle for m in meshes])
    try:
        info = swe.swe_batch_info_get(b)
        n, t, nt = info.n_scenarios, info.n_cells, info.n_tiles
        assert n == 5 and t == sum(m.n_cells for m in meshes)
        assert nt == sum(m.info.n_tiles for m in meshes)
        ex = lambda w, k, dt: swe.swe_batch_export(b, w, k, dt)
        off = ex(swe._abi.SWE_BARR_CELL_OFF, n + 1, np.int64)
        start = ex(swe._abi.SWE_BARR_TILE_START, nt + 1, np.int32)
        scen = ex(swe._abi.SWE_BARR_TILE_SCEN, nt, np.int32)
        toff = ex(swe._abi.SWE_BARR_SCEN_TILE_OFF, n + 1, np.int32)
        nbr = ex(swe.SWE_ARR_NBR, 3 * t, np.int32).reshape(3, t)
        for s, m in enumerate(meshes):
            sl = slice(off[s], off[s + 1])
            local = m.nbr.reshape(3, m.n_cells)
            assert np.array_equal(np.where(local >= 0, local + off[s], local), nbr[:, sl])
            tiles = np.arange(toff[s], toff[s + 1])
            assert (scen[tiles] == s).all()
            assert start[tiles[0]] == off[s] and start[tiles[-1] + 1] == off[s + 1]
            assert (np.diff(start[toff[s]:toff[s + 1] + 1]) <= swe.SWE_TILE).all()
        assert info.max_inflow_segments == 1
        with pytest.raises(swe.SweError):
            swe.swe_batch_create([])
    finally:
        swe.swe_batch_destroy(b)


def test_tuning_table_records_erases_and_rejects_without_a_device():
    r = swe.swe_tune_result()
    r.variant, r.xcd_remap = swe.SWE_CELL, 0
    swe.swe_tune_set(5, swe.SWE_F32, 1000, r)
    got = swe.swe_tune_get(5, swe.SWE_F32, 1023)    # same size class floor(log2 n) = 9
    assert got.variant == swe.SWE_CELL and got.xcd_remap == 0
    assert swe.swe_tune_get(5, swe.SWE_F32, 1024).variant == swe.SWE_AUTO   # class 10
    assert swe.swe_tune_get(5, swe.SWE_F64, 1000).variant == swe.SWE_AUTO   # other precision
    assert swe.swe_tune_get(4, swe.SWE_F32, 1000).variant == swe.SWE_AUTO   # other device
    swe.swe_tune_set(5, swe.SWE_F32, 600, swe.swe_tune_result())           # SWE_AUTO erases
    assert swe.swe_tune_get(5, swe.SWE_F32, 1000).variant == swe.SWE_AUTO
    bad = swe.swe_tune_result()
    bad.variant = 9
    assert swe.lib.swe_tune_set(0, swe.SWE_F64, 10, C.byref(bad)) == swe.SWE_EINVAL
    bad.variant, bad.xcd_remap = swe.SWE_TILED, 2
    assert swe.lib.swe_tune_set(0, swe.SWE_F64, 10, C.byref(bad)) == swe.SWE_EINVAL
    assert swe.lib.swe_tune_get(0, 7, 10, C.byref(r)) == swe.SWE_EINVAL
    assert swe.lib.swe_tune(None, None, None, None, 10, None, None) == swe.SWE_EINVAL


@pytest.mark.parametrize("k,c0,c1", [(3, 0, 2500), (3, 2500, 7700), (3, 7700, 10200), (2, 1000, 1001)])
def test_shard_mesh_is_the_range_and_its_halo_with_matching_neighbours(k, c0, c1):
    c = gen.small(k)
    full = swe.Mesh(c.xy, c.tri, device=None)
    sh = swe.Mesh.shard(full, c0, c1, device=None)
    T, t = full.n_cells, sh.n_cells
    g = sh.global_ids.astype(np.int64)
    assert sh.n_owned == c1 - c0 and np.array_equal(g[:sh.n_owned], np.arange(c0, c1))
    fn = full.nbr.reshape(3, T)
    own = fn[:, c0:c1]
    halo = np.unique(own[(own >= 0) & ((own < c0) | (own >= c1))])
    assert np.array_equal(g[sh.n_owned:], halo)            # exactly the outside neighbours
    sn = sh.nbr.reshape(3, t)
    # owned cells keep their neighbours (through the global map) and boundary codes, in the
    # same local edge order
    mapped = np.where(sn[:, :sh.n_owned] >= 0, g[np.maximum(sn[:, :sh.n_owned], 0)],
                      sn[:, :sh.n_owned])
    assert np.array_equal(mapped, own)
    # halo cells: neighbours inside the shard are kept, the rest became walls
    hn = sn[:, sh.n_owned:]
    fh = fn[:, g[sh.n_owned:]]
    inside = np.isin(fh, g)
    assert np.array_equal(np.where(hn >= 0, g[np.maximum(hn, 0)], -1)[inside], fh[inside])
    assert np.all(hn[~inside & (fh >= 0)] == swe.SWE_WALL)
    # same triangles (coordinates of the nodes, counter-clockwise order kept)
    fxy, sxy = full.xy.reshape(-1, 2), sh.xy.reshape(-1, 2)
    assert np.array_equal(sxy[sh.c2n.reshape(3, t)], fxy[full.c2n.reshape(3, T)[:, g]])
    assert full.n_owned == T and np.array_equal(full.global_ids, np.arange(T))


def test_shard_keeps_inflow_tags_and_rejects_bad_ranges():
    c = gen.ensemble_scenario(0, t_max=6e3, t_min=5e3)
    full = swe.Mesh(c.xy, c.tri, c.edge_tag, device=None)
    T = full.n_cells
    sh = swe.Mesh.shard(full, 0, T // 2, device=None)
    codes = full.nbr.reshape(3, T)[:, : T // 2]
    assert np.array_equal(sh.nbr.reshape(3, -1)[:, : T // 2][codes < -1], codes[codes < -1])
    assert (codes < -1).any()
    for a, b in ((-1, 5), (5, 5), (10, 3), (0, T + 1)):
        with pytest.raises(swe.SweError):
            swe.swe_mesh_create_shard(full.handle, a, b)
    assert swe.lib.swe_shard_dt_combine(None, 1, None) == swe.SWE_EINVAL
    assert swe.lib.swe_halo_pack(0, 5, None, None, None, None, None, None) == swe.SWE_EINVAL
    assert swe.lib.swe_halo_pack(0, 0, None, None, None, None, None, None) == swe.SWE_OK


def test_python_binding_refuses_inputs_the_kernels_would_read_out_of_bounds():
    """The C calls take bare device pointers; the binding checks sizes before any of them:
    per-cell fields of the wrong shape, a batch with fewer cases than scenarios, gauges out of
    range or repeated, and a replayed dt sequence shorter than the run."""
    import torch
    case = gen.small(5)
    m = swe.Mesh(case.xy, case.tri, device="cpu")
    t = m.n_cells
    for bad in (case.h[:-1], np.concatenate([case.h, case.h]), case.h.reshape(-1, 1)):
        with pytest.raises(ValueError, match="one value per cell"):
            swe.Solver(m, case.z, case.n, bad, case.hu, case.hv)
    with pytest.raises(ValueError, match="one value per cell"):
        swe.Solver(m, case.z[:10], case.n, case.h, case.hu, case.hv)
    for g in ([-1, 3], [3, 3], [t], []):
        with pytest.raises(ValueError, match="gauges"):
            swe.Calibration(m, [0.1] * 20, g, np.zeros((2, max(len(g), 1))), every=10)
    with pytest.raises(ValueError, match="dt_seq"):
        swe.Calibration(m, [], [3], np.zeros((0, 1)), every=10)
    b = swe.Batch([m, m], device="cpu")
    with pytest.raises(ValueError, match="one case per scenario"):
        swe.BatchSolver(b, [case])
    s = swe.Solver.__new__(swe.Solver)   # only the dt_seq check of run, before any C call
    s.mesh = m
    with pytest.raises(ValueError, match="holds 5 values for 8 steps"):
        s.run(8, dt_seq=torch.zeros(5, dtype=torch.float64))


def test_tile_size_is_a_mesh_property():
    """swe_mesh_create takes at most one tile-size flag; shards keep their mesh's size and a
    batch takes meshes of one size only."""
    c = gen.small(1)
    for tile in (64, 128, 256, 512):
        m = swe.Mesh(c.xy, c.tri, device=None, tile=tile)
        assert m.info.tile_cells == tile and m.info.n_tiles == -(-c.n_cells // tile)
        sh = swe.Mesh.shard(m, 100, 3000, device=None)
        assert sh.info.tile_cells == tile
    out = C.c_void_p()
    xy = np.ascontiguousarray(c.xy, np.float64)
    tri = np.ascontiguousarray(c.tri, np.int32)
    two = swe.SWE_MORTON | swe._abi.SWE_TILE_64 | swe._abi.SWE_TILE_512
    assert swe.lib.swe_mesh_create(xy.ctypes.data, len(xy), tri.ctypes.data, len(tri), None,
                                   two, C.byref(out)) == swe.SWE_EINVAL
    with pytest.raises(ValueError):
        swe.Mesh(c.xy, c.tri, device=None, tile=100)
    a = swe.Mesh(c.xy, c.tri, device=None, tile=64)
    b = swe.Mesh(c.xy, c.tri, device=None, tile=128)
    h = (C.c_void_p * 2)(a.handle.value, b.handle.value)
    assert swe.lib.swe_batch_create(h, 2, C.byref(out)) == swe.SWE_EINVAL
    assert "tile sizes" in swe.swe_last_error()
    # workspace: room for the partials of the smallest tiles
    assert swe.swe_workspace_bytes(c.n_cells) >= 16 * (-(-c.n_cells // 64))


def test_adjoint_workspace_holds_checkpoints_segment_and_loss_shares():
    """swe_adjoint's workspace: the checkpoints, one recompute segment (states and U*), the
    adjoint state and the loss with a share per step; with ckpt_every = 1 every state and U*
    instead of the segment.  Bad step counts and intervals are rejected."""
    c = gen.small(1)
    m = swe.Mesh(c.xy, c.tri, device=None)
    st = 3 * m.n_cells * 8   # one state (h, hu, hv) in doubles

    def ws(n, k):
        return swe.swe_adjoint_workspace_bytes(m.handle, n, k)

    n, k = 200, 50
    n_ckpt = -(-n // k) + 1
    assert ws(n, k) >= st * n_ckpt + st * (k + 1) + st * k + 3 * st + 8 * (n + 1)
    assert ws(n, 1) >= st * (n + 1) + st * n + 3 * st + 8 * (n + 1)
    # an interval beyond both step counts keeps the checkpoints and the segment: what a
    # thousand more steps add is the loss shares, a double each (256-byte aligned)
    grow = ws(2000, 5000) - ws(1000, 5000)
    assert 8 * 1000 - 256 <= grow <= 8 * 1000 + 256
    for bad in ((0, 50), (200, 0), (-1, 1)):
        with pytest.raises(swe.SweError):
            ws(*bad)
