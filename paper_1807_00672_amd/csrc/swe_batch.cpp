// Batches: many scenarios (independent meshes with their own dt and time) stepped by one launch
// of the step kernel (tiled or per-cell) per step.  The builder concatenates built meshes so that no tile straddles
// two scenarios; the per-tile scenario index selects the control block (dt, time, counters)
// and the inflow discharges, and a dt pass with one workgroup per scenario reduces each
// scenario's tile partials on its own.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "swe_internal.h"

struct swe_batch {
    swe_batch_info info;
    std::vector<int64_t> cell_off, node_off;
    std::vector<int32_t> tile_start, tile_scen, scen_tile_off;
    std::vector<int32_t> perm, nbr, c2n, halo_off, halo, edge_off, tile_node_off;
    std::vector<uint32_t> edges;
    std::vector<uint16_t> slot, edge_nodes;
    std::vector<double> xy, edge_vec, cell_geo, tile_nodes;
    swe::TileLayout tiles;
    void *graph = nullptr;
    ~swe_batch();
};

namespace swe {
namespace {

int32_t bfail(int32_t code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int32_t bcheck_hip(int err, const char *where)
{
    if (err == hipSuccess) return SWE_OK;
    return bfail(SWE_EDEVICE, std::string(where) + ": " +
                                  hipGetErrorString(static_cast<hipError_t>(err)));
}

struct BatchGraph {
    unsigned char key[512];
    size_t key_len = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Per-device capture streams, created on first use; captures from several threads (on different
// batches) take turns.
hipStream_t g_bcapture[64] = {};
std::mutex g_bcapture_mu;
int g_blimit[64];
bool g_blimit_known[64] = {};
size_t g_bprepared[64] = {};
std::mutex g_blimit_mu;   // guards g_blimit, g_blimit_known and g_bprepared

int32_t check_batch_call(const swe_batch *b, const swe_batch_dev *d, const swe_batch_params *p,
                         const swe_state *s, const char *where)
{
    const std::string w(where);
    if (!b || !d || !p || !s) return bfail(SWE_EINVAL, w + ": null argument");
    if (!(p->g > 0.0) || !(p->courant > 0.0) || !(p->courant <= 1.0) || !(p->h_dry >= 0.0))
        return bfail(SWE_EINVAL, w + ": bad g, courant or h_dry");
    if (p->dtype != SWE_F64 && p->dtype != SWE_F32) return bfail(SWE_EINVAL, w + ": bad dtype");
    if (p->variant != SWE_AUTO && p->variant != SWE_CELL && p->variant != SWE_TILED)
        return bfail(SWE_EINVAL, w + ": unknown variant");
    if (p->flags & ~(SWE_NO_XCD_REMAP | SWE_EXACT)) return bfail(SWE_EINVAL, w + ": unknown flags");
    if (b->info.max_inflow_segments > 0 && !p->inflow_q)
        return bfail(SWE_EINVAL, w + ": scenarios have inflow segments but inflow_q is null");
    const swe_dev_mesh &m = d->mesh;
    if (m.n_cells != b->info.n_cells || m.n_nodes != b->info.n_nodes)
        return bfail(SWE_EINVAL, w + ": device arrays sized for another batch");
    const bool f64 = p->dtype == SWE_F64;
    const void *ev = f64 ? (const void *)m.edge_vec : (const void *)m.edge_vec32;
    const void *cg = f64 ? (const void *)m.cell_geo : (const void *)m.cell_geo32;
    if (!m.nbr || !m.c2n || !m.xy || !m.halo_off || !m.halo || !m.edge_off || !m.edges ||
        !m.slot || !ev || !cg || !d->tile_start || !d->tile_scen || !d->scen_tile_off)
        return bfail(SWE_EINVAL, w + ": null device array");
    if (reinterpret_cast<uintptr_t>(m.xy) % 16 || reinterpret_cast<uintptr_t>(ev) % (f64 ? 16 : 8))
        return bfail(SWE_EINVAL, w + ": xy or edge vectors misaligned");
    if (reinterpret_cast<uintptr_t>(m.tile_nodes) % 16)
        return bfail(SWE_EINVAL, w + ": tile nodes misaligned");
    for (int k = 0; k < 2; ++k)
        if (!s->h[k] || !s->hu[k] || !s->hv[k]) return bfail(SWE_EINVAL, w + ": null state buffer");
    if (!s->z || !s->n || !s->ctrl || !s->work) return bfail(SWE_EINVAL, w + ": null z, n, ctrl or work");
    if (reinterpret_cast<uintptr_t>(s->ctrl) % 16 || reinterpret_cast<uintptr_t>(s->work) % 256)
        return bfail(SWE_EINVAL, w + ": ctrl or work misaligned");
    if (s->cur != 0 && s->cur != 1) return bfail(SWE_EINVAL, w + ": cur must be 0 or 1");
    return SWE_OK;
}

StepConfig batch_config(const swe_batch *b, const swe_batch_params *p)
{
    StepConfig c;
    memset(&c, 0, sizeof(c));
    c.n_cells = b->info.n_cells;
    c.n_owned = b->info.n_cells;
    c.fast = (p->dtype == SWE_F64 && !(p->flags & SWE_EXACT)) ? 1 : 0;
    c.tile = b->tiles.tile;
    c.g = p->g;
    c.courant = p->courant;
    c.h_dry = p->h_dry;
    c.n_inflow = b->info.max_inflow_segments;
    return c;
}

BatchLaunch launch_view(const swe_batch *b, const swe_batch_dev *d, const swe_batch_params *p)
{
    BatchLaunch l;
    l.tile_start = d->tile_start;
    l.tile_scen = d->tile_scen;
    l.scen_tile_off = d->scen_tile_off;
    l.q_table = p->inflow_q;
    l.n_scen = b->info.n_scenarios;
    l.n_tiles = b->info.n_tiles;
    return l;
}

// The tile's LDS must fit the device; allow more than the default 64 KiB when needed.
// Whether a batch step runs the tiled kernel (choose_variant's rule: SWE_AUTO takes it when a
// tile's LDS fits the device); an explicit SWE_TILED that cannot run is an error.
int32_t check_lds(const swe_batch *b, int dtype, int variant, bool *tiled, const char *where)
{
    *tiled = false;
    if (variant == SWE_CELL) return SWE_OK;
    int dev = 0;
    if (int32_t rc = bcheck_hip(hipGetDevice(&dev), where)) return rc;
    if (dev < 0 || dev >= 64) return bfail(SWE_EUNSUPPORTED, std::string(where) + ": device index");
    std::lock_guard<std::mutex> lk(g_blimit_mu);
    if (!g_blimit_known[dev]) {
        int lim = 0;
        if (int32_t rc = bcheck_hip(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                                    where))
            return rc;
        g_blimit[dev] = lim - static_cast<int>(kTileStaticLdsMax);   // left for dynamic LDS
        g_blimit_known[dev] = true;
    }
    const size_t need = tile_lds_bytes_for(dtype, b->tiles);
    if (need > static_cast<size_t>(g_blimit[dev]) && variant == SWE_AUTO) return SWE_OK;
    if (need > static_cast<size_t>(g_blimit[dev]))
        return bfail(SWE_EUNSUPPORTED, std::string(where) + ": a tile needs " + std::to_string(need) +
                                           " bytes of LDS");
    if (need + kTileStaticLdsMax > 65536 && g_bprepared[dev] < need) {
        if (int32_t rc = bcheck_hip(prepare_tile_kernels(static_cast<size_t>(g_blimit[dev])), where))
            return rc;
        g_bprepared[dev] = static_cast<size_t>(g_blimit[dev]);
    }
    *tiled = true;
    return SWE_OK;
}

hipGraphExec_t batch_graph(const swe_batch *b, const swe_batch_dev *d, const swe_batch_params *p,
                           const StepConfig &cfg, const swe_state *s, bool tiled)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    unsigned char key[512];
    size_t n = 0;
    auto put = [&](const void *v, size_t len) {
        memcpy(key + n, v, len);
        n += len;
    };
    put(d, sizeof(*d));
    put(p, sizeof(*p));
    put(s, sizeof(*s));
    put(&dev, sizeof(dev));
    swe_batch *mb = const_cast<swe_batch *>(b);
    BatchGraph *g = static_cast<BatchGraph *>(mb->graph);
    if (g && g->key_len == n && memcmp(g->key, key, n) == 0) return g->exec;
    delete g;
    mb->graph = nullptr;
    std::lock_guard<std::mutex> lk(g_bcapture_mu);
    if (!g_bcapture[dev] && hipStreamCreateWithFlags(&g_bcapture[dev], hipStreamNonBlocking) != hipSuccess) {
        g_bcapture[dev] = nullptr;
        return nullptr;
    }
    hipStream_t cs = g_bcapture[dev];
    const BatchLaunch bl = launch_view(b, d, p);
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    const TileLayout *tl = tiled ? &b->tiles : nullptr;
    const int rm = (p->flags & SWE_NO_XCD_REMAP) ? 0 : 1;
    int e0 = hipSuccess;
    for (int q = 0; q < kGraphSteps && e0 == hipSuccess; ++q)
        e0 = launch_step(p->dtype, d->mesh, cfg, *s, (s->cur + q) & 1, nullptr, 0, cs, tl, &bl, rm);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (e0 != hipSuccess || ee != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    g = new (std::nothrow) BatchGraph();
    if (!g) {   // no host memory for the cache: the caller launches step by step
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return nullptr;
    }
    memcpy(g->key, key, n);
    g->key_len = n;
    g->graph = graph;
    g->exec = exec;
    mb->graph = g;
    return exec;
}

}  // namespace
}  // namespace swe

swe_batch::~swe_batch() { delete static_cast<swe::BatchGraph *>(graph); }

using namespace swe;

extern "C" {

int32_t swe_batch_create(const swe_mesh *const *meshes, int32_t n, swe_batch **out)
{
    if (!out) return bfail(SWE_EINVAL, "swe_batch_create: null out");
    *out = nullptr;
    if (!meshes || n < 1) return bfail(SWE_EINVAL, "swe_batch_create: need at least one mesh");
    for (int32_t s = 0; s < n; ++s)
        if (!meshes[s]) return bfail(SWE_EINVAL, "swe_batch_create: null mesh " + std::to_string(s));
    swe_batch *b = nullptr;
    try {
        b = new swe_batch();
        memset(&b->info, 0, sizeof(b->info));
        b->cell_off.assign(n + 1, 0);
        b->node_off.assign(n + 1, 0);
        b->scen_tile_off.assign(n + 1, 0);
        int64_t nt_total = 0, nh = 0, ne = 0, nn = 0;
        bool nodes = true;   // node lists only if every scenario has them
        const int32_t tile = meshes[0]->info.tile_cells;
        for (int32_t s = 0; s < n; ++s) {
            const swe_mesh_info &mi = meshes[s]->info;
            if (mi.tile_cells != tile) {
                delete b;
                return bfail(SWE_EINVAL, "swe_batch_create: the meshes have different tile sizes");
            }
            b->cell_off[s + 1] = b->cell_off[s] + mi.n_cells;
            b->node_off[s + 1] = b->node_off[s] + mi.n_nodes;
            nt_total += mi.n_tiles;
            nh += mi.n_halo;
            ne += mi.n_tile_edges;
            b->info.max_inflow_segments = std::max(b->info.max_inflow_segments, mi.n_inflow_segments);
            b->tiles.max_halo = std::max(b->tiles.max_halo, mi.max_halo);
            b->tiles.max_edges = std::max(b->tiles.max_edges, mi.max_tile_edges);
            b->info.max_tile_nodes = std::max(b->info.max_tile_nodes, mi.max_tile_nodes);
            nn += mi.n_tile_nodes;
            if (meshes[s]->tile_node_off.empty()) nodes = false;
        }
        const int64_t T = b->cell_off[n], V = b->node_off[n];
        if (T > INT32_MAX / 3 || V > INT32_MAX / 2 || nt_total >= INT32_MAX || nh >= INT32_MAX ||
            ne >= INT32_MAX || nn >= INT32_MAX) {
            delete b;
            return bfail(SWE_EINVAL, "swe_batch_create: batch too large for int32 indices");
        }
        b->nbr.resize(3 * T);
        b->c2n.resize(3 * T);
        b->slot.resize(3 * T);
        b->perm.resize(T);
        b->xy.resize(2 * V);
        b->cell_geo.resize(2 * T);
        b->edge_vec.reserve(2 * ne);
        b->tile_start.reserve(nt_total + 1);
        b->tile_scen.reserve(nt_total);
        b->halo_off.assign(1, 0);
        b->edge_off.assign(1, 0);
        b->halo.reserve(nh);
        b->edges.reserve(ne);
        if (nodes) {
            b->tile_node_off.assign(1, 0);
            b->tile_nodes.reserve(2 * nn);
            b->edge_nodes.reserve(ne);
        }
        for (int32_t s = 0; s < n; ++s) {
            const swe_mesh &m = *meshes[s];
            const int64_t Ts = m.info.n_cells, c0 = b->cell_off[s], v0 = b->node_off[s];
            for (int k = 0; k < 3; ++k)
                for (int64_t i = 0; i < Ts; ++i) {
                    const int32_t j = m.nbr[k * Ts + i];
                    b->nbr[k * T + c0 + i] = j >= 0 ? static_cast<int32_t>(j + c0) : j;
                    b->c2n[k * T + c0 + i] = static_cast<int32_t>(m.c2n[k * Ts + i] + v0);
                    b->slot[k * T + c0 + i] = m.slot[k * Ts + i];
                }
            for (int64_t i = 0; i < Ts; ++i) {
                b->perm[c0 + i] = m.perm[i];
                b->cell_geo[c0 + i] = m.cell_geo[i];
                b->cell_geo[T + c0 + i] = m.cell_geo[Ts + i];
            }
            memcpy(&b->xy[2 * v0], m.xy.data(), sizeof(double) * 2 * m.info.n_nodes);
            for (int64_t t = 0; t < m.info.n_tiles; ++t) {
                b->tile_start.push_back(static_cast<int32_t>(c0 + t * tile));
                b->tile_scen.push_back(s);
                for (int32_t q = m.halo_off[t]; q < m.halo_off[t + 1]; ++q)
                    b->halo.push_back(static_cast<int32_t>(m.halo[q] + c0));
                b->halo_off.push_back(static_cast<int32_t>(b->halo.size()));
                b->edges.insert(b->edges.end(), m.edges.begin() + m.edge_off[t],
                                m.edges.begin() + m.edge_off[t + 1]);
                b->edge_vec.insert(b->edge_vec.end(), m.edge_vec.begin() + 2 * m.edge_off[t],
                                   m.edge_vec.begin() + 2 * m.edge_off[t + 1]);
                b->edge_off.push_back(static_cast<int32_t>(b->edges.size()));
                if (nodes) {   // ids are tile-local: copied as they are
                    b->edge_nodes.insert(b->edge_nodes.end(), m.edge_nodes.begin() + m.edge_off[t],
                                         m.edge_nodes.begin() + m.edge_off[t + 1]);
                    b->tile_nodes.insert(b->tile_nodes.end(), m.tile_nodes.begin() + 2 * m.tile_node_off[t],
                                         m.tile_nodes.begin() + 2 * m.tile_node_off[t + 1]);
                    b->tile_node_off.push_back(static_cast<int32_t>(b->tile_nodes.size() / 2));
                }
            }
            b->scen_tile_off[s + 1] = static_cast<int32_t>(b->tile_scen.size());
        }
        b->tile_start.push_back(static_cast<int32_t>(T));
        b->info.n_scenarios = n;
        b->info.n_cells = T;
        b->info.n_nodes = V;
        b->info.n_tiles = nt_total;
        b->info.n_halo = static_cast<int64_t>(b->halo.size());
        b->info.n_tile_edges = static_cast<int64_t>(b->edges.size());
        b->info.max_halo = b->tiles.max_halo;
        b->info.max_tile_edges = b->tiles.max_edges;
        b->tiles.n_tiles = nt_total;
        b->info.n_tile_nodes = static_cast<int64_t>(b->tile_nodes.size() / 2);
        b->tiles.max_nodes = nodes ? b->info.max_tile_nodes : 0;
        b->tiles.tile = tile;
        b->info.tile_cells = tile;
    } catch (...) {
        delete b;
        return bfail(SWE_EINVAL, "swe_batch_create: out of host memory");
    }
    *out = b;
    return SWE_OK;
}

int32_t swe_batch_info_get(const swe_batch *batch, swe_batch_info *out)
{
    if (!batch || !out) return bfail(SWE_EINVAL, "swe_batch_info_get: null argument");
    *out = batch->info;
    return SWE_OK;
}

int32_t swe_batch_export(const swe_batch *b, int32_t which, void *dst, int64_t dst_bytes)
{
    if (!b || !dst) return bfail(SWE_EINVAL, "swe_batch_export: null argument");
    const void *src = nullptr;
    int64_t bytes = 0;
    auto pick = [&](const auto &v) {
        src = v.data();
        bytes = static_cast<int64_t>(v.size() * sizeof(v[0]));
    };
    switch (which) {
    case SWE_ARR_PERM: pick(b->perm); break;
    case SWE_ARR_NBR: pick(b->nbr); break;
    case SWE_ARR_C2N: pick(b->c2n); break;
    case SWE_ARR_XY: pick(b->xy); break;
    case SWE_ARR_HALO_OFF: pick(b->halo_off); break;
    case SWE_ARR_HALO: pick(b->halo); break;
    case SWE_ARR_EDGE_OFF: pick(b->edge_off); break;
    case SWE_ARR_EDGES: pick(b->edges); break;
    case SWE_ARR_SLOT: pick(b->slot); break;
    case SWE_ARR_EDGE_VEC: pick(b->edge_vec); break;
    case SWE_ARR_CELL_GEO: pick(b->cell_geo); break;
    case SWE_ARR_EDGE_VEC32: return export_as_float(b->edge_vec, dst, dst_bytes, "swe_batch_export");
    case SWE_ARR_CELL_GEO32: return export_as_float(b->cell_geo, dst, dst_bytes, "swe_batch_export");
    case SWE_ARR_TILE_NODE_OFF: pick(b->tile_node_off); break;
    case SWE_ARR_TILE_NODES: pick(b->tile_nodes); break;
    case SWE_ARR_EDGE_NODES: pick(b->edge_nodes); break;
    case SWE_BARR_CELL_OFF: pick(b->cell_off); break;
    case SWE_BARR_NODE_OFF: pick(b->node_off); break;
    case SWE_BARR_TILE_START: pick(b->tile_start); break;
    case SWE_BARR_TILE_SCEN: pick(b->tile_scen); break;
    case SWE_BARR_SCEN_TILE_OFF: pick(b->scen_tile_off); break;
    default: return bfail(SWE_EINVAL, "swe_batch_export: unknown array " + std::to_string(which));
    }
    if (dst_bytes < bytes) return bfail(SWE_EINVAL, "swe_batch_export: destination too small");
    if (bytes) memcpy(dst, src, static_cast<size_t>(bytes));
    return SWE_OK;
}

void swe_batch_destroy(swe_batch *batch) { delete batch; }

int32_t swe_batch_workspace_bytes(const swe_batch *batch, int64_t *bytes)
{
    if (!batch || !bytes) return bfail(SWE_EINVAL, "swe_batch_workspace_bytes: null argument");
    *bytes = workspace_bytes_for_tiles(batch->info.n_tiles);
    return SWE_OK;
}

int32_t swe_batch_state_init(const swe_batch *batch, const swe_batch_dev *dev,
                             const swe_batch_params *p, swe_state *s, double t0, double t_end,
                             void *stream)
{
    if (int32_t rc = check_batch_call(batch, dev, p, s, "swe_batch_state_init")) return rc;
    if (!isfinite(t0) || !isfinite(t_end)) return bfail(SWE_EINVAL, "swe_batch_state_init: bad t0/t_end");
    const StepConfig cfg = batch_config(batch, p);
    const BatchLaunch bl = launch_view(batch, dev, p);
    return bcheck_hip(launch_init(p->dtype, dev->mesh, cfg, *s, t0, t_end, stream, &bl),
                      "swe_batch_state_init");
}

int32_t swe_batch_run(const swe_batch *batch, const swe_batch_dev *dev,
                      const swe_batch_params *p, swe_state *s, int64_t n_steps,
                      swe_run_stats *out, void *stream)
{
    if (int32_t rc = check_batch_call(batch, dev, p, s, "swe_batch_run")) return rc;
    if (n_steps < 0) return bfail(SWE_EINVAL, "swe_batch_run: n_steps < 0");
    bool tiled = false;
    if (int32_t rc = check_lds(batch, p->dtype, p->variant, &tiled, "swe_batch_run")) return rc;
    const StepConfig cfg = batch_config(batch, p);
    const BatchLaunch bl = launch_view(batch, dev, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t k = 0;
    if (n_steps >= 2 * kGraphSteps) {
        // the graph starts from buffer 0 (one capture serves every run): a state in buffer 1
        // takes one step on its own first
        if (s->cur == 1) {
            if (int32_t rc = bcheck_hip(launch_step(p->dtype, dev->mesh, cfg, *s, s->cur, nullptr,
                                                    0, stream, tiled ? &batch->tiles : nullptr,
                                                    &bl, (p->flags & SWE_NO_XCD_REMAP) ? 0 : 1),
                                        "swe_batch_run"))
                return rc;
            s->cur ^= 1;
            k = 1;
        }
        if (hipGraphExec_t ex = batch_graph(batch, dev, p, cfg, s, tiled)) {
            for (; k + kGraphSteps <= n_steps; k += kGraphSteps)
                if (int32_t rc = bcheck_hip(hipGraphLaunch(ex, st), "swe_batch_run")) return rc;
        }
    }
    for (; k < n_steps; ++k) {
        if (int32_t rc = bcheck_hip(launch_step(p->dtype, dev->mesh, cfg, *s, s->cur, nullptr, 0,
                                                stream, tiled ? &batch->tiles : nullptr,
                                                &bl, (p->flags & SWE_NO_XCD_REMAP) ? 0 : 1),
                                    "swe_batch_run"))
            return rc;
        s->cur ^= 1;
    }
    if (!out) return SWE_OK;
    const int32_t n = batch->info.n_scenarios;
    std::vector<unsigned char> host(static_cast<size_t>(n) * SWE_CTRL_BYTES);
    if (int32_t rc = bcheck_hip(hipMemcpyAsync(host.data(), s->ctrl, host.size(),
                                               hipMemcpyDeviceToHost, st),
                                "swe_batch_run"))
        return rc;
    if (int32_t rc = bcheck_hip(hipStreamSynchronize(st), "swe_batch_run")) return rc;
    int32_t first = SWE_OK;
    for (int32_t q = 0; q < n; ++q) {
        Ctrl c;
        memcpy(&c, host.data() + static_cast<size_t>(q) * SWE_CTRL_BYTES, sizeof(c));
        swe_run_stats &o = out[q];
        memset(&o, 0, sizeof(o));
        o.steps = c.steps;
        o.clamps = c.clamps;
        o.t = c.t;
        o.dt_next = c.dt;
        o.dt_min = c.dt_min;
        o.dt_max = c.dt_max;
        o.dt_sum = c.dt_sum;
        o.status = (c.status & (kStatusNonFinite | kStatusBadDt)) ? SWE_ENONFINITE
                   : (c.status & kStatusDry)                      ? SWE_EDRY
                                                                   : SWE_OK;
        o.done = c.done;
        o.cur = static_cast<int32_t>((c.cur0 + c.steps) & 1);
        if (o.status != SWE_OK && first == SWE_OK) first = o.status;
    }
    if (first != SWE_OK) set_error("a scenario of the batch stopped with an error");
    return first;
}

}  // extern "C"
