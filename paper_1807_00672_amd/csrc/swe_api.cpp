// C ABI of libswe: argument checks, launch sequencing and counters.  Device memory and streams
// belong to the caller; nothing here allocates device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "swe_internal.h"

namespace swe {

namespace {
thread_local std::string g_last_error;

int32_t fail(int32_t code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int32_t check_hip(int err, const char *where)
{
    if (err == hipSuccess) return SWE_OK;
    return fail(SWE_EDEVICE, std::string(where) + ": " +
                                 hipGetErrorString(static_cast<hipError_t>(err)));
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int32_t check_params(const swe_params *p, const char *where)
{
    if (!p) return fail(SWE_EINVAL, std::string(where) + ": null params");
    if (!(p->g > 0.0) || !isfinite(p->g)) return fail(SWE_EINVAL, std::string(where) + ": g must be > 0");
    if (!(p->courant > 0.0) || !(p->courant <= 1.0))
        return fail(SWE_EINVAL, std::string(where) + ": courant must be in (0, 1]");
    if (!(p->h_dry >= 0.0) || !isfinite(p->h_dry))
        return fail(SWE_EINVAL, std::string(where) + ": h_dry must be >= 0");
    if (p->dtype != SWE_F64 && p->dtype != SWE_F32)
        return fail(SWE_EINVAL, std::string(where) + ": dtype must be SWE_F64 or SWE_F32");
    if (p->n_inflow < 0 || p->n_inflow > SWE_MAX_INFLOW)
        return fail(SWE_EINVAL, std::string(where) + ": n_inflow out of range");
    if (p->n_inflow > 0 && !p->inflow_q)
        return fail(SWE_EINVAL, std::string(where) + ": null inflow_q");
    for (int k = 0; k < p->n_inflow; ++k)
        if (!(p->inflow_q[k] >= 0.0) || !isfinite(p->inflow_q[k]))
            return fail(SWE_EINVAL, std::string(where) + ": inflow_q must be finite and >= 0");
    return SWE_OK;
}

int32_t check_call(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                   const swe_state *s, const char *where)
{
    const std::string w(where);
    if (!mesh || !dm || !s) return fail(SWE_EINVAL, w + ": null mesh, device mesh or state");
    if (int32_t rc = check_params(p, where)) return rc;
    if (dm->n_cells != mesh->info.n_cells || dm->n_nodes != mesh->info.n_nodes)
        return fail(SWE_EINVAL, w + ": device mesh sizes differ from the mesh");
    if (!dm->nbr || !dm->c2n || !dm->xy || !(p->dtype == SWE_F64 ? (const void *)dm->cell_geo : (const void *)dm->cell_geo32))
        return fail(SWE_EINVAL, w + ": null device mesh array");
    if (!aligned(dm->xy, 16)) return fail(SWE_EINVAL, w + ": xy must be 16-byte aligned");
    if (mesh->info.n_inflow_segments > p->n_inflow)
        return fail(SWE_EINVAL, w + ": mesh has inflow segment " +
                                    std::to_string(mesh->info.n_inflow_segments) +
                                    " but params give " + std::to_string(p->n_inflow));
    for (int b = 0; b < 2; ++b)
        if (!s->h[b] || !s->hu[b] || !s->hv[b]) return fail(SWE_EINVAL, w + ": null state buffer");
    if (!s->z || !s->n || !s->ctrl || !s->work) return fail(SWE_EINVAL, w + ": null z, n, ctrl or work");
    if (!aligned(s->ctrl, 16)) return fail(SWE_EINVAL, w + ": ctrl must be 16-byte aligned");
    if (!aligned(s->work, 256)) return fail(SWE_EINVAL, w + ": work must be 256-byte aligned");
    if (s->cur != 0 && s->cur != 1) return fail(SWE_EINVAL, w + ": cur must be 0 or 1");
    return SWE_OK;
}

StepConfig make_config(const swe_mesh *mesh, const swe_params *p)
{
    StepConfig c;
    memset(&c, 0, sizeof(c));
    c.n_cells = mesh->info.n_cells;
    c.n_owned = mesh->info.n_owned;
    c.shard = (p->flags & SWE_SHARD) ? 1 : 0;
    c.index64 = (p->flags & SWE_INDEX64) ? 1 : 0;
    c.fast = (p->dtype == SWE_F64 && !(p->flags & SWE_EXACT)) ? 1 : 0;
    c.tile = mesh->info.tile_cells;
    c.g = p->g;
    c.courant = p->courant;
    c.h_dry = p->h_dry;
    c.n_inflow = p->n_inflow;
    for (int k = 0; k < p->n_inflow; ++k) c.inflow_q[k] = p->inflow_q[k];
    return c;
}

// Largest dynamic LDS of a workgroup on the current device, and whether the tiled kernels
// have been allowed to use more than the default 64 KiB there.
struct DeviceLds {
    int limit = -1;
    size_t prepared = 0;
};
DeviceLds g_lds[64];
std::mutex g_lds_mu;   // guards g_lds


// kGraphSteps steps (an even number: the state ends in the buffer it started from) captured
// once as a graph and replayed by swe_run; the launch arguments it bakes in form its key.
struct GraphKey {
    swe_dev_mesh dm;
    double g, courant, h_dry;
    int32_t dtype, variant, n_inflow, cur, remap, flags;
    double q[SWE_MAX_INFLOW];
    void *h[2], *hu[2], *hv[2];
    const void *z, *n;
    void *ctrl, *work;
    const double *dt_seq;
    int64_t n_seq;
    const void *tl;
    int device;
};

struct GraphEntry {
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;   // last use (GraphCache::tick); 0: empty
    void clear()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        used = 0;
    }
};

// A mesh's captured graphs, one per launch key (a state, a precision, a variant, a dt
// sequence...), so that runs alternating between a few keys (several states on one mesh, the
// tuner's candidates) replay their graphs instead of capturing again; the least recently used
// entry gives way when all are taken.
struct GraphCache {
    static constexpr int kEntries = 8;
    GraphEntry e[kEntries];
    uint64_t tick = 0;
    ~GraphCache()
    {
        for (GraphEntry &x : e) x.clear();
    }
};

// Per-device capture streams, created on first use; captures from several threads (on different
// meshes) take turns.
hipStream_t g_capture[64] = {};
std::mutex g_capture_mu;

GraphKey make_key(const swe_dev_mesh *dm, const swe_params *p, const swe_state *s,
                  const double *dt_seq, int64_t n_seq, const TileLayout *tl, int remap, int dev)
{
    GraphKey k;
    memset(&k, 0, sizeof(k));
    k.dm = *dm;
    k.g = p->g; k.courant = p->courant; k.h_dry = p->h_dry;
    k.dtype = p->dtype; k.variant = p->variant; k.n_inflow = p->n_inflow; k.cur = s->cur;
    k.remap = remap;
    k.flags = p->flags;
    for (int i = 0; i < p->n_inflow; ++i) k.q[i] = p->inflow_q[i];
    for (int b = 0; b < 2; ++b) { k.h[b] = s->h[b]; k.hu[b] = s->hu[b]; k.hv[b] = s->hv[b]; }
    k.z = s->z; k.n = s->n; k.ctrl = s->ctrl; k.work = s->work;
    k.dt_seq = dt_seq;
    k.n_seq = dt_seq ? n_seq : 0;
    k.tl = tl;
    k.device = dev;
    return k;
}

// The executable graph of kGraphSteps steps (an even number, so the state returns to the same
// buffer) for these arguments, captured on a library-owned stream (nullptr if graphs are
// unavailable: the caller then launches step by step).
hipGraphExec_t step_graph(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                              const StepConfig &cfg, const swe_state *s, const double *dt_seq,
                              int64_t n_seq, const TileLayout *tl, int remap)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    const GraphKey key = make_key(dm, p, s, dt_seq, n_seq, tl, remap, dev);
    swe_mesh *m = const_cast<swe_mesh *>(mesh);
    GraphCache *gc = static_cast<GraphCache *>(m->graph);
    if (!gc) {
        gc = new (std::nothrow) GraphCache();
        if (!gc) return nullptr;   // no host memory for the cache: the caller launches step by step
        m->graph = gc;
    }
    GraphEntry *slot = &gc->e[0];
    for (GraphEntry &x : gc->e) {
        if (x.used && memcmp(&x.key, &key, sizeof(key)) == 0) {
            x.used = ++gc->tick;
            return x.exec;
        }
        if (x.used < slot->used) slot = &x;   // an empty entry, else the least recently used
    }
    slot->clear();
    std::lock_guard<std::mutex> lk(g_capture_mu);
    if (!g_capture[dev] && hipStreamCreateWithFlags(&g_capture[dev], hipStreamNonBlocking) != hipSuccess) {
        g_capture[dev] = nullptr;
        return nullptr;
    }
    hipStream_t cs = g_capture[dev];
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    int e0 = hipSuccess;
    for (int q = 0; q < kGraphSteps && e0 == hipSuccess; ++q)
        e0 = launch_step(p->dtype, *dm, cfg, *s, (s->cur + q) & 1, dt_seq, n_seq, cs, tl, nullptr,
                         remap);
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
    slot->key = key;
    slot->graph = graph;
    slot->exec = exec;
    slot->used = ++gc->tick;
    return exec;
}

int32_t status_code(int32_t bits)
{
    if (bits & (kStatusNonFinite | kStatusBadDt)) return SWE_ENONFINITE;
    if (bits & kStatusDry) return SWE_EDRY;
    return SWE_OK;
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

// Pick the step kernel: SWE_CELL the per-cell one, SWE_TILED the tiled one (an error when it
// cannot run), SWE_AUTO the tiled one when the device mesh carries the tile arrays and a
// tile's LDS fits the device, else the per-cell one.
int32_t choose_variant(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                       const TileLayout **out, int *remap, const char *where)
{
    *out = nullptr;
    *remap = (p->flags & SWE_NO_XCD_REMAP) ? 0 : 1;
    const std::string w(where);
    if (p->variant != SWE_AUTO && p->variant != SWE_CELL && p->variant != SWE_TILED)
        return fail(SWE_EINVAL, w + ": unknown variant");
    if (p->flags & ~(SWE_NO_XCD_REMAP | SWE_SHARD | SWE_INDEX64 | SWE_EXACT))
        return fail(SWE_EINVAL, w + ": unknown flags");
    int variant = p->variant;
    if (variant == SWE_AUTO) {
        // a swe_tune result for this device, precision and size class decides, if there is one
        int dev = 0, tv = SWE_AUTO, trm = 1;
        if (hipGetDevice(&dev) == hipSuccess && tuned_choice(dev, p->dtype, mesh->info.n_cells, &tv, &trm)) {
            if (!(p->flags & SWE_NO_XCD_REMAP)) *remap = trm;
            if (tv == SWE_CELL) return SWE_OK;
        }
    }
    if (variant == SWE_CELL) return SWE_OK;
    const bool auto_ = variant == SWE_AUTO;
    const void *ev = p->dtype == SWE_F64 ? (const void *)dm->edge_vec : (const void *)dm->edge_vec32;
    const bool have = dm->halo_off && dm->halo && dm->edge_off && dm->edges && dm->slot && ev;
    if (have && !aligned(ev, p->dtype == SWE_F64 ? 16 : 8))
        return fail(SWE_EINVAL, w + ": edge vectors misaligned (16 bytes for FP64, 8 for FP32)");
    if (have && dm->tile_nodes && !aligned(dm->tile_nodes, 16))
        return fail(SWE_EINVAL, w + ": tile nodes misaligned (16 bytes)");
    if (!have) return auto_ ? SWE_OK : fail(SWE_EINVAL, w + ": device mesh has no tile arrays");
    int dev = 0;
    if (int32_t rc = check_hip(hipGetDevice(&dev), where)) return rc;
    if (dev < 0 || dev >= 64) return fail(SWE_EUNSUPPORTED, w + ": device index beyond 63");
    std::lock_guard<std::mutex> lk(g_lds_mu);
    DeviceLds &d = g_lds[dev];
    if (d.limit < 0) {
        int lim = 0;
        if (int32_t rc = check_hip(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), where))
            return rc;
        d.limit = lim - static_cast<int>(kTileStaticLdsMax);   // left for dynamic LDS
    }
    const size_t need = tile_lds_bytes_for(p->dtype, mesh->tiles);
    if (need > static_cast<size_t>(d.limit) && auto_) return SWE_OK;
    if (need > static_cast<size_t>(d.limit))
        return fail(SWE_EUNSUPPORTED, w + ": tile needs " + std::to_string(need) +
                                          " bytes of LDS, device allows " + std::to_string(d.limit));
    if (need + kTileStaticLdsMax > 65536 && d.prepared < need) {
        if (int32_t rc = check_hip(prepare_tile_kernels(static_cast<size_t>(d.limit)), where)) return rc;
        d.prepared = static_cast<size_t>(d.limit);
    }
    *out = &mesh->tiles;
    return SWE_OK;
}

}  // namespace swe

namespace swe {

int32_t run_steps(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                  swe_state *s, int64_t n_steps, const double *dt_seq, bool graphs, void *stream)
{
    if (int32_t rc = check_call(mesh, dm, p, s, "swe_run")) return rc;
    if (n_steps < 0) return fail(SWE_EINVAL, "swe_run: n_steps < 0");
    if (dt_seq && n_steps < 1) return fail(SWE_EINVAL, "swe_run: dt_seq needs n_steps >= 1");
    if (dt_seq && (p->flags & SWE_SHARD))
        return fail(SWE_EINVAL, "swe_run: a shard takes its dt from swe_shard_dt_combine");
    const StepConfig cfg = make_config(mesh, p);
    const TileLayout *tl = nullptr;
    int remap = 1;
    if (int32_t rc = choose_variant(mesh, dm, p, &tl, &remap, "swe_run")) return rc;
    if (int32_t rc = check_hip(launch_run_begin(*s, dt_seq, stream), "swe_run")) return rc;
    int64_t k = 0;
    if (graphs && n_steps >= 2 * kGraphSteps) {
        // graphs start from buffer 0, so one capture serves every run with these arguments: a
        // state in buffer 1 takes one step on its own first
        if (s->cur == 1) {
            if (int32_t rc = check_hip(launch_step(p->dtype, *dm, cfg, *s, s->cur, dt_seq, n_steps,
                                                   stream, tl, nullptr, remap),
                                       "swe_run"))
                return rc;
            s->cur ^= 1;
            k = 1;
        }
        if (hipGraphExec_t ex = step_graph(mesh, dm, p, cfg, s, dt_seq, n_steps, tl, remap)) {
            for (; k + kGraphSteps <= n_steps; k += kGraphSteps)
                if (int32_t rc = check_hip(hipGraphLaunch(ex, static_cast<hipStream_t>(stream)),
                                           "swe_run"))
                    return rc;
        }
    }
    for (; k < n_steps; ++k) {
        if (int32_t rc = check_hip(launch_step(p->dtype, *dm, cfg, *s, s->cur, dt_seq, n_steps,
                                               stream, tl, nullptr, remap),
                                   "swe_run"))
            return rc;
        s->cur ^= 1;
    }
    return SWE_OK;
}

}  // namespace swe

swe_mesh::~swe_mesh() { delete static_cast<swe::GraphCache *>(graph); }

using namespace swe;

extern "C" {

const char *swe_last_error(void) { return g_last_error.c_str(); }

int32_t swe_workspace_bytes(int64_t n_cells, int64_t *bytes)
{
    if (!bytes || n_cells < 1) return fail(SWE_EINVAL, "swe_workspace_bytes: bad argument");
    *bytes = workspace_bytes(n_cells);
    return SWE_OK;
}

int32_t swe_state_init(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                       swe_state *s, double t0, double t_end, void *stream)
{
    if (int32_t rc = check_call(mesh, dm, p, s, "swe_state_init")) return rc;
    if (!isfinite(t0) || !isfinite(t_end)) return fail(SWE_EINVAL, "swe_state_init: t0 and t_end must be finite");
    const StepConfig cfg = make_config(mesh, p);
    return check_hip(launch_init(p->dtype, *dm, cfg, *s, t0, t_end, stream), "swe_state_init");
}

int32_t swe_step(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                 swe_state *s, void *stream)
{
    if (int32_t rc = check_call(mesh, dm, p, s, "swe_step")) return rc;
    const StepConfig cfg = make_config(mesh, p);
    const TileLayout *tl = nullptr;
    int remap = 1;
    if (int32_t rc = choose_variant(mesh, dm, p, &tl, &remap, "swe_step")) return rc;
    if (int32_t rc = check_hip(launch_step(p->dtype, *dm, cfg, *s, s->cur, nullptr, 0, stream, tl, nullptr,
                                           remap),
                               "swe_step"))
        return rc;
    s->cur ^= 1;
    return SWE_OK;
}

int32_t swe_read_stats(swe_state *s, swe_run_stats *out, void *stream)
{
    if (!s || !out || !s->ctrl) return fail(SWE_EINVAL, "swe_read_stats: null argument");
    Ctrl c;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int32_t rc = check_hip(hipMemcpyAsync(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st),
                               "swe_read_stats"))
        return rc;
    if (int32_t rc = check_hip(hipStreamSynchronize(st), "swe_read_stats")) return rc;
    memset(out, 0, sizeof(*out));
    out->steps = c.steps;
    out->clamps = c.clamps;
    out->t = c.t;
    out->dt_next = c.dt;
    out->dt_min = c.dt_min;
    out->dt_max = c.dt_max;
    out->dt_sum = c.dt_sum;
    out->status = status_code(c.status);
    out->done = c.done;
    out->cur = static_cast<int32_t>((c.cur0 + c.steps) & 1);
    s->cur = out->cur;
    if (out->status != SWE_OK)
        g_last_error = out->status == SWE_EDRY ? "state has no wet cell: dt undefined"
                                               : "state or dt stopped being finite";
    return out->status;
}

int32_t swe_run(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                swe_state *s, int64_t n_steps, const double *dt_seq, swe_run_stats *out,
                void *stream)
{
    if (int32_t rc = run_steps(mesh, dm, p, s, n_steps, dt_seq, true, stream)) return rc;
    if (!out) return SWE_OK;
    return swe_read_stats(s, out, stream);
}

int32_t swe_flux_eval(int32_t dtype, int32_t flags, int64_t n, double g, double h_dry, const void *hl,
                      const void *hul, const void *hvl, const void *zl, const void *hr,
                      const void *hur, const void *hvr, const void *zr, const void *nx,
                      const void *ny, void *f, void *p, void *stream)
{
    if (dtype != SWE_F64 && dtype != SWE_F32) return fail(SWE_EINVAL, "swe_flux_eval: bad dtype");
    if (flags & ~SWE_EXACT) return fail(SWE_EINVAL, "swe_flux_eval: unknown flags");
    if (n < 0) return fail(SWE_EINVAL, "swe_flux_eval: n < 0");
    if (n == 0) return SWE_OK;
    if (!hl || !hul || !hvl || !zl || !nx || !ny || !f || !p)
        return fail(SWE_EINVAL, "swe_flux_eval: null argument");
    if (hr && (!hur || !hvr || !zr)) return fail(SWE_EINVAL, "swe_flux_eval: partial right state");
    if (!(g > 0.0) || !(h_dry >= 0.0)) return fail(SWE_EINVAL, "swe_flux_eval: bad g or h_dry");
    const bool fast_math = dtype == SWE_F64 && !(flags & SWE_EXACT);
    return check_hip(launch_flux_eval(dtype, fast_math, n, g, h_dry, hl, hul, hvl, zl, hr, hur, hvr,
                                      zr, nx, ny, f, p, stream),
                     "swe_flux_eval");
}

int32_t swe_halo_pack(int32_t dtype, int64_t n, const int32_t *idx, const void *h,
                      const void *hu, const void *hv, void *buf, void *stream)
{
    if (dtype != SWE_F64 && dtype != SWE_F32) return fail(SWE_EINVAL, "swe_halo_pack: bad dtype");
    if (n < 0 || n > INT32_MAX) return fail(SWE_EINVAL, "swe_halo_pack: bad n");
    if (n == 0) return SWE_OK;
    if (!idx || !h || !hu || !hv || !buf) return fail(SWE_EINVAL, "swe_halo_pack: null argument");
    return check_hip(launch_halo(dtype, true, n, idx, nullptr, buf, h, hu, hv, nullptr, nullptr,
                                 nullptr, stream),
                     "swe_halo_pack");
}

int32_t swe_halo_unpack(int32_t dtype, int64_t n, const int32_t *idx, const void *buf, void *h,
                        void *hu, void *hv, void *stream)
{
    if (dtype != SWE_F64 && dtype != SWE_F32) return fail(SWE_EINVAL, "swe_halo_unpack: bad dtype");
    if (n < 0 || n > INT32_MAX) return fail(SWE_EINVAL, "swe_halo_unpack: bad n");
    if (n == 0) return SWE_OK;
    if (!idx || !h || !hu || !hv || !buf) return fail(SWE_EINVAL, "swe_halo_unpack: null argument");
    return check_hip(launch_halo(dtype, false, n, idx, buf, nullptr, nullptr, nullptr, nullptr, h,
                                 hu, hv, stream),
                     "swe_halo_unpack");
}

int32_t swe_shard_dt_combine(void *const *ctrls, int32_t n, void *stream)
{
    if (!ctrls || n < 1 || n > kMaxShards)
        return fail(SWE_EINVAL, "swe_shard_dt_combine: need 1 to 64 control blocks");
    for (int32_t p = 0; p < n; ++p)
        if (!ctrls[p] || !aligned(ctrls[p], 16))
            return fail(SWE_EINVAL, "swe_shard_dt_combine: null or misaligned control block");
    return check_hip(launch_shard_combine(ctrls, n, stream), "swe_shard_dt_combine");
}

}  // extern "C"
