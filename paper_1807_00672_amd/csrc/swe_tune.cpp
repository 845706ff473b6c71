// Autotuning of the step launch: which kernel variant (per-cell gather or LDS-tiled) and which
// workgroup order (XCD-contiguous tiles or the hardware order) run fastest on this device for
// a precision and a mesh size class.  Results live in a process-wide table that SWE_AUTO
// consults; callers may persist them (swe_tune_get / swe_tune_set).  The choice never changes
// results: every candidate computes the same bits.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>

#include "swe_internal.h"

namespace swe {

namespace {

using Key = std::tuple<int, int, int>;   // device, dtype, size class

std::mutex g_mu;
std::map<Key, swe_tune_result> g_table;

int size_class(int64_t n_cells)
{
    int c = 0;
    while (c < 62 && (int64_t{1} << (c + 1)) <= n_cells) ++c;
    return c;   // floor(log2(n_cells))
}

int32_t tfail(int32_t code, const std::string &msg)
{
    set_error(msg);
    return code;
}

}  // namespace

bool tuned_choice(int device, int dtype, int64_t n_cells, int *variant, int *remap)
{
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_table.find(Key{device, dtype, size_class(n_cells)});
    if (it == g_table.end()) return false;
    *variant = it->second.variant;
    *remap = it->second.xcd_remap;
    return true;
}

}  // namespace swe

using namespace swe;

extern "C" {

int32_t swe_tune(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                 swe_state *s, int32_t n_steps, swe_tune_result *out, void *stream)
{
    if (!mesh || !dm || !p || !s || !out) return tfail(SWE_EINVAL, "swe_tune: null argument");
    if (n_steps < 2) return tfail(SWE_EINVAL, "swe_tune: n_steps must be >= 2");
    if (p->flags & SWE_SHARD) return tfail(SWE_EINVAL, "swe_tune: tune the unsharded mesh");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return tfail(SWE_EDEVICE, "swe_tune: no device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return tfail(SWE_EDEVICE, "swe_tune: cannot create events");
    }
    swe_tune_result r;
    memset(&r, 0, sizeof(r));
    int32_t rc = SWE_OK;
    swe_params q[4];
    bool runs[4] = {false, false, false, false};
    // candidates in the order of ms_per_step: cell + remap, cell, tiled + remap, tiled; each
    // warmed up by a run that captures its graph (the mesh keeps one per candidate), then
    // timed in kRounds interleaved rounds (best round kept) so that drift of the state or the
    // clock favours none of them
    constexpr int kRounds = 3;
    for (int c = 0; c < 4 && rc == SWE_OK; ++c) {
        q[c] = *p;
        q[c].variant = c < 2 ? SWE_CELL : SWE_TILED;
        q[c].flags = (p->flags & ~SWE_NO_XCD_REMAP) | ((c & 1) ? SWE_NO_XCD_REMAP : 0);
        swe_run_stats stats;
        const int32_t w = swe_run(mesh, dm, &q[c], s, 2 * kGraphSteps, nullptr, &stats, stream);
        if ((w == SWE_EUNSUPPORTED || w == SWE_EINVAL) && q[c].variant == SWE_TILED)
            continue;   // no tile arrays, or its LDS does not fit
        if (w != SWE_OK) rc = w;
        runs[c] = w == SWE_OK;
    }
    double best_ms[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    for (int round = 0; round < kRounds && rc == SWE_OK; ++round)
        for (int c = 0; c < 4 && rc == SWE_OK; ++c) {
            if (!runs[c]) continue;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = tfail(SWE_EDEVICE, "swe_tune: event"); break; }
            if (int32_t k = swe_run(mesh, dm, &q[c], s, n_steps, nullptr, nullptr, stream)) { rc = k; break; }
            float ms = 0.0f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = tfail(SWE_EDEVICE, "swe_tune: event");
                break;
            }
            best_ms[c] = std::min(best_ms[c], static_cast<double>(ms) / n_steps);
        }
    if (rc == SWE_OK) {
        swe_run_stats stats;
        if (int32_t k = swe_read_stats(s, &stats, stream))
            rc = k;
        else if (stats.done)
            rc = tfail(SWE_EINVAL, "swe_tune: the state stopped (t_end or an error) while tuning");
    }
    double best = INFINITY;
    int pick = -1;
    for (int c = 0; c < 4 && rc == SWE_OK; ++c) {
        if (!runs[c]) continue;
        r.ms_per_step[c] = best_ms[c];
        if (best_ms[c] < best) {
            best = best_ms[c];
            pick = c;
        }
    }
    // The XCD-contiguous order keeps a tile's neighbours in its XCD's L2 and moves far fewer
    // HBM bytes; keep it unless the hardware order is clearly (kTieBreak) faster.
    constexpr double kTieBreak = 1.02;
    if (pick >= 0 && (pick & 1) && runs[pick - 1] && best_ms[pick - 1] <= kTieBreak * best_ms[pick])
        --pick;
    if (pick >= 0) {
        r.variant = q[pick].variant;
        r.xcd_remap = (pick & 1) ? 0 : 1;
    }
    r.tile_cells = mesh->info.tile_cells;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SWE_OK) return rc;
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[Key{dev, p->dtype, size_class(mesh->info.n_cells)}] = r;
    } catch (const std::bad_alloc &) {
        return tfail(SWE_EINVAL, "swe_tune: out of host memory");
    }
    *out = r;
    return SWE_OK;
}

int32_t swe_tune_get(int32_t device, int32_t dtype, int64_t n_cells, swe_tune_result *out)
{
    if (!out || n_cells < 1 || (dtype != SWE_F64 && dtype != SWE_F32))
        return tfail(SWE_EINVAL, "swe_tune_get: bad argument");
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_table.find(Key{device, dtype, size_class(n_cells)});
    if (it == g_table.end()) {
        memset(out, 0, sizeof(*out));   // variant SWE_AUTO: nothing recorded
        return SWE_OK;
    }
    *out = it->second;
    return SWE_OK;
}

int32_t swe_tune_set(int32_t device, int32_t dtype, int64_t n_cells, const swe_tune_result *r)
{
    if (!r || n_cells < 1 || (dtype != SWE_F64 && dtype != SWE_F32))
        return tfail(SWE_EINVAL, "swe_tune_set: bad argument");
    if (r->variant != SWE_AUTO && r->variant != SWE_CELL && r->variant != SWE_TILED)
        return tfail(SWE_EINVAL, "swe_tune_set: unknown variant");
    if (r->xcd_remap != 0 && r->xcd_remap != 1) return tfail(SWE_EINVAL, "swe_tune_set: xcd_remap must be 0 or 1");
    if (r->tile_cells != 0 && !valid_tile(r->tile_cells))
        return tfail(SWE_EINVAL, "swe_tune_set: tile_cells must be 0, 64, 128, 256 or 512");
    std::lock_guard<std::mutex> lk(g_mu);
    const Key k{device, dtype, size_class(n_cells)};
    try {
        if (r->variant == SWE_AUTO)
            g_table.erase(k);
        else
            g_table[k] = *r;
    } catch (const std::bad_alloc &) {
        return tfail(SWE_EINVAL, "swe_tune_set: out of host memory");
    }
    return SWE_OK;
}

}  // extern "C"
