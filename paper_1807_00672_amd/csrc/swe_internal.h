// Internal declarations shared by the mesh builder, the C ABI and the HIP kernels of libswe.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "swe.h"

namespace swe {

// Device control block of a state (SWE_CTRL_BYTES bytes, written by the kernels only).
struct Ctrl {
    double t;          // time of the current state
    double dt;         // dt of the next step
    double t_end;      // stop time, <= 0: none
    double dt_min, dt_max, dt_sum;
    int64_t steps;     // steps taken since swe_state_init
    int64_t run_step;  // steps taken by the current swe_run (index into dt_seq)
    int64_t clamps;    // negative depths clamped to zero
    int32_t status;    // kStatus* bits
    int32_t done;      // 1: steps change nothing (t_end reached or error)
    int32_t last;      // 1: the next step ends at t_end exactly
    int32_t cur0;      // buffer holding the state at swe_state_init
    double dt_cfl;     // SWE_SHARD: this shard's CFL candidate for the next dt
};
static_assert(sizeof(Ctrl) <= SWE_CTRL_BYTES, "control block too large");

enum : int32_t { kStatusNonFinite = 1, kStatusDry = 2, kStatusBadDt = 4 };

// Cells per tile (the workgroup size of the step kernels): a mesh's own choice among these.
constexpr int kTileMin = 64, kTileMax = 512;
inline bool valid_tile(int64_t tile)
{
    return tile == 64 || tile == 128 || tile == 256 || tile == 512;
}

// Packed edge-list entry (SWE_ARR_EDGES): bits 0-8 side a (tile-local), bits 9-10 a's local
// edge, bits 11-12 b's local edge (b a tile cell), bits 16-31 side b as an int16.
constexpr uint32_t kEdgeA = 0x1ffu;
constexpr int kEdgeKa = 9, kEdgeKb = 11;

constexpr int kGroup = 256;          // tiles whose partials one workgroup folds together

// Per-block partial results of a step and their second level, laid out in the workspace.  A
// single-mesh step folds them itself: the last workgroup of each group of kGroup tiles to
// finish reduces the group, the last group to finish reduces the groups and advances the
// control block; count[] holds the arrivals and is zero between steps.
struct Partials {
    double *dt;         // [nb] min over the block's cells of r / (|u| + c)
    int32_t *clamps;    // [nb]
    int32_t *flags;     // [nb] kStatus* bits
    double *gdt;        // [n_groups(nb)] the same per group of kGroup tiles
    int32_t *gclamps;   // [n_groups(nb)]
    int32_t *gflags;    // [n_groups(nb)]
    uint32_t *count;    // [n_groups(nb) + 1] arrivals per group, then of the groups
};

// A single mesh's step merges the partials of every kSlotTiles consecutive tiles into one slot
// of the per-tile arrays (slot q at index q, q < n_slots(nb)) with device-scope atomics; the bit
// pattern of +inf is the reset value of a slot's bound, which the workgroups lower by an
// unsigned min of their bounds' bits.
constexpr int kSlotTiles = 16;
constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;
constexpr int64_t n_slots(int64_t nb) { return (nb + kSlotTiles - 1) / kSlotTiles; }

inline int64_t n_tiles_of(int64_t n_cells, int64_t tile) { return (n_cells + tile - 1) / tile; }
inline int64_t n_groups(int64_t nb) { return (nb + kGroup - 1) / kGroup; }
inline int64_t round256(int64_t b) { return ((b + 255) / 256) * 256; }

// Partials of nb tiles laid out in a workspace (every array 256-byte aligned).
inline Partials partials_for(void *work, int64_t nb)
{
    char *p = static_cast<char *>(work);
    const int64_t ng = n_groups(nb);
    Partials r;
    r.dt = reinterpret_cast<double *>(p);
    p += round256(nb * 8);
    r.clamps = reinterpret_cast<int32_t *>(p);
    p += round256(nb * 4);
    r.flags = reinterpret_cast<int32_t *>(p);
    p += round256(nb * 4);
    r.gdt = reinterpret_cast<double *>(p);
    p += round256(ng * 8);
    r.gclamps = reinterpret_cast<int32_t *>(p);
    p += round256(ng * 4);
    r.gflags = reinterpret_cast<int32_t *>(p);
    p += round256(ng * 4);
    r.count = reinterpret_cast<uint32_t *>(p);
    return r;
}

inline int64_t workspace_bytes_for_tiles(int64_t nb)
{
    const int64_t ng = n_groups(nb);
    return round256(nb * 8) + 2 * round256(nb * 4) + round256(ng * 8) + 2 * round256(ng * 4) +
           round256((ng + 1) * 4);
}

// A state's workspace: room for the partials of the smallest tiles, so any mesh of n_cells fits.
inline int64_t workspace_bytes(int64_t n_cells)
{
    return workspace_bytes_for_tiles(n_tiles_of(n_cells, kTileMin));
}

// Everything a launch needs besides the state: plain values, passed by value to kernels.
struct StepConfig {
    int64_t n_cells;
    int64_t n_owned;   // cells [0, n_owned) enter the dt reduction and the counters
    double g, courant, h_dry;
    int32_t n_inflow;
    int32_t shard;     // 1: leave the next dt to swe_shard_dt_combine (SWE_SHARD)
    int32_t index64;   // 1: 64-bit index arithmetic in the tiled kernel (SWE_INDEX64)
    int32_t fast;      // 1: FP64 division and square root by Newton forms (not SWE_EXACT)
    int32_t tile;      // cells per tile (the workgroup size of the step kernels)
    int32_t pad;
    double inflow_q[SWE_MAX_INFLOW];
};

// Tile sizes of a mesh that the tiled step needs at launch.
// Static LDS the tiled step kernels may use besides their dynamic LDS (the slot table and the
// block reduction); the device's per-workgroup limit less this is what dynamic LDS may take.
constexpr size_t kTileStaticLdsMax = 4096;

struct TileLayout {
    int64_t n_tiles;
    int32_t max_halo, max_edges;
    int32_t max_nodes;   // largest node list of a tile; 0: the mesh has no node lists
    int32_t tile;        // cells per tile
};

// Device arrays of a batch of meshes stepped together (swe_batch_*).
struct BatchLaunch {
    const int32_t *tile_start;      // [n_tiles + 1] first cell of each tile
    const int32_t *tile_scen;       // [n_tiles] scenario of each tile
    const int32_t *scen_tile_off;   // [n_scen + 1] tiles of each scenario
    const double *q_table;          // [n_scen * SWE_MAX_INFLOW] inflow discharges
    int32_t n_scen;
    int64_t n_tiles;
};

constexpr int kMaxShards = 64;

// Steps per captured graph of swe_run and swe_batch_run (even: the state returns to its buffer).
#ifndef SWE_GRAPH_STEPS
#define SWE_GRAPH_STEPS 8
#endif
constexpr int kGraphSteps = SWE_GRAPH_STEPS;
static_assert(kGraphSteps >= 2 && kGraphSteps % 2 == 0, "graph step count must be even");

// Launchers.  swe_kernels.hip defines them twice, in swe::exact (correctly rounded FP64
// division and square root) and swe::fast (their hardware-seeded Newton forms, within an ulp);
// the ones in swe itself (swe_launch.cpp) pick by StepConfig::fast.  batch == nullptr: a single
// mesh.  All queue work on `stream` and return a hipError_t as int.
#define SWE_LAUNCHERS                                                                          \
    int launch_init(int dtype, const swe_dev_mesh &dm, const StepConfig &cfg,                  \
                    const swe_state &s, double t0, double t_end, void *stream,                 \
                    const BatchLaunch *batch = nullptr);                                       \
    /* tl == nullptr: the per-cell kernel; else the tiled kernel (its LDS must fit) */         \
    int launch_step(int dtype, const swe_dev_mesh &dm, const StepConfig &cfg,                  \
                    const swe_state &s, int cur, const double *dt_seq, int64_t n_seq,          \
                    void *stream, const TileLayout *tl, const BatchLaunch *batch = nullptr,    \
                    int remap = 1,                                                             \
                    double *const *ustar = nullptr,  /* FP64: also write U* before clamp */    \
                    const double *dt_direct = nullptr); /* replay: dt here, no reduction */    \
    size_t tile_lds_bytes_for(int dtype, const TileLayout &tl);                                \
    int prepare_tile_kernels(size_t max_lds); /* allow dynamic LDS up to max_lds bytes */      \
    int launch_run_begin(const swe_state &s, const double *dt_seq, void *stream);              \
    int launch_halo(int dtype, bool pack, int64_t n, const int32_t *idx, const void *buf_in,   \
                    void *buf_out, const void *h, const void *hu, const void *hv, void *ho,    \
                    void *huo, void *hvo, void *stream);                                       \
    int launch_shard_combine(void *const *ctrls, int n, void *stream);                         \
    int launch_flux_eval(int dtype, int64_t n, double g, double h_dry, const void *hl,         \
                         const void *hul, const void *hvl, const void *zl, const void *hr,     \
                         const void *hur, const void *hvr, const void *zr, const void *nx,     \
                         const void *ny, void *f, void *p, void *stream);
namespace exact {
SWE_LAUNCHERS
}
namespace fast {
SWE_LAUNCHERS
}
SWE_LAUNCHERS
// the flux test hook in either mode
int launch_flux_eval(int dtype, bool fast_math, int64_t n, double g, double h_dry,
                     const void *hl, const void *hul, const void *hvl, const void *zl,
                     const void *hr, const void *hur, const void *hvr, const void *zr,
                     const void *nx, const void *ny, void *f, void *p, void *stream);

void set_error(const std::string &msg);

// swe_run without the stats read: queue n_steps steps, replaying captured graphs where
// `graphs` allows it (swe_api.cpp).
int32_t run_steps(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                  swe_state *s, int64_t n_steps, const double *dt_seq, bool graphs, void *stream);

// The step kernel a launch uses (swe_api.cpp): *tl = the mesh's tile layout for the tiled
// kernel, nullptr for the per-cell one; *remap = 1 for the XCD-contiguous workgroup order.
int32_t choose_variant(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                       const TileLayout **tl, int *remap, const char *where);

// swe_tune's result for (device, dtype, size class of n_cells), if one was recorded: the
// variant (SWE_CELL or SWE_TILED) and XCD order (1 remapped) that ran fastest (swe_tune.cpp).
bool tuned_choice(int device, int dtype, int64_t n_cells, int *variant, int *remap);

}  // namespace swe

// The host-side mesh object behind the opaque swe_mesh handle.
namespace swe {
// Copy `v` rounded to float (round to nearest) into a host buffer of dst_bytes bytes.
inline int32_t export_as_float(const std::vector<double> &v, void *dst, int64_t dst_bytes,
                               const char *where)
{
    if (dst_bytes < static_cast<int64_t>(4 * v.size())) {
        set_error(std::string(where) + ": destination too small");
        return SWE_EINVAL;
    }
    float *d = static_cast<float *>(dst);
    for (size_t k = 0; k < v.size(); ++k) d[k] = static_cast<float>(v[k]);
    return SWE_OK;
}
}  // namespace swe

struct swe_mesh {
    swe_mesh_info info;
    std::vector<int32_t> perm;       // mesh cell -> input cell
    std::vector<int32_t> nbr;        // [3][T]
    std::vector<int32_t> c2n;        // [3][T]
    std::vector<double> xy;          // [V][2]
    std::vector<int32_t> node_perm;  // mesh node -> input node
    std::vector<int32_t> halo_off;   // [n_tiles + 1]
    std::vector<int32_t> halo;       // cells neighbouring a tile from outside, per tile
    std::vector<int32_t> edge_off;   // [n_tiles + 1]
    std::vector<uint32_t> edges;     // packed edge-list entries, per tile
    std::vector<uint16_t> slot;      // [3][T]
    std::vector<double> edge_vec;    // [n_tile_edges][2]: edge vector of each edge-list entry
    std::vector<int32_t> tile_node_off;   // [n_tiles + 1]; empty: no node lists
    std::vector<double> tile_nodes;  // [n_tile_nodes][2]: coordinates of each tile's nodes
    std::vector<uint16_t> edge_nodes;     // [n_tile_edges]: tile-local ids of an entry's nodes
    std::vector<double> cell_geo;    // [2][T]: area, inradius
    std::vector<int32_t> global;     // shards: cell index in the mesh cut from; else empty
    swe::TileLayout tiles;           // sizes the tiled step needs at launch
    void *graph = nullptr;           // cached two-step graph of swe_run (swe_api.cpp)
    ~swe_mesh();
};
