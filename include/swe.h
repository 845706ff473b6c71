/*
 * swe.h -- C ABI of libswe.so, one explicit step of the cell-centred HLLC finite-volume
 * shallow-water solver of Zaoui, "A GPU-enabled finite volume solver for large shallow water
 * simulations" (EDF R&D, 2016), written for AMD MI355X (gfx950).
 *
 * Problem (section 2.1, eq. 1): U = (h, hu, hv) on a triangle mesh (section 2.2) over a bed z
 * with Manning roughness n and gravity g, advanced by explicit Euler steps (eq. 4) whose dt
 * follows the CFL condition with a Courant number (0.7 in the paper).  Fluxes are HLLC with a
 * hydrostatic reconstruction of the bed; friction is semi-implicit (section 2.2).  The host
 * loops over time and the device does the work, with no per-step transfers (section 2.3).
 *
 * Conventions shared by every call:
 *  - Every function returns an int32 status (SWE_OK or a negative code) and never aborts or
 *    throws; swe_last_error() gives a message for the calling thread's last failure.
 *  - Host pointers are read during the call only.  Device pointers are owned by the caller
 *    (the library allocates no device memory in the step path) and must stay valid until the
 *    work queued on the stream has finished.
 *  - Per-cell device arrays are in MESH order: the cell order chosen by swe_mesh_create
 *    (Morton order of the centroids with SWE_MORTON).  SWE_ARR_PERM maps mesh order to input
 *    order.
 *  - `stream` is a hipStream_t (NULL: the null stream).  swe_state_init, swe_step and swe_run
 *    (with out == NULL) only queue work; swe_read_stats and swe_run (with out != NULL)
 *    synchronise the stream.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define SWE_OK 0
#define SWE_EINVAL (-1)        /* null pointer, bad size or parameter */
#define SWE_EMESH (-2)         /* degenerate triangle, edge shared by > 2 cells, bad index */
#define SWE_EDEVICE (-3)       /* a HIP runtime call failed */
#define SWE_ENONFINITE (-4)    /* the state stopped being finite */
#define SWE_EDRY (-5)          /* no wet cell: the CFL time step is undefined */
#define SWE_EUNSUPPORTED (-6)  /* valid request this build cannot serve */

/* ------------------------------------------------------------------ constants */
#define SWE_F64 0              /* state, bed and roughness in double */
#define SWE_F32 1              /* state, bed and roughness in float (coordinates stay double) */
#define SWE_MORTON 1u          /* swe_mesh_create flag: renumber cells along a Morton curve */
#define SWE_HILBERT 2u         /* swe_mesh_create flag: renumber cells along a Hilbert curve */
#define SWE_MAX_INFLOW 16      /* inflow segments per mesh */
#define SWE_CTRL_BYTES 512     /* size of the device control block of a state */
#define SWE_WALL (-1)          /* boundary code of a reflective wall (section 3) */
#define SWE_AUTO 0             /* variant: swe_tune's choice for this device, precision and
                                  size class if one is recorded; else the tiled kernel where
                                  its LDS fits, else the per-cell one */
#define SWE_CELL 1             /* variant: one work-item per cell gathering its neighbours */
#define SWE_TILED 2            /* variant: tile-staged states, each tile interface once */
#define SWE_NO_XCD_REMAP 1u    /* flag: launch tiles in mesh order instead of giving each XCD
                                  a contiguous run of tiles (same results) */
#define SWE_SHARD 2u           /* flag: the state is one shard of a mesh run on several devices;
                                  its steps leave the next dt to swe_shard_dt_combine */
#define SWE_INDEX64 4u         /* flag: 64-bit index arithmetic in the tiled kernel even where
                                  every array spans less than 4 GiB (same results) */
#define SWE_EXACT 8u           /* flag: FP64 division and square root correctly rounded, the
                                  same bits as the host's IEEE operations in the same order;
                                  default: hardware-seeded Newton forms, within an ulp */
#define SWE_TILE 256           /* default cells per tile: consecutive mesh-order cells stepped
                                  by one workgroup, which stages them and their neighbours in
                                  LDS (the workgroup size of the step kernels) */
#define SWE_TILE_64 16u        /* swe_mesh_create flag: tiles of 64 cells */
#define SWE_TILE_128 32u       /* swe_mesh_create flag: tiles of 128 cells */
#define SWE_TILE_512 64u       /* swe_mesh_create flag: tiles of 512 cells (none of the three
                                  flags: SWE_TILE cells); swe_tune times a mesh's own size,
                                  tune.tune_tiles builds one mesh per size and keeps the fastest */

typedef struct swe_mesh swe_mesh;   /* host-side mesh object, owned by the library */

typedef struct swe_mesh_info {
    int64_t n_cells;           /* T: triangles (finite volumes) */
    int64_t n_nodes;           /* V */
    int64_t n_edges;           /* E: interfaces */
    int64_t n_boundary_edges;  /* B = 2E - 3T */
    int64_t n_inflow_edges;
    int32_t n_inflow_segments; /* largest inflow tag used */
    uint32_t flags;            /* flags given to swe_mesh_create */
    double min_area, max_area, total_area, min_inradius;
    double bbox[4];            /* xmin, ymin, xmax, ymax */
    int64_t n_tiles;           /* ceil(T / tile_cells) */
    int64_t n_halo;            /* total halo entries over all tiles */
    int64_t n_tile_edges;      /* total edge-list entries over all tiles */
    int32_t max_halo;          /* largest halo of a tile */
    int32_t max_tile_edges;    /* longest edge list of a tile */
    int64_t n_owned;           /* cells [0, n_owned) are owned: they alone enter the dt
                                  reduction and the counters (T except for shards) */
    int64_t n_tile_nodes;      /* total node-list entries over all tiles; 0: no node lists
                                  (a tile has more than 256 nodes) */
    int32_t max_tile_nodes;    /* most distinct nodes of a tile's cells */
    int32_t tile_cells;        /* cells per tile: 64, 128, 256 or 512 (swe_mesh_create flags) */
} swe_mesh_info;

/* Arrays swe_mesh_export copies out (sizes in elements). */
enum swe_mesh_array {
    SWE_ARR_PERM = 0,      /* int32[T]: input index of mesh cell i */
    SWE_ARR_NBR = 1,       /* int32[3T], structure of arrays: [k*T + i] = neighbour (mesh
                              order) across local edge k of cell i, or a boundary code:
                              SWE_WALL, or -1 - s for inflow segment s >= 1 */
    SWE_ARR_C2N = 2,       /* int32[3T], [k*T + i] = node k of cell i (mesh node order);
                              counter-clockwise, local edge k runs from node k to node k+1 */
    SWE_ARR_XY = 3,        /* double[2V]: (x, y) of mesh node j at [2j], [2j+1] */
    SWE_ARR_NODE_PERM = 4, /* int32[V]: input index of mesh node j */
    SWE_ARR_HALO_OFF = 5,  /* int32[n_tiles+1]: tile t's halo is HALO[off[t] .. off[t+1]) */
    SWE_ARR_HALO = 6,      /* int32[n_halo]: cells outside a tile that neighbour it, ascending */
    SWE_ARR_EDGE_OFF = 7,  /* int32[n_tiles+1]: tile t's edges are EDGES[off[t] .. off[t+1]) */
    SWE_ARR_EDGES = 8,     /* uint32[n_tile_edges]: one per interface a tile evaluates:
                              bits 0-8 owning cell a (tile-local), bits 9-10 a's local edge k,
                              bits 11-12 b's local edge when b is a tile cell (else 0),
                              bits 16-31 int16 b: tile-local cell (< tile_cells), halo slot
                              tile_cells + j, or a boundary code (SWE_WALL, -1 - s) */
    SWE_ARR_SLOT = 9,      /* uint16[3T], [k*T + i]: entry of cell i's local edge k in its
                              tile's edge list; bit 15 set when i is the edge's side b */
    SWE_ARR_GLOBAL = 10,   /* int32[T]: index of cell i in the mesh a shard was cut from
                              (swe_mesh_create_shard); i for other meshes */
    SWE_ARR_EDGE_VEC = 11, /* double[2 n_tile_edges]: (dx, dy) of each EDGES entry, node k+1
                              minus node k of its owning cell (the outward normal of eq. 3
                              is (dy, -dx) / l) */
    SWE_ARR_CELL_GEO = 12, /* double[2T]: area A_i of cell i at [i] (eq. 4), inradius
                              r_i = 2 A_i / P_i at [T + i] (the CFL bound); IEEE square root
                              and division, l_k summed in local-edge order */
    SWE_ARR_EDGE_VEC32 = 13, /* float[2 n_tile_edges]: SWE_ARR_EDGE_VEC rounded to float */
    SWE_ARR_CELL_GEO32 = 14, /* float[2T]: SWE_ARR_CELL_GEO rounded to float */
    /* (ids 16-20 are the batch arrays of enum swe_batch_array) */
    SWE_ARR_TILE_NODE_OFF = 21, /* int32[n_tiles+1]: tile t's nodes are TILE_NODES entries
                                   [off[t] .. off[t+1]); only where every tile has at most 256 */
    SWE_ARR_TILE_NODES = 22,    /* double[2 n_tile_nodes]: (x, y) of each tile's nodes, the
                                   nodes of its cells in first-use order (cell, then local node) */
    SWE_ARR_EDGE_NODES = 23     /* uint16[n_tile_edges]: bits 0-7 and 8-15 the tile-local node
                                   ids of node k and node k+1 of each EDGES entry's owning cell:
                                   their difference is the entry's SWE_ARR_EDGE_VEC, bit for bit */
};

/* Device view of a mesh: the arrays of swe_mesh_export copied to device memory.  nbr, c2n,
 * xy and the cell geometry of the step's precision are required; halo_off, halo, edge_off,
 * edges, slot and the edge vectors of the step's precision are the tiled kernels' (the tiled
 * step reads all but slot, which the tiled adjoint reads): when one is NULL, SWE_AUTO runs the
 * per-cell kernel and SWE_TILED is an error.  tile_node_off, tile_nodes and edge_nodes are
 * optional: with all three the FP64 tiled step, in its shared LDS layout (the one it takes
 * unless the plain one fits as many tiles per CU), forms each edge vector from its tile's node
 * list instead of reading edge_vec (the same bits, fewer bytes). */
typedef struct swe_dev_mesh {
    int64_t n_cells, n_nodes;
    const int32_t *nbr;    /* device, as SWE_ARR_NBR */
    const int32_t *c2n;    /* device, as SWE_ARR_C2N */
    const double *xy;      /* device, as SWE_ARR_XY, 16-byte aligned */
    const int32_t *halo_off;   /* device, as SWE_ARR_HALO_OFF */
    const int32_t *halo;       /* device, as SWE_ARR_HALO */
    const int32_t *edge_off;   /* device, as SWE_ARR_EDGE_OFF */
    const uint32_t *edges;     /* device, as SWE_ARR_EDGES */
    const uint16_t *slot;      /* device, as SWE_ARR_SLOT */
    const double *edge_vec;    /* device, as SWE_ARR_EDGE_VEC, 16-byte aligned (FP64 tiled step) */
    const double *cell_geo;    /* device, as SWE_ARR_CELL_GEO (FP64 steps and the adjoint) */
    const float *edge_vec32;   /* device, as SWE_ARR_EDGE_VEC32, 8-byte aligned (FP32 tiled
                                  step); may be NULL for FP64-only use */
    const float *cell_geo32;   /* device, as SWE_ARR_CELL_GEO32 (FP32 steps); may be NULL for
                                  FP64-only use */
    const int32_t *tile_node_off;  /* device, as SWE_ARR_TILE_NODE_OFF, or NULL */
    const double *tile_nodes;      /* device, as SWE_ARR_TILE_NODES, 16-byte aligned, or NULL */
    const uint16_t *edge_nodes;    /* device, as SWE_ARR_EDGE_NODES, or NULL */
} swe_dev_mesh;

/* Physical and numerical parameters (section 2.1-2.2). */
typedef struct swe_params {
    double g;              /* gravity, > 0 */
    double courant;        /* CFL number, in (0, 1]; the paper uses 0.7 */
    double h_dry;          /* dry threshold (m), >= 0: velocities are zero at or below it */
    int32_t dtype;         /* SWE_F64 or SWE_F32 */
    int32_t n_inflow;      /* number of inflow segments, <= SWE_MAX_INFLOW */
    const double *inflow_q;/* host, n_inflow unit discharges (m^2/s) entering, >= 0 */
    int32_t variant;       /* step kernel: SWE_AUTO, SWE_CELL or SWE_TILED (same results) */
    int32_t flags;         /* SWE_NO_XCD_REMAP | SWE_SHARD | SWE_INDEX64 | SWE_EXACT, or 0 */
} swe_params;

/* Device state of one simulation.  All pointers device, element type given by dtype. */
typedef struct swe_state {
    void *h[2], *hu[2], *hv[2];  /* two buffers of T values each; buffer `cur` holds U^n */
    const void *z;               /* bed elevation, T values */
    const void *n;               /* Manning coefficient, T values, >= 0 */
    void *ctrl;                  /* SWE_CTRL_BYTES, 16-byte aligned: time, dt, counters */
    void *work;                  /* swe_workspace_bytes(T) bytes, 256-byte aligned: step
                                    partials (a single mesh's steps merge them into atomic
                                    slots) and arrival counters, which swe_state_init resets
                                    and every step leaves reset; never shared by two states */
    int32_t cur;                 /* host: buffer holding the current state */
    int32_t reserved;
} swe_state;

/* Counters of a state since swe_state_init. */
typedef struct swe_run_stats {
    int64_t steps;         /* steps taken */
    int64_t clamps;        /* negative depths set to zero */
    double t;              /* current time */
    double dt_next;        /* dt of the next step */
    double dt_min, dt_max, dt_sum;   /* over the steps taken */
    int32_t status;        /* SWE_OK, SWE_ENONFINITE or SWE_EDRY */
    int32_t done;          /* t_end reached or an error stopped the state */
    int32_t cur;           /* buffer holding the current state */
    int32_t reserved;
} swe_run_stats;

/* ------------------------------------------------------------------ mesh (host only) */

/*
 * Build a mesh from a raw triangle list (section 2.2: the domain is divided into triangles;
 * section 2.3: fluxes live on the interfaces).  xy: host double[2*nv] node coordinates;
 * tri: host int32[3*nt] node ids, either orientation (clockwise triangles are reordered
 * (v0, v2, v1)); edge_tag: host int32[3*nt] or NULL (all walls): for a boundary edge k of
 * triangle t (nodes k, k+1 of the input triangle), 0 = wall, s >= 1 = inflow segment s.
 * flags: SWE_MORTON, SWE_HILBERT or 0 (keep the input order); the curves run through the
 * centroids quantised to 16 bits per axis over the bounding box, ties keep the input order;
 * plus at most one of SWE_TILE_64, SWE_TILE_128, SWE_TILE_512 (else tiles of SWE_TILE cells):
 * the workgroup size of the step kernels, with the tile lists built for it.
 * On success *out owns a new mesh.
 * Errors: SWE_EINVAL (null pointer, nv < 3, nt < 1, sizes beyond int32, non-finite
 * coordinates, tag out of range), SWE_EMESH (repeated or out-of-range node, zero-area
 * triangle, edge shared by more than two triangles or twice in the same direction).
 */
int32_t swe_mesh_create(const double *xy, int64_t nv, const int32_t *tri, int64_t nt,
                        const int32_t *edge_tag, uint32_t flags, swe_mesh **out);

/* Counts and geometry summary of a mesh.  Errors: SWE_EINVAL. */
int32_t swe_mesh_info_get(const swe_mesh *mesh, swe_mesh_info *out);

/* Copy array `which` (enum swe_mesh_array) into host memory dst of dst_bytes bytes.
 * Errors: SWE_EINVAL (unknown array, null pointer, dst_bytes too small). */
int32_t swe_mesh_export(const swe_mesh *mesh, int32_t which, void *dst, int64_t dst_bytes);

/* Free a mesh (NULL is ignored). */
void swe_mesh_destroy(swe_mesh *mesh);

/* Bytes of the device workspace a state of n_cells cells needs, whatever its mesh's tile size
 * (it holds one partial result per tile of the smallest size).  Errors: SWE_EINVAL. */
int32_t swe_workspace_bytes(int64_t n_cells, int64_t *bytes);

/* ------------------------------------------------------------------ stepping (device) */

/*
 * Start a state at time t0: computes the first CFL dt from U in buffer state->cur (section
 * 2.2, Courant number params->courant) and clears the counters.  t_end > 0 makes every later
 * step stop at t_end exactly (the step that would pass it is shortened); t_end <= 0: no end.
 * Queues work only.  Errors: SWE_EINVAL (bad parameter, pointer or size), SWE_EDEVICE.  A
 * state without a wet cell is reported later, by swe_read_stats, as SWE_EDRY.
 */
int32_t swe_state_init(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                       swe_state *s, double t0, double t_end, void *stream);

/*
 * One explicit Euler step (eq. 4) of the dt held in the control block: hydrostatic
 * reconstruction and HLLC flux on each cell's three edges, bed correction, update, negative
 * depths clamped, semi-implicit Manning friction, then the CFL dt of the next step reduced
 * over the owned cells (every cell but a shard's halo; under SWE_SHARD the candidate is left
 * for swe_shard_dt_combine).  Reads buffer s->cur, writes the other one and flips s->cur.  Once
 * the state is done (t_end reached, or an error) the step changes nothing and s->cur is kept.
 * Queues work only.  Errors: SWE_EINVAL, SWE_EDEVICE.
 */
int32_t swe_step(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                 swe_state *s, void *stream);

/*
 * n_steps steps (the host time loop of section 2.3) with no host round trip between them:
 * groups of 8 steps are captured once as a hipGraph (cached on the mesh, up to 8 graphs keyed
 * by the launch's arguments, the least recently used replaced) and replayed, starting from
 * buffer 0 (a state in buffer 1 takes one step on its own first); runs shorter than 16 steps
 * launch step by step.  dt_seq:
 * NULL (CFL dt) or a device array of n_steps doubles replayed as the steps' dt (the t_end
 * clip still applies; not with SWE_SHARD).  out: NULL to only queue the work, or a stats
 * record: then the stream is synchronised, *out filled, and s->cur set to the buffer holding
 * the result; the return value is then also the state's status (SWE_ENONFINITE, SWE_EDRY).
 * The graph cache makes calls on one mesh from several threads at once unsafe; use one mesh
 * object per thread.
 * Errors: SWE_EINVAL, SWE_EDEVICE, and with out != NULL the state's status.
 */
int32_t swe_run(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                swe_state *s, int64_t n_steps, const double *dt_seq, swe_run_stats *out,
                void *stream);

/* Synchronise the stream and read the state's counters; sets s->cur.  Returns the state's
 * status (SWE_OK, SWE_ENONFINITE, SWE_EDRY) or SWE_EINVAL / SWE_EDEVICE. */
int32_t swe_read_stats(swe_state *s, swe_run_stats *out, void *stream);

/* Message of the calling thread's last failure ("" if none).  Valid until the next call. */
const char *swe_last_error(void);

/* ------------------------------------------------------------------ batches */

/*
 * A batch steps many independent meshes (scenarios: an ensemble of inflows and roughness) in
 * one launch per step, each scenario with its own CFL dt and time.  Its arrays are the
 * scenarios' mesh arrays concatenated (cells and nodes offset per scenario); its tiles never
 * straddle two scenarios.
 */
typedef struct swe_batch swe_batch;

typedef struct swe_batch_info {
    int32_t n_scenarios;
    int32_t max_inflow_segments;   /* largest inflow tag over the scenarios */
    int64_t n_cells, n_nodes, n_tiles, n_halo, n_tile_edges;
    int32_t max_halo, max_tile_edges;
    int64_t n_tile_nodes;          /* 0: a scenario has no node lists */
    int32_t max_tile_nodes, tile_cells;   /* the scenarios' common tile size */
} swe_batch_info;

/* Arrays of a batch besides the concatenated SWE_ARR_* ones (which swe_batch_export also
 * gives: NBR, C2N, XY, HALO_OFF, HALO, EDGE_OFF, EDGES, SLOT, EDGE_VEC, CELL_GEO, EDGE_VEC32,
 * CELL_GEO32, TILE_NODE_OFF, TILE_NODES, EDGE_NODES, and PERM = each scenario's own
 * SWE_ARR_PERM, concatenated). */
enum swe_batch_array {
    SWE_BARR_CELL_OFF = 16,      /* int64[n+1]: scenario s owns cells [off[s], off[s+1]) */
    SWE_BARR_NODE_OFF = 17,      /* int64[n+1]: and nodes [off[s], off[s+1]) */
    SWE_BARR_TILE_START = 18,    /* int32[n_tiles+1]: tile t holds cells [start[t], start[t+1]) */
    SWE_BARR_TILE_SCEN = 19,     /* int32[n_tiles]: scenario of tile t */
    SWE_BARR_SCEN_TILE_OFF = 20  /* int32[n+1]: scenario s owns tiles [off[s], off[s+1]) */
};

typedef struct swe_batch_dev {
    swe_dev_mesh mesh;             /* device copies of the concatenated SWE_ARR_* arrays */
    const int32_t *tile_start;     /* device, SWE_BARR_TILE_START */
    const int32_t *tile_scen;      /* device, SWE_BARR_TILE_SCEN */
    const int32_t *scen_tile_off;  /* device, SWE_BARR_SCEN_TILE_OFF */
} swe_batch_dev;

typedef struct swe_batch_params {
    double g, courant, h_dry;      /* shared by all scenarios, as in swe_params */
    int32_t dtype;                 /* SWE_F64 or SWE_F32 */
    int32_t variant;               /* SWE_AUTO, SWE_CELL or SWE_TILED */
    const double *inflow_q;        /* device, n_scenarios * SWE_MAX_INFLOW unit discharges
                                      (m^2/s): scenario s's segment k at [s*16 + k-1] */
    int32_t flags;                 /* SWE_NO_XCD_REMAP | SWE_EXACT, or 0 */
    int32_t reserved;
} swe_batch_params;

/* Concatenate n built meshes (each keeps its own cell and node order), all of one tile size.
 * The meshes may be destroyed afterwards.  Errors: SWE_EINVAL. */
int32_t swe_batch_create(const swe_mesh *const *meshes, int32_t n, swe_batch **out);
int32_t swe_batch_info_get(const swe_batch *batch, swe_batch_info *out);
/* Copy a SWE_ARR_* or SWE_BARR_* array of the batch to host memory.  Errors: SWE_EINVAL. */
int32_t swe_batch_export(const swe_batch *batch, int32_t which, void *dst, int64_t dst_bytes);
void swe_batch_destroy(swe_batch *batch);
/* Workspace bytes of a batch state (its per-tile partials).  Errors: SWE_EINVAL. */
int32_t swe_batch_workspace_bytes(const swe_batch *batch, int64_t *bytes);

/*
 * Start every scenario of a batch state at t0 (t_end as in swe_state_init).  The state's
 * buffers hold the concatenated cells; ctrl holds n_scenarios control blocks of
 * SWE_CTRL_BYTES each.  Queues work only.  Errors: SWE_EINVAL, SWE_EDEVICE.
 */
int32_t swe_batch_state_init(const swe_batch *batch, const swe_batch_dev *dev,
                             const swe_batch_params *p, swe_state *s, double t0, double t_end,
                             void *stream);

/*
 * n_steps steps of every scenario, one launch of the step kernel and one of the per-scenario dt
 * pass per step, replayed from a captured graph.  Each scenario takes its own CFL dt and stops
 * on its own at t_end or on an error.  out: NULL (queue only) or n_scenarios records; then the
 * stream is synchronised and out[s].cur tells in which buffer scenario s's cells are.  Returns
 * SWE_OK, or with out != NULL the first failing scenario's status.  Errors: SWE_EINVAL,
 * SWE_EUNSUPPORTED (tile LDS does not fit the device), SWE_EDEVICE.
 */
int32_t swe_batch_run(const swe_batch *batch, const swe_batch_dev *dev,
                      const swe_batch_params *p, swe_state *s, int64_t n_steps,
                      swe_run_stats *out, void *stream);

/* ------------------------------------------------------------------ adjoint */

/* Gauge misfit J = sum over observations m = 1 .. n_steps/every and gauges g of
 * (h_g after step m*every - obs[(m-1)*n_gauges + g])^2. */
typedef struct swe_loss {
    const int32_t *gauges;   /* device, n_gauges distinct mesh-order cells */
    int32_t n_gauges;
    int32_t every;           /* steps between observations, >= 1 */
    const double *obs;       /* device, (n_steps/every) * n_gauges observed depths */
} swe_loss;

/* Gradients of J, device arrays of n_cells doubles each, mesh order (written). */
typedef struct swe_grads {
    double *dn;              /* dJ/d(Manning n) */
    double *dz;              /* dJ/d(bed z) */
    double *dh, *dhu, *dhv;  /* dJ/d(initial state) */
} swe_grads;

/* Workspace bytes of swe_adjoint: checkpoints, a recompute segment, the adjoint state and
 * the loss with each observation's share (n_steps + 1 doubles); with ckpt_every = 1, every
 * state and every step's U* instead (6 T doubles per step) and no segment.
 * Errors: SWE_EINVAL. */
int32_t swe_adjoint_workspace_bytes(const swe_mesh *mesh, int64_t n_steps, int32_t ckpt_every,
                                    int64_t *bytes);

/*
 * Loss and gradient of a replayed run: n_steps FP64 steps from the state in buffer s->cur of
 * s (with s->z and s->n) using dt_seq (device, n_steps doubles, not differentiated), the
 * misfit J of `loss`, and the hand-written reverse sweep of the step (friction and clamp,
 * then the transposed interface fluxes with hydrostatic reconstruction, every branch frozen
 * to the forward run).  Forward states are checkpointed every ckpt_every steps and recomputed
 * segment by segment in the reverse pass, except the last segment, whose states the forward
 * pass keeps; ckpt_every = 1 stores every state and U* in the forward pass and recomputes
 * nothing (the same gradients, bit for bit).  The caller's state
 * is not modified.  ws: device, swe_adjoint_workspace_bytes bytes, 256-byte aligned.
 * *loss_out (host, may be NULL) receives J; then the stream is synchronised.
 * Errors: SWE_EINVAL, SWE_EUNSUPPORTED (FP32), SWE_EDEVICE.
 */
int32_t swe_adjoint(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                    const swe_state *s, int64_t n_steps, const double *dt_seq,
                    const swe_loss *loss, int32_t ckpt_every, swe_grads *out, double *loss_out,
                    void *ws, int64_t ws_bytes, void *stream);

/* Device time of this thread's last completed swe_adjoint call, in milliseconds, from HIP
 * events on its stream: the forward pass (checkpoints or every state) and the reverse sweep
 * (segment recompute, unless every state was stored, adjoint steps and the loss).
 * Waits for that call's work to finish.
 * Errors: SWE_EINVAL (no completed call on this thread), SWE_EDEVICE. */
int32_t swe_adjoint_timings(double *forward_ms, double *reverse_ms);

/* ------------------------------------------------------------------ shards */

/*
 * A shard of a mesh, for running one mesh on several devices (section 2.3's two loops
 * restricted to a range of cells; section 5 names multi-GPU runs as the continuation): cells
 * [c0, c1) of `full` in its mesh order (Morton ranges keep the halo small), followed by their
 * halo — every cell outside the range that shares an edge with it, ascending — as a mesh of
 * its own in that order (no renumbering).  info.n_owned = c1 - c0.  A step updates every cell
 * of the shard but only owned cells enter the dt reduction and the counters; halo edges to
 * cells outside the shard act as walls, so the halo's own update is meaningless and the halo
 * must be refreshed from its owners (swe_halo_pack, then swe_halo_unpack) before each step.
 * Inflow tags are kept.  SWE_ARR_GLOBAL maps shard cells to `full` cells.  On success *out
 * owns a new mesh.  Errors: SWE_EINVAL (null argument, bad range).
 */
int32_t swe_mesh_create_shard(const swe_mesh *full, int64_t c0, int64_t c1, swe_mesh **out);

/* Gather rows idx[0..n) (device int32) of the device arrays h, hu, hv (dtype) into the device
 * buffer buf: n values of h, then n of hu, then n of hv.  Queues work only.
 * Errors: SWE_EINVAL. */
int32_t swe_halo_pack(int32_t dtype, int64_t n, const int32_t *idx, const void *h,
                      const void *hu, const void *hv, void *buf, void *stream);

/* Scatter a buffer laid out as swe_halo_pack writes it into rows idx[0..n) of h, hu, hv.
 * Queues work only.  Errors: SWE_EINVAL. */
int32_t swe_halo_unpack(int32_t dtype, int64_t n, const int32_t *idx, const void *buf,
                        void *h, void *hu, void *hv, void *stream);

/*
 * The dt all-reduce of a sharded run: states initialised or stepped with SWE_SHARD hold their
 * own CFL candidate (C min r/(|u|+c) over owned cells); this sets every shard's next dt to the
 * minimum over the shards, cut at t_end (then marking the last step), or stops them all (a
 * shard that stopped on an error stops every shard; no wet cell anywhere is SWE_EDRY).
 * ctrls: host array of n <= 64 device pointers to the shards' control blocks, all on the
 * current device (a multi-device run reduces the one candidate over the interconnect
 * instead).  Queues work only.  Errors: SWE_EINVAL.
 */
int32_t swe_shard_dt_combine(void *const *ctrls, int32_t n, void *stream);

/* ------------------------------------------------------------------ launch tuning */

/* Timings of the step variants on one mesh (milliseconds per step, 0: not run), and the
 * fastest.  Order of ms_per_step: per-cell + XCD remap, per-cell, tiled + XCD remap, tiled. */
typedef struct swe_tune_result {
    int32_t variant;         /* SWE_CELL or SWE_TILED; SWE_AUTO: nothing recorded */
    int32_t xcd_remap;       /* 1: XCD-contiguous tile order, 0: hardware order */
    double ms_per_step[4];
    int32_t tile_cells;      /* tile size of the mesh timed (64, 128, 256 or 512); 0: unknown */
    int32_t reserved;
} swe_tune_result;

/*
 * Autotuning of the step launch (section 2.3's loops as GPU launches; the paper leaves the
 * mapping to the hardware open).  Times each variant x workgroup order for n_steps >= 2 steps
 * (graph replay, after a warm-up of 16 steps each that captures its graph) in three
 * interleaved rounds, keeping each one's best, on the initialised state s, which it advances by
 * 64 + 12 n_steps steps at most (pass a scratch state, or re-initialise afterwards).  The tile
 * size is the mesh's (a mesh is built for one); comparing tile sizes takes one mesh per size,
 * each tuned, and swe_tune_set of the fastest (tune.tune_tiles does that).  Records the fastest
 * for this device, the params' dtype and the size class floor(log2 n_cells) in a process-wide
 * table, with the mesh's tile size, keeping the
 * XCD-contiguous order unless the hardware order is more than 2 % faster (it moves fewer HBM
 * bytes at equal time).  SWE_AUTO then launches that choice (SWE_NO_XCD_REMAP still forces
 * the hardware order).  All candidates compute the same bits.  Synchronises the stream.
 * *out (host) receives the timings.  Errors: SWE_EINVAL (bad argument, a shard, or the state
 * stopped while tuning), SWE_EDEVICE, and any status of swe_run.
 */
int32_t swe_tune(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                 swe_state *s, int32_t n_steps, swe_tune_result *out, void *stream);

/* The recorded choice for (device, dtype, size class of n_cells); variant SWE_AUTO if none.
 * Errors: SWE_EINVAL. */
int32_t swe_tune_get(int32_t device, int32_t dtype, int64_t n_cells, swe_tune_result *out);

/* Record a choice (e.g. one saved from an earlier process); variant SWE_AUTO erases it.
 * Errors: SWE_EINVAL (unknown variant, xcd_remap not 0 or 1, tile_cells not 0, 64, 128, 256
 * or 512). */
int32_t swe_tune_set(int32_t device, int32_t dtype, int64_t n_cells, const swe_tune_result *r);

/* ------------------------------------------------------------------ without allocation */

/* Bytes of the device array that swe_run_static keeps per GPU in place of a workspace: enough
 * for the step partials of about 262,000 tiles (67 million cells in tiles of 256, 16.7 million
 * in tiles of 64). */
#define SWE_STATIC_WORK_BYTES 4194304

/*
 * For callers that cannot allocate device memory (code under stream capture into a graph,
 * serving loops that forbid allocation): swe_state_init (when init != 0, at t0 with t_end)
 * followed by swe_run, in one call that uses no workspace.  s->work is ignored and may be NULL;
 * the step partials and arrival counters live in a library-owned device array of
 * SWE_STATIC_WORK_BYTES, one per GPU, looked up on the first call on each device and kept until
 * the process ends.  The call allocates nothing: no hipMalloc, no graph instantiation (steps are
 * launched one by one), no host-side device allocation by any library routine.  The caller still
 * provides the state's buffers and control block.  Every call on one GPU shares its array, which
 * keeps the last call's contents: the call clears what must start at zero, and calls whose work
 * overlaps on one GPU (several streams or threads at once) race and give undefined results.
 * The results are those of swe_state_init + swe_run with a workspace, bit for bit.  With
 * out != NULL the stream is synchronised and the state's status returned, as by swe_run.
 * Errors: SWE_EINVAL (as swe_state_init and swe_run, or a mesh whose partials, for its tile
 * count, exceed SWE_STATIC_WORK_BYTES), SWE_EDEVICE.
 */
int32_t swe_run_static(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                       swe_state *s, int32_t init, double t0, double t_end, int64_t n_steps,
                       const double *dt_seq, swe_run_stats *out, void *stream);

/* ------------------------------------------------------------------ test hook */

/*
 * Evaluate the device interface flux on n independent edges, exactly as the step does for a
 * cell facing a neighbour (section 2.2: hydrostatic reconstruction, then HLLC).  Device
 * arrays of n elements of the dtype: left and right states (h, hu, hv, z) and a unit normal
 * (nx, ny) pointing from left to right; outputs f (3n: mass, x- and y-momentum flux per unit
 * length, at [3i..3i+2]) and the left bed correction p (n).  right_h == NULL evaluates a
 * reflective wall instead of a neighbour.  flags: SWE_EXACT or 0, as for the step.  Queues work
 * only.  Errors: SWE_EINVAL, SWE_EDEVICE.
 */
int32_t swe_flux_eval(int32_t dtype, int32_t flags, int64_t n, double g, double h_dry, const void *hl,
                      const void *hul, const void *hvl, const void *zl, const void *hr,
                      const void *hur, const void *hvr, const void *zr, const void *nx,
                      const void *ny, void *f, void *p, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SWE_H */
