/*
 * swe_oracle.c -- plain, slow FP64 CPU oracle of the explicit cell-centred finite-volume
 * shallow-water scheme of Zaoui, "A GPU-enabled finite volume solver for large shallow water
 * simulations" (EDF R&D, 2016), section 2.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load this file.  It shares no code with the HIP path: it builds its own connectivity and
 * geometry, loops over interfaces for the fluxes (section 2.3: one loop over interfaces, then
 * one over cells) and then over cells for the update.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no -march flags: every product and
 * sum is rounded on its own, in the order the expressions below are written).
 *
 * Readings of points the paper leaves open (each is listed with its justification in the
 * design notes of the repository):
 *   - HLLC wave speeds: two-rarefaction estimates with the dry-bed speeds of Fraccarollo and
 *     Toro (1995); mass and normal momentum are HLL, the tangential momentum is the mass flux
 *     times the upwind tangential velocity chosen by the sign of the contact speed S*.
 *   - Hydrostatic reconstruction: first-order scheme of Audusse et al. (2004).
 *   - Semi-implicit friction: linearly implicit in (hu, hv) after the flux update.
 *   - CFL: dt = C min over wet cells of r_i / (|u_i| + sqrt(g h_i)), r_i the inradius.
 *   - Walls: mirror ghost state.  Inflow segments: prescribed discharge per unit length.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OM_OK 0
#define OM_EINVAL (-1)
#define OM_EMESH (-2)
#define OM_ENONFINITE (-4)
#define OM_EDRY (-5)

/* Boundary codes stored in place of a neighbour: -1 wall, -1-k inflow segment k (k >= 1). */
#define OM_WALL (-1)

typedef struct {
    double g, courant, h_dry;
    int n_inflow;
    const double *inflow_q; /* unit discharge (m^2/s) of inflow segment k at index k-1 */
} om_params;

typedef struct {
    double t;            /* current time, in and out */
    long steps;          /* steps taken by the call */
    long clamps;         /* negative depths set to zero */
    double clamped_mass; /* volume added by those clamps */
    double dt_min, dt_max, dt_sum;
    int last_reached;    /* t_end reached */
} om_stats;

typedef struct {
    long nt, nv, ne, nb;
    int *cell_node;      /* [nt*3], counter-clockwise */
    int *cell_edge;      /* [nt*3], edge of local edge k (from node k to node k+1) */
    int *cell_nbr;       /* [nt*3], neighbour across local edge k, or boundary code */
    int *edge_l;         /* [ne] cell whose local edge defines the edge's normal */
    int *edge_kl;        /* [ne] that local index */
    int *edge_r;         /* [ne] the other cell, or boundary code */
    double *edge_nx, *edge_ny, *edge_len; /* unit normal pointing out of edge_l, length */
    double *area, *inradius;
    const double *xy;    /* borrowed node coordinates [nv*2] */
} om_mesh;

/* ------------------------------------------------------------------------------- mesh */

typedef struct { uint64_t key; long half; } om_half;

static int om_half_cmp(const void *a, const void *b)
{
    const om_half *x = (const om_half *)a, *y = (const om_half *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->half < y->half ? -1 : (x->half > y->half);
}

void om_mesh_free(om_mesh *m)
{
    if (!m) return;
    free(m->cell_node); free(m->cell_edge); free(m->cell_nbr);
    free(m->edge_l); free(m->edge_kl); free(m->edge_r);
    free(m->edge_nx); free(m->edge_ny); free(m->edge_len);
    free(m->area); free(m->inradius);
    free(m);
}

/* Geometry of local edge k of cell c (section 2.2, eq. 3 and Fig. 1): the edge runs from node
 * k to node k+1 of the counter-clockwise triangle; its outward unit normal is (dy, -dx)/l. */
static void om_edge_geom(const om_mesh *m, long c, int k, double *nx, double *ny, double *len)
{
    const int a = m->cell_node[3 * c + k], b = m->cell_node[3 * c + (k + 1) % 3];
    const double dx = m->xy[2 * b] - m->xy[2 * a];
    const double dy = m->xy[2 * b + 1] - m->xy[2 * a + 1];
    const double l = sqrt(dx * dx + dy * dy);
    *nx = dy / l;
    *ny = -dx / l;
    *len = l;
}

/*
 * Build cells, edges and geometry from a raw triangle list (section 2.2: the domain is divided
 * into triangles; section 2.3: fluxes are computed per interface).  Triangles given clockwise
 * are reordered (v0, v2, v1).  tags[3*c+k] (may be NULL) marks boundary edge k of input
 * triangle c: 0 wall, k >= 1 inflow segment k.
 */
int om_mesh_build(const double *xy, long nv, const int *tri, long nt, const int *tags,
                  om_mesh **out)
{
    *out = NULL;
    if (nv < 3 || nt < 1 || !xy || !tri) return OM_EINVAL;
    om_mesh *m = (om_mesh *)calloc(1, sizeof(om_mesh));
    m->nt = nt; m->nv = nv; m->xy = xy;
    m->cell_node = (int *)malloc(sizeof(int) * 3 * nt);
    m->cell_edge = (int *)malloc(sizeof(int) * 3 * nt);
    m->cell_nbr = (int *)malloc(sizeof(int) * 3 * nt);
    m->area = (double *)malloc(sizeof(double) * nt);
    m->inradius = (double *)malloc(sizeof(double) * nt);
    int *ctag = (int *)calloc(3 * nt, sizeof(int));

    for (long c = 0; c < nt; ++c) {
        int v0 = tri[3 * c], v1 = tri[3 * c + 1], v2 = tri[3 * c + 2];
        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nv || v1 >= nv || v2 >= nv ||
            v0 == v1 || v1 == v2 || v0 == v2) {
            free(ctag); om_mesh_free(m); return OM_EMESH;
        }
        const double e0x = xy[2 * v1] - xy[2 * v0], e0y = xy[2 * v1 + 1] - xy[2 * v0 + 1];
        const double e1x = xy[2 * v2] - xy[2 * v1], e1y = xy[2 * v2 + 1] - xy[2 * v1 + 1];
        const double cr = e0x * e1y - e0y * e1x;
        if (!(cr != 0.0) || !isfinite(cr)) { free(ctag); om_mesh_free(m); return OM_EMESH; }
        int t0 = tags ? tags[3 * c] : 0, t1 = tags ? tags[3 * c + 1] : 0,
            t2 = tags ? tags[3 * c + 2] : 0;
        if (cr < 0.0) { /* clockwise: (v0, v2, v1); edges become (e2 reversed, e1, e0) */
            int s = v1; v1 = v2; v2 = s;
            int u = t0; t0 = t2; t2 = u;
        }
        m->cell_node[3 * c] = v0; m->cell_node[3 * c + 1] = v1; m->cell_node[3 * c + 2] = v2;
        ctag[3 * c] = t0; ctag[3 * c + 1] = t1; ctag[3 * c + 2] = t2;
    }

    /* Match half-edges by their unordered node pair. */
    om_half *hs = (om_half *)malloc(sizeof(om_half) * 3 * nt);
    for (long c = 0; c < nt; ++c)
        for (int k = 0; k < 3; ++k) {
            uint64_t a = (uint64_t)m->cell_node[3 * c + k];
            uint64_t b = (uint64_t)m->cell_node[3 * c + (k + 1) % 3];
            uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
            hs[3 * c + k].key = (lo << 32) | hi;
            hs[3 * c + k].half = 3 * c + k;
        }
    qsort(hs, 3 * nt, sizeof(om_half), om_half_cmp);

    long ne = 0, nb = 0;
    for (long i = 0; i < 3 * nt;) {
        long j = i + 1;
        while (j < 3 * nt && hs[j].key == hs[i].key) ++j;
        if (j - i > 2) { free(hs); free(ctag); om_mesh_free(m); return OM_EMESH; }
        ++ne;
        if (j - i == 1) ++nb;
        i = j;
    }
    m->ne = ne; m->nb = nb;
    m->edge_l = (int *)malloc(sizeof(int) * ne);
    m->edge_kl = (int *)malloc(sizeof(int) * ne);
    m->edge_r = (int *)malloc(sizeof(int) * ne);
    m->edge_nx = (double *)malloc(sizeof(double) * ne);
    m->edge_ny = (double *)malloc(sizeof(double) * ne);
    m->edge_len = (double *)malloc(sizeof(double) * ne);
    long e = 0;
    for (long i = 0; i < 3 * nt; ++e) {
        long j = i + 1;
        while (j < 3 * nt && hs[j].key == hs[i].key) ++j;
        const long h0 = hs[i].half; /* lower cell id first: it defines the normal */
        const int c0 = (int)(h0 / 3), k0 = (int)(h0 % 3);
        m->edge_l[e] = c0; m->edge_kl[e] = k0;
        m->cell_edge[h0] = (int)e;
        if (j - i == 2) {
            const long h1 = hs[i + 1].half;
            const int c1 = (int)(h1 / 3), k1 = (int)(h1 % 3);
            /* Two counter-clockwise cells traverse a shared edge in opposite directions. */
            if (m->cell_node[3 * c0 + k0] != m->cell_node[3 * c1 + (k1 + 1) % 3]) {
                free(hs); free(ctag); om_mesh_free(m); return OM_EMESH;
            }
            m->edge_r[e] = c1;
            m->cell_edge[h1] = (int)e;
            m->cell_nbr[h0] = c1;
            m->cell_nbr[h1] = c0;
        } else {
            const int tg = ctag[h0];
            m->edge_r[e] = tg > 0 ? -1 - tg : OM_WALL;
            m->cell_nbr[h0] = m->edge_r[e];
        }
        om_edge_geom(m, c0, k0, &m->edge_nx[e], &m->edge_ny[e], &m->edge_len[e]);
        i = j;
    }
    free(hs); free(ctag);

    /* Cell area (the control volume of eq. 4) and inradius r = 2A/P (CFL length scale). */
    for (long c = 0; c < nt; ++c) {
        const int v0 = m->cell_node[3 * c], v1 = m->cell_node[3 * c + 1],
                  v2 = m->cell_node[3 * c + 2];
        const double e0x = xy[2 * v1] - xy[2 * v0], e0y = xy[2 * v1 + 1] - xy[2 * v0 + 1];
        const double e1x = xy[2 * v2] - xy[2 * v1], e1y = xy[2 * v2 + 1] - xy[2 * v1 + 1];
        const double a = 0.5 * (e0x * e1y - e0y * e1x);
        double nx, ny, l0, l1, l2;
        om_edge_geom(m, c, 0, &nx, &ny, &l0);
        om_edge_geom(m, c, 1, &nx, &ny, &l1);
        om_edge_geom(m, c, 2, &nx, &ny, &l2);
        m->area[c] = a;
        m->inradius[c] = 2.0 * a / (l0 + l1 + l2);
    }
    *out = m;
    return OM_OK;
}

void om_mesh_counts(const om_mesh *m, long *out4)
{
    out4[0] = m->nt; out4[1] = m->nv; out4[2] = m->ne; out4[3] = m->nb;
}

/* Copy the oracle's connectivity and geometry out (for tests). */
void om_mesh_arrays(const om_mesh *m, int *cell_node, int *cell_nbr, double *area,
                    double *inradius)
{
    if (cell_node) memcpy(cell_node, m->cell_node, sizeof(int) * 3 * m->nt);
    if (cell_nbr) memcpy(cell_nbr, m->cell_nbr, sizeof(int) * 3 * m->nt);
    if (area) memcpy(area, m->area, sizeof(double) * m->nt);
    if (inradius) memcpy(inradius, m->inradius, sizeof(double) * m->nt);
}

/* ------------------------------------------------------------------------- Riemann flux */

/* The branches the last flux evaluation of this thread took (wave-speed case and min/max
 * choices, flux region and contact side, reconstruction cases).  Recorded only: nothing reads
 * them but the branch signature of a run (om_run_loss_sig), which tells whether two runs
 * took the same branches everywhere. */
static __thread unsigned om_branch;

/* Wave-speed estimates S_L < S_R of the HLLC solver (section 2.2, ref. [6]) from the
 * reconstructed depths and normal velocities.  Returns 0 when both sides are dry. */
int om_wave_speeds(double g, double hl, double ql, double hr, double qr, double *sl, double *sr)
{
    if (hl == 0.0 && hr == 0.0) { *sl = 0.0; *sr = 0.0; om_branch = 0u; return 0; }
    const double cl = sqrt(g * hl), cr = sqrt(g * hr);
    if (hl == 0.0) {            /* dry left: the right state's rarefaction reaches the dry bed */
        *sl = qr - 2.0 * cr;
        *sr = qr + cr;
        om_branch = 1u;
    } else if (hr == 0.0) {     /* dry right */
        *sl = ql - cl;
        *sr = ql + 2.0 * cl;
        om_branch = 2u;
    } else {                    /* two-rarefaction estimate of the star state */
        const double us = (ql + qr) / 2.0 + (cl - cr);
        const double cs = (cl + cr) / 2.0 + (ql - qr) / 4.0;
        *sl = fmin(ql - cl, us - cs);
        *sr = fmax(qr + cr, us + cs);
        om_branch = 3u + (ql - cl <= us - cs ? 0u : 4u) + (qr + cr >= us + cs ? 0u : 8u);
    }
    return 1;
}

/*
 * HLLC numerical flux in the edge frame (section 2.2, ref. [6]): left and right reconstructed
 * depths with their normal (q) and tangential (w) velocities, normal pointing from left to
 * right.  Depths at or below the dry threshold must already be zero.  Outputs the mass,
 * normal-momentum and tangential-momentum fluxes per unit edge length.
 */
void om_hllc_normal(double g, double hl, double ql, double wl, double hr, double qr, double wr,
                    double *fh_out, double *fq_out, double *fw_out)
{
    double sl, sr;
    if (!om_wave_speeds(g, hl, ql, hr, qr, &sl, &sr)) {
        *fh_out = 0.0; *fq_out = 0.0; *fw_out = 0.0;
        return;
    }
    /* physical normal fluxes of eq. 1, (h q, h q^2 + g h^2 / 2) */
    const double fhl = hl * ql, fql = hl * ql * ql + 0.5 * g * hl * hl;
    const double fhr = hr * qr, fqr = hr * qr * qr + 0.5 * g * hr * hr;
    double fh, fq, fw;
    if (sl >= 0.0) {
        fh = fhl; fq = fql; fw = fh * wl;
        om_branch |= 16u;
    } else if (sr <= 0.0) {
        fh = fhr; fq = fqr; fw = fh * wr;
        om_branch |= 32u;
    } else {
        const double den = sr - sl;
        fh = ((sr * fhl - sl * fhr) + sl * sr * (hr - hl)) / den;
        fq = ((sr * fql - sl * fqr) + sl * sr * (hr * qr - hl * ql)) / den;
        const double sstar = (sl * hr * (qr - sr) - sr * hl * (ql - sl)) /
                             (hr * (qr - sr) - hl * (ql - sl));
        const double wup = sstar > 0.0 ? wl : (sstar < 0.0 ? wr : (wl + wr) / 2.0);
        fw = fh * wup;
        om_branch |= sstar > 0.0 ? 64u : (sstar < 0.0 ? 128u : 192u);
    }
    *fh_out = fh; *fq_out = fq; *fw_out = fw;
}

/* HLLC flux F_k . n_k of eq. 3 in (x, y) components: rotate the velocities into the edge
 * frame of the unit normal (nx, ny), solve there, rotate the momentum flux back. */
void om_hllc(double g, double hl, double ul, double vl, double hr, double ur, double vr,
             double nx, double ny, double *f)
{
    const double ql = ul * nx + vl * ny, wl = vl * nx - ul * ny;
    const double qr = ur * nx + vr * ny, wr = vr * nx - ur * ny;
    double fh, fq, fw;
    om_hllc_normal(g, hl, ql, wl, hr, qr, wr, &fh, &fq, &fw);
    f[0] = fh;
    f[1] = fq * nx - fw * ny;
    f[2] = fq * ny + fw * nx;
}

static inline double om_vel(double h, double hq, double h_dry)
{
    return h > h_dry ? hq / h : 0.0;
}

/*
 * Flux through one interface with hydrostatic reconstruction of the bed (section 2.2, S0
 * treatment): z* = max(zl, zr), h* = max(0, h - (z* - z)), velocities kept, and the bed
 * correction p = g/2 (h^2 - h*^2) on each side.  Right state given as conserved variables.
 * Outputs the flux (per unit length) and the two side pressures pl, pr.
 */
void om_interface(double g, double h_dry, double hl, double hul, double hvl, double zl,
                  double hr, double hur, double hvr, double zr, double nx, double ny,
                  double *f, double *pl, double *pr)
{
    const double zs = fmax(zl, zr);
    double hsl = fmax(0.0, hl - (zs - zl));
    double hsr = fmax(0.0, hr - (zs - zr));
    const unsigned rec = (zl > zr ? 1u : (zr > zl ? 2u : 3u)) |
                         (hl - (zs - zl) < 0.0 ? 4u : 0u) | (hsl <= h_dry ? 8u : 0u) |
                         (hr - (zs - zr) < 0.0 ? 16u : 0u) | (hsr <= h_dry ? 32u : 0u) |
                         (hl > h_dry ? 64u : 0u) | (hr > h_dry ? 128u : 0u);
    if (hsl <= h_dry) hsl = 0.0;
    if (hsr <= h_dry) hsr = 0.0;
    om_hllc(g, hsl, om_vel(hl, hul, h_dry), om_vel(hl, hvl, h_dry), hsr,
            om_vel(hr, hur, h_dry), om_vel(hr, hvr, h_dry), nx, ny, f);
    om_branch |= rec << 8;
    *pl = 0.5 * g * (hl * hl - hsl * hsl);
    *pr = 0.5 * g * (hr * hr - hsr * hsr);
}

/* Reflective wall (section 3): the ghost has the cell's depth and bed, its normal velocity
 * reversed and its tangential velocity kept, built directly in the edge frame so that the mass
 * flux through the wall is exactly zero.  The reconstruction leaves the depth unchanged (equal
 * beds), so the bed correction is g/2 (h^2 - h*^2) with h* = h unless the cell is dry. */
void om_wall(double g, double h_dry, double h, double hu, double hv, double nx, double ny,
             double *f, double *p)
{
    const double u = om_vel(h, hu, h_dry), v = om_vel(h, hv, h_dry);
    const double q = u * nx + v * ny, w = v * nx - u * ny;
    const double hs = h > h_dry ? h : 0.0;
    double fh, fq, fw;
    om_hllc_normal(g, hs, q, w, hs, -q, w, &fh, &fq, &fw);
    f[0] = fh;
    f[1] = fq * nx - fw * ny;
    f[2] = fq * ny + fw * nx;
    *p = 0.5 * g * (h * h - hs * hs);
}

/* Inflow segment: prescribed discharge q_in (m^2/s) entering through the edge, boundary depth
 * h_b = max(h, (q_in^2/g)^(1/3)).  Returns the flux and the boundary wave speed. */
static double om_inflow(double g, double q_in, double h, double nx, double ny, double *f)
{
    const double hc = cbrt(q_in * q_in / g);
    const double hb = fmax(h, hc);
    const double mom = q_in * q_in / hb + 0.5 * g * hb * hb;
    f[0] = -q_in;
    f[1] = mom * nx;
    f[2] = mom * ny;
    return q_in / hb + sqrt(g * hb);
}

/* ---------------------------------------------------------------------------- stepping */

/* CFL time step of section 2.2 with Courant number C: C min over wet cells of
 * r_i / (|u_i| + sqrt(g h_i)); inflow cells also bound it with their boundary wave speed.
 * Returns +inf when no cell is wet. */
double om_cfl_dt(const om_mesh *m, const double *h, const double *hu, const double *hv,
                 const om_params *p)
{
    double best = INFINITY;
#pragma omp parallel for reduction(min : best) schedule(static)
    for (long c = 0; c < m->nt; ++c) {
        double s = 0.0;
        if (h[c] > p->h_dry) {
            const double u = hu[c] / h[c], v = hv[c] / h[c];
            s = sqrt(u * u + v * v) + sqrt(p->g * h[c]);
        }
        for (int k = 0; k < 3; ++k) {
            const int nb = m->cell_nbr[3 * c + k];
            if (nb < OM_WALL) {
                double f[3];
                const double sb = om_inflow(p->g, p->inflow_q[-1 - nb - 1], h[c], 0.0, 0.0, f);
                if (sb > s) s = sb;
            }
        }
        if (s > 0.0) {
            const double d = m->inradius[c] / s;
            if (d < best) best = d;
        }
    }
    return p->courant * best;
}

/* Workspace of one step: per-edge flux and side pressures. */
typedef struct {
    double *f, *pl, *pr;
    unsigned *ecode, *ccode;   /* NULL, or each edge's and cell's branches (om_run_loss_sig) */
} om_work;

/*
 * One explicit Euler step (eq. 4) of length dt: fluxes over all interfaces (section 2.3,
 * first parallel loop), then the cell update (second loop): U* = U - dt/A sum_k l_k (F_k +
 * bed correction), negative depths clamped to zero, then semi-implicit Manning friction
 * (the S_f term of eq. 1) and zero momentum in dry cells.
 */
static void om_step(const om_mesh *m, const double *z, const double *n, double *h, double *hu,
                    double *hv, const om_params *p, double dt, om_work *w, om_stats *st)
{
    const double g = p->g, hd = p->h_dry;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < m->ne; ++e) {
        const int l = m->edge_l[e], r = m->edge_r[e];
        double *f = w->f + 3 * e;
        if (r >= 0) {
            om_interface(g, hd, h[l], hu[l], hv[l], z[l], h[r], hu[r], hv[r], z[r],
                         m->edge_nx[e], m->edge_ny[e], f, &w->pl[e], &w->pr[e]);
        } else if (r == OM_WALL) {
            om_wall(g, hd, h[l], hu[l], hv[l], m->edge_nx[e], m->edge_ny[e], f, &w->pl[e]);
            w->pr[e] = 0.0;
            om_branch |= (h[l] > hd ? 1u : 2u) << 16;
        } else {
            om_inflow(g, p->inflow_q[-1 - r - 1], h[l], m->edge_nx[e], m->edge_ny[e], f);
            w->pl[e] = 0.0;
            w->pr[e] = 0.0;
            om_branch = (h[l] >= cbrt(p->inflow_q[-1 - r - 1] * p->inflow_q[-1 - r - 1] / g)
                             ? 4u : 8u) << 16;
        }
        if (w->ecode) w->ecode[e] = om_branch;
    }
    long clamps = 0;
    double clamped = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : clamps, clamped)
    for (long c = 0; c < m->nt; ++c) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3; ++k) {
            const int e = m->cell_edge[3 * c + k];
            const double s = (m->edge_l[e] == c) ? 1.0 : -1.0;
            const double pk = (m->edge_l[e] == c) ? w->pl[e] : w->pr[e];
            const double l = m->edge_len[e];
            const double nx = s * m->edge_nx[e], ny = s * m->edge_ny[e];
            const double c0 = l * (s * w->f[3 * e]);
            const double c1 = l * (s * w->f[3 * e + 1] + pk * nx);
            const double c2 = l * (s * w->f[3 * e + 2] + pk * ny);
            if (k == 0) { acc[0] = c0; acc[1] = c1; acc[2] = c2; }
            else { acc[0] = acc[0] + c0; acc[1] = acc[1] + c1; acc[2] = acc[2] + c2; }
        }
        const double r = dt / m->area[c];
        double hs = h[c] - r * acc[0];
        const double hus = hu[c] - r * acc[1];
        const double hvs = hv[c] - r * acc[2];
        if (w->ccode) w->ccode[c] = (hs < 0.0 ? 1u : 0u) | (hs > hd ? 2u : 0u);
        if (hs < 0.0) { ++clamps; clamped += -hs * m->area[c]; hs = 0.0; }
        if (hs > hd) {
            const double mag = sqrt(hus * hus + hvs * hvs);
            const double d = 1.0 + dt * g * n[c] * n[c] * mag / (hs * hs * cbrt(hs));
            hu[c] = hus / d;
            hv[c] = hvs / d;
        } else {
            hu[c] = 0.0;
            hv[c] = 0.0;
        }
        h[c] = hs;
    }
    st->clamps += clamps;
    st->clamped_mass += clamped;
}

/*
 * Run up to nsteps steps (the host time loop of section 2.3).  dt comes from the CFL
 * condition on the current state unless dt_seq is given.  With t_end > 0 the run stops at
 * t_end: a step whose CFL dt reaches past it is shortened to end exactly there.  dt_out (may
 * be NULL) receives each step's dt.  Returns OM_EDRY if a step finds no wet cell and
 * OM_ENONFINITE if the state stops being finite.
 */
int om_run(const om_mesh *m, const double *z, const double *n, double *h, double *hu,
           double *hv, const om_params *p, long nsteps, double t_end, const double *dt_seq,
           double *dt_out, om_stats *st)
{
    for (long c = 0; c < 3 * m->nt; ++c) {
        const int nb = m->cell_nbr[c];
        if (nb < OM_WALL && (-1 - nb > p->n_inflow || !p->inflow_q)) return OM_EINVAL;
    }
    if (!(p->g > 0.0) || !(p->courant > 0.0) || !(p->courant <= 1.0) || !(p->h_dry >= 0.0))
        return OM_EINVAL;
    om_work w;
    w.ecode = w.ccode = NULL;
    w.f = (double *)malloc(sizeof(double) * 3 * m->ne);
    w.pl = (double *)malloc(sizeof(double) * m->ne);
    w.pr = (double *)malloc(sizeof(double) * m->ne);
    int rc = OM_OK;
    st->steps = 0;
    st->last_reached = 0;
    for (long s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && st->t >= t_end) { st->last_reached = 1; break; }
        double dt = dt_seq ? dt_seq[s] : om_cfl_dt(m, h, hu, hv, p);
        if (!(dt < INFINITY)) { rc = OM_EDRY; break; }
        if (!(dt > 0.0)) { rc = OM_ENONFINITE; break; }
        int last = 0;
        if (t_end > 0.0 && dt >= t_end - st->t) { dt = t_end - st->t; last = 1; }
        om_step(m, z, n, h, hu, hv, p, dt, &w, st);
        st->t = last ? t_end : st->t + dt;
        if (dt_out) dt_out[s] = dt;
        if (st->steps == 0 || dt < st->dt_min) st->dt_min = dt;
        if (st->steps == 0 || dt > st->dt_max) st->dt_max = dt;
        st->dt_sum += dt;
        st->steps += 1;
        if (last) { st->last_reached = 1; break; }
    }
    if (rc == OM_OK) {
        for (long c = 0; c < m->nt; ++c)
            if (!isfinite(h[c]) || !isfinite(hu[c]) || !isfinite(hv[c])) { rc = OM_ENONFINITE; break; }
    }
    free(w.f); free(w.pl); free(w.pr);
    return rc;
}

void om_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int om_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------- batched entry points
 * Vector forms of the flux functions above, so tests can probe millions of states. */

void om_hllc_batch(long n, double g, const double *hl, const double *ul, const double *vl,
                   const double *hr, const double *ur, const double *vr, const double *nx,
                   const double *ny, double *f)
{
    for (long i = 0; i < n; ++i)
        om_hllc(g, hl[i], ul[i], vl[i], hr[i], ur[i], vr[i], nx[i], ny[i], f + 3 * i);
}

void om_interface_batch(long n, double g, double h_dry, const double *hl, const double *hul,
                        const double *hvl, const double *zl, const double *hr,
                        const double *hur, const double *hvr, const double *zr,
                        const double *nx, const double *ny, double *f, double *pl, double *pr)
{
    for (long i = 0; i < n; ++i)
        om_interface(g, h_dry, hl[i], hul[i], hvl[i], zl[i], hr[i], hur[i], hvr[i], zr[i],
                     nx[i], ny[i], f + 3 * i, pl + i, pr + i);
}

void om_wall_batch(long n, double g, double h_dry, const double *h, const double *hu,
                   const double *hv, const double *nx, const double *ny, double *f, double *p)
{
    for (long i = 0; i < n; ++i)
        om_wall(g, h_dry, h[i], hu[i], hv[i], nx[i], ny[i], f + 3 * i, p + i);
}

void om_wave_speeds_batch(long n, double g, const double *hl, const double *ql,
                          const double *hr, const double *qr, double *sl, double *sr)
{
    for (long i = 0; i < n; ++i) om_wave_speeds(g, hl[i], ql[i], hr[i], qr[i], sl + i, sr + i);
}

/* Inflow flux (3 values per edge) and boundary wave speed of n independent inflow edges. */
void om_inflow_batch(long n, double g, const double *q_in, const double *h, const double *nx,
                     const double *ny, double *f, double *speed)
{
    for (long i = 0; i < n; ++i) speed[i] = om_inflow(g, q_in[i], h[i], nx[i], ny[i], f + 3 * i);
}

/* ----------------------------------------------------------------- tangent-linear model
 *
 * Forward-mode derivative of om_run with the dt sequence replayed (dt is not differentiated),
 * for the gauge misfit J = sum over observation steps m*every (m >= 1) and gauges g of
 * (h_g - obs[m-1][g])^2.  Every quantity carries (value, derivative along one direction);
 * every branch (max, min, dry tests, wave-speed cases, the sign of S*) is taken on values, so
 * the derivative is that of the branch the plain run takes.  Used to pin the GPU adjoint.
 */
typedef struct { double v, d; } om_dual;

static inline om_dual dv(double v, double d) { om_dual r = {v, d}; return r; }
static inline om_dual dc(double v) { return dv(v, 0.0); }
static inline om_dual dadd(om_dual a, om_dual b) { return dv(a.v + b.v, a.d + b.d); }
static inline om_dual dsub(om_dual a, om_dual b) { return dv(a.v - b.v, a.d - b.d); }
static inline om_dual dmul(om_dual a, om_dual b) { return dv(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline om_dual ddiv(om_dual a, om_dual b)
{
    const double q = a.v / b.v;
    return dv(q, (a.d - q * b.d) / b.v);
}
static inline om_dual dneg(om_dual a) { return dv(-a.v, -a.d); }
static inline om_dual dscale(double s, om_dual a) { return dv(s * a.v, s * a.d); }
static inline om_dual dsqrt(om_dual a)
{
    const double r = sqrt(a.v);
    return dv(r, r > 0.0 ? a.d / (2.0 * r) : 0.0);
}
static inline om_dual dcbrt(om_dual a)
{
    const double r = cbrt(a.v);
    return dv(r, r != 0.0 ? a.d / (3.0 * r * r) : 0.0);
}
static inline om_dual dmax(om_dual a, om_dual b) { return a.v >= b.v ? a : b; }
static inline om_dual dmin(om_dual a, om_dual b) { return a.v <= b.v ? a : b; }

static void om_hllc_normal_tl(double g, om_dual hl, om_dual ql, om_dual wl, om_dual hr,
                              om_dual qr, om_dual wr, om_dual *fh_o, om_dual *fq_o,
                              om_dual *fw_o)
{
    if (hl.v == 0.0 && hr.v == 0.0) { *fh_o = dc(0.0); *fq_o = dc(0.0); *fw_o = dc(0.0); return; }
    const om_dual cl = dsqrt(dscale(g, hl)), cr = dsqrt(dscale(g, hr));
    om_dual sl, sr;
    if (hl.v == 0.0) {
        sl = dsub(qr, dscale(2.0, cr));
        sr = dadd(qr, cr);
    } else if (hr.v == 0.0) {
        sl = dsub(ql, cl);
        sr = dadd(ql, dscale(2.0, cl));
    } else {
        const om_dual us = dadd(dscale(0.5, dadd(ql, qr)), dsub(cl, cr));
        const om_dual cs = dadd(dscale(0.5, dadd(cl, cr)), dscale(0.25, dsub(ql, qr)));
        sl = dmin(dsub(ql, cl), dsub(us, cs));
        sr = dmax(dadd(qr, cr), dadd(us, cs));
    }
    const om_dual fhl = dmul(hl, ql);
    const om_dual fql = dadd(dmul(dmul(hl, ql), ql), dmul(dscale(0.5 * g, hl), hl));
    const om_dual fhr = dmul(hr, qr);
    const om_dual fqr = dadd(dmul(dmul(hr, qr), qr), dmul(dscale(0.5 * g, hr), hr));
    om_dual fh, fq, fw;
    if (sl.v >= 0.0) {
        fh = fhl; fq = fql; fw = dmul(fh, wl);
    } else if (sr.v <= 0.0) {
        fh = fhr; fq = fqr; fw = dmul(fh, wr);
    } else {
        const om_dual den = dsub(sr, sl);
        const om_dual slsr = dmul(sl, sr);
        fh = ddiv(dadd(dsub(dmul(sr, fhl), dmul(sl, fhr)), dmul(slsr, dsub(hr, hl))), den);
        fq = ddiv(dadd(dsub(dmul(sr, fql), dmul(sl, fqr)),
                       dmul(slsr, dsub(dmul(hr, qr), dmul(hl, ql)))), den);
        const double sstar = (sl.v * hr.v * (qr.v - sr.v) - sr.v * hl.v * (ql.v - sl.v)) /
                             (hr.v * (qr.v - sr.v) - hl.v * (ql.v - sl.v));
        const om_dual wup = sstar > 0.0 ? wl : (sstar < 0.0 ? wr : dscale(0.5, dadd(wl, wr)));
        fw = dmul(fh, wup);
    }
    *fh_o = fh; *fq_o = fq; *fw_o = fw;
}

static inline om_dual om_vel_tl(om_dual h, om_dual hq, double h_dry)
{
    return h.v > h_dry ? ddiv(hq, h) : dc(0.0);
}

static void om_interface_tl(double g, double hd, om_dual hl, om_dual hul, om_dual hvl,
                            om_dual zl, om_dual hr, om_dual hur, om_dual hvr, om_dual zr,
                            double nx, double ny, om_dual *f, om_dual *pl, om_dual *pr)
{
    /* max of the beds; at a tie the derivative is split between the two sides */
    const om_dual zs = zl.v > zr.v ? zl : (zr.v > zl.v ? zr : dv(zl.v, 0.5 * (zl.d + zr.d)));
    om_dual hsl = dmax(dc(0.0), dsub(hl, dsub(zs, zl)));
    om_dual hsr = dmax(dc(0.0), dsub(hr, dsub(zs, zr)));
    if (hsl.v <= hd) hsl = dc(0.0);
    if (hsr.v <= hd) hsr = dc(0.0);
    const om_dual ul = om_vel_tl(hl, hul, hd), vl = om_vel_tl(hl, hvl, hd);
    const om_dual ur = om_vel_tl(hr, hur, hd), vr = om_vel_tl(hr, hvr, hd);
    const om_dual ql = dadd(dscale(nx, ul), dscale(ny, vl)), wl = dsub(dscale(nx, vl), dscale(ny, ul));
    const om_dual qr = dadd(dscale(nx, ur), dscale(ny, vr)), wr = dsub(dscale(nx, vr), dscale(ny, ur));
    om_dual fh, fq, fw;
    om_hllc_normal_tl(g, hsl, ql, wl, hsr, qr, wr, &fh, &fq, &fw);
    f[0] = fh;
    f[1] = dsub(dscale(nx, fq), dscale(ny, fw));
    f[2] = dadd(dscale(ny, fq), dscale(nx, fw));
    *pl = dscale(0.5 * g, dsub(dmul(hl, hl), dmul(hsl, hsl)));
    *pr = dscale(0.5 * g, dsub(dmul(hr, hr), dmul(hsr, hsr)));
}

static void om_wall_tl(double g, double hd, om_dual h, om_dual hu, om_dual hv, double nx,
                       double ny, om_dual *f, om_dual *p)
{
    const om_dual u = om_vel_tl(h, hu, hd), v = om_vel_tl(h, hv, hd);
    const om_dual q = dadd(dscale(nx, u), dscale(ny, v)), w = dsub(dscale(nx, v), dscale(ny, u));
    const om_dual hs = h.v > hd ? h : dc(0.0);
    om_dual fh, fq, fw;
    om_hllc_normal_tl(g, hs, q, w, hs, dneg(q), w, &fh, &fq, &fw);
    f[0] = fh;
    f[1] = dsub(dscale(nx, fq), dscale(ny, fw));
    f[2] = dadd(dscale(ny, fq), dscale(nx, fw));
    *p = dscale(0.5 * g, dsub(dmul(h, h), dmul(hs, hs)));
}

static void om_inflow_tl(double g, double q_in, om_dual h, double nx, double ny, om_dual *f)
{
    const om_dual hc = dc(cbrt(q_in * q_in / g));
    const om_dual hb = dmax(h, hc);
    const om_dual mom = dadd(ddiv(dc(q_in * q_in), hb), dmul(dscale(0.5 * g, hb), hb));
    f[0] = dc(-q_in);
    f[1] = dscale(nx, mom);
    f[2] = dscale(ny, mom);
}

/* One step of the tangent-linear model (the same operations as om_step on duals). */
static void om_step_tl(const om_mesh *m, const om_dual *z, const om_dual *n, om_dual *h,
                       om_dual *hu, om_dual *hv, const om_params *p, double dt, om_dual *f,
                       om_dual *pl, om_dual *pr)
{
    const double g = p->g, hd = p->h_dry;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < m->ne; ++e) {
        const int l = m->edge_l[e], r = m->edge_r[e];
        if (r >= 0) {
            om_interface_tl(g, hd, h[l], hu[l], hv[l], z[l], h[r], hu[r], hv[r], z[r],
                            m->edge_nx[e], m->edge_ny[e], f + 3 * e, &pl[e], &pr[e]);
        } else if (r == OM_WALL) {
            om_wall_tl(g, hd, h[l], hu[l], hv[l], m->edge_nx[e], m->edge_ny[e], f + 3 * e, &pl[e]);
            pr[e] = dc(0.0);
        } else {
            om_inflow_tl(g, p->inflow_q[-1 - r - 1], h[l], m->edge_nx[e], m->edge_ny[e], f + 3 * e);
            pl[e] = dc(0.0);
            pr[e] = dc(0.0);
        }
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < m->nt; ++c) {
        om_dual acc[3];
        for (int k = 0; k < 3; ++k) {
            const int e = m->cell_edge[3 * c + k];
            const double s = (m->edge_l[e] == c) ? 1.0 : -1.0;
            const om_dual pk = (m->edge_l[e] == c) ? pl[e] : pr[e];
            const double l = m->edge_len[e];
            const double nx = s * m->edge_nx[e], ny = s * m->edge_ny[e];
            const om_dual c0 = dscale(l, dscale(s, f[3 * e]));
            const om_dual c1 = dscale(l, dadd(dscale(s, f[3 * e + 1]), dscale(nx, pk)));
            const om_dual c2 = dscale(l, dadd(dscale(s, f[3 * e + 2]), dscale(ny, pk)));
            if (k == 0) { acc[0] = c0; acc[1] = c1; acc[2] = c2; }
            else { acc[0] = dadd(acc[0], c0); acc[1] = dadd(acc[1], c1); acc[2] = dadd(acc[2], c2); }
        }
        const double r = dt / m->area[c];
        om_dual hs = dsub(h[c], dscale(r, acc[0]));
        const om_dual hus = dsub(hu[c], dscale(r, acc[1]));
        const om_dual hvs = dsub(hv[c], dscale(r, acc[2]));
        if (hs.v < 0.0) hs = dc(0.0);
        if (hs.v > hd) {
            const om_dual mag = dsqrt(dadd(dmul(hus, hus), dmul(hvs, hvs)));
            const om_dual kk = dmul(dmul(dc(dt * g), n[c]), n[c]);
            const om_dual d = dadd(dc(1.0), ddiv(dmul(kk, mag), dmul(dmul(hs, hs), dcbrt(hs))));
            hu[c] = ddiv(hus, d);
            hv[c] = ddiv(hvs, d);
        } else {
            hu[c] = dc(0.0);
            hv[c] = dc(0.0);
        }
        h[c] = hs;
    }
}

/*
 * Run nsteps tangent-linear steps from (U, dU) with the bed, roughness and their directions;
 * J and its directional derivative dJ are returned for gauges (mesh cells of the oracle, i.e.
 * input order) observed every `every` steps with obs[(m-1)*ng + g].  State arrays are
 * overwritten with the final values and derivatives.
 */
int om_run_tl(const om_mesh *m, const double *z, const double *zd, const double *n,
              const double *nd, double *h, double *hdot, double *hu, double *hudot, double *hv,
              double *hvdot, const om_params *p, long nsteps, const double *dt_seq,
              const int *gauges, int ng, int every, const double *obs, double *J, double *dJ)
{
    if (!dt_seq || every < 1) return OM_EINVAL;
    const long T = m->nt;
    om_dual *Z = (om_dual *)malloc(sizeof(om_dual) * T), *N = (om_dual *)malloc(sizeof(om_dual) * T);
    om_dual *H = (om_dual *)malloc(sizeof(om_dual) * T), *HU = (om_dual *)malloc(sizeof(om_dual) * T);
    om_dual *HV = (om_dual *)malloc(sizeof(om_dual) * T);
    om_dual *f = (om_dual *)malloc(sizeof(om_dual) * 3 * m->ne);
    om_dual *pl = (om_dual *)malloc(sizeof(om_dual) * m->ne), *pr = (om_dual *)malloc(sizeof(om_dual) * m->ne);
    for (long c = 0; c < T; ++c) {
        Z[c] = dv(z[c], zd ? zd[c] : 0.0);
        N[c] = dv(n[c], nd ? nd[c] : 0.0);
        H[c] = dv(h[c], hdot ? hdot[c] : 0.0);
        HU[c] = dv(hu[c], hudot ? hudot[c] : 0.0);
        HV[c] = dv(hv[c], hvdot ? hvdot[c] : 0.0);
    }
    double jv = 0.0, jd = 0.0;
    for (long s = 0; s < nsteps; ++s) {
        om_step_tl(m, Z, N, H, HU, HV, p, dt_seq[s], f, pl, pr);
        if ((s + 1) % every == 0) {
            const double *o = obs + ((s + 1) / every - 1) * (long)ng;
            for (int q = 0; q < ng; ++q) {
                const om_dual r = dsub(H[gauges[q]], dc(o[q]));
                jv += r.v * r.v;
                jd += 2.0 * r.v * r.d;
            }
        }
    }
    for (long c = 0; c < T; ++c) {
        h[c] = H[c].v; hu[c] = HU[c].v; hv[c] = HV[c].v;
        if (hdot) hdot[c] = H[c].d;
        if (hudot) hudot[c] = HU[c].d;
        if (hvdot) hvdot[c] = HV[c].d;
    }
    *J = jv;
    *dJ = jd;
    free(Z); free(N); free(H); free(HU); free(HV); free(f); free(pl); free(pr);
    return OM_OK;
}

/* A 64-bit mix of (step, index, branch code), summed by exclusive or over every edge and cell
 * of every step: equal signatures mean, barring a collision, runs that took the same branches
 * everywhere (the splitmix64 finaliser). */
static unsigned long om_mix(unsigned long x)
{
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ul;
    x ^= x >> 27; x *= 0x94d049bb133111ebul;
    return x ^ (x >> 31);
}

/* om_run_loss with the replayed dt sequence, plus the branch signature of the run: finite
 * differences of the loss are compared with the adjoint only where the perturbed runs keep the
 * base run's signature, i.e. away from switches. */
int om_run_loss_sig(const om_mesh *m, const double *z, const double *n, double *h, double *hu,
                    double *hv, const om_params *p, long nsteps, const double *dt_seq,
                    const int *gauges, int ng, int every, const double *obs, double *J,
                    unsigned long *sig)
{
    if (!(p->g > 0.0) || !(p->h_dry >= 0.0) || every < 1) return OM_EINVAL;
    om_work w;
    w.f = (double *)malloc(sizeof(double) * 3 * m->ne);
    w.pl = (double *)malloc(sizeof(double) * m->ne);
    w.pr = (double *)malloc(sizeof(double) * m->ne);
    w.ecode = (unsigned *)malloc(sizeof(unsigned) * m->ne);
    w.ccode = (unsigned *)malloc(sizeof(unsigned) * m->nt);
    om_stats st;
    memset(&st, 0, sizeof(st));
    double jv = 0.0;
    unsigned long sg = 0;
    for (long s = 0; s < nsteps; ++s) {
        om_step(m, z, n, h, hu, hv, p, dt_seq[s], &w, &st);
        const unsigned long base = om_mix((unsigned long)s);
#pragma omp parallel for reduction(^ : sg) schedule(static)
        for (long e = 0; e < m->ne; ++e)
            sg ^= om_mix(base ^ ((unsigned long)e << 24) ^ w.ecode[e]);
#pragma omp parallel for reduction(^ : sg) schedule(static)
        for (long c = 0; c < m->nt; ++c)
            sg ^= om_mix(~base ^ ((unsigned long)c << 24) ^ w.ccode[c]);
        if ((s + 1) % every == 0) {
            const double *o = obs + ((s + 1) / every - 1) * (long)ng;
            for (int q = 0; q < ng; ++q) {
                const double r = h[gauges[q]] - o[q];
                jv += r * r;
            }
        }
    }
    free(w.f); free(w.pl); free(w.pr); free(w.ecode); free(w.ccode);
    *J = jv;
    *sig = sg;
    return OM_OK;
}

/* The misfit alone, from a plain run with the replayed dt sequence (for finite differences). */
int om_run_loss(const om_mesh *m, const double *z, const double *n, double *h, double *hu,
                double *hv, const om_params *p, long nsteps, const double *dt_seq,
                const int *gauges, int ng, int every, const double *obs, double *J)
{
    double jv = 0.0;
    om_stats st;
    memset(&st, 0, sizeof(st));
    for (long s = 0; s < nsteps; ++s) {
        int rc = om_run(m, z, n, h, hu, hv, p, 1, 0.0, dt_seq + s, NULL, &st);
        if (rc != OM_OK) return rc;
        if ((s + 1) % every == 0) {
            const double *o = obs + ((s + 1) / every - 1) * (long)ng;
            for (int q = 0; q < ng; ++q) {
                const double r = h[gauges[q]] - o[q];
                jv += r * r;
            }
        }
    }
    *J = jv;
    return OM_OK;
}
