// Hand-written reverse (adjoint) sweep of the FP64 step, for the gradient of a gauge misfit
// with respect to the Manning roughness, the bed and the initial state.
//
// The forward map of one step is U^{n+1} = friction(clamp(U^n - dt/A sum_k c_k(U^n, z))) with
// the interface contributions c_k of eq. 3 (HLLC with hydrostatic reconstruction) and the
// semi-implicit friction of the S_f term of eq. 1.  Its transpose is applied in two per-cell
// kernels: the friction/clamp adjoint mu = (dU^{n+1}/dU*)^T lambda^{n+1} (with the roughness
// gradient), then the flux adjoint lambda^n = mu + sum over the cell's edges of the transposed
// edge Jacobians applied to both sides' cotangents -dt/A mu.  Adjacency is symmetric, so each
// cell gathers its own share: no atomics, deterministic.  Every branch of the forward step
// (max of the beds, positive parts, dry tests, wave-speed cases, min/max of the speed
// estimates, supersonic or HLL, the sign of the contact speed, the clamp) is re-evaluated on
// the forward values and its derivative taken as is.  dt is replayed, not differentiated.
//
// Forward states are checkpointed every K steps; the reverse pass recomputes each segment
// (storing U^n and the pre-friction U*) and then runs the adjoint through it backwards; the
// forward pass stores the last segment so, and it is not recomputed.  With
// K = 1 the forward pass itself stores every U^n and U* (HBM holds them for the meshes and
// step counts of a calibration run) and the reverse pass recomputes nothing.  The forward
// passes replay dt without the control block.  FP64 divisions and square roots of the
// adjoint use the Newton forms of swe_device_math.h; quotients by one divisor are products
// with its reciprocal (within about an ulp), as in the default step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "swe_device_math.h"
#include "swe_internal.h"

// 1: the flux adjoint runs tiled (each interface once) wherever the step runs tiled.
#ifndef SWE_TILE_ADJOINT
#define SWE_TILE_ADJOINT 1
#endif

namespace swe {
namespace {

struct Vjp3 {
    double h, hu, hv;
};

// Forward values are recomputed in the forms of the default FP64 step (one reciprocal per
// divisor, lengths and unit normals from one reciprocal square root), so the branches taken
// here are the forward run's.
__device__ __forceinline__ double vel(double h, double hq, double hd)
{
    return h > hd ? hq * rcp_nr(h) : 0.0;
}

// Length and outward unit normal of an edge vector, as the step forms them.
__device__ __forceinline__ void edge_normal_nr(double dx, double dy, double &nx, double &ny,
                                               double &l)
{
    double il;
    len_rcp_nr(dx * dx + dy * dy, l, il);
    nx = quot_nr(dy, il, l);
    ny = quot_nr(-dx, il, l);
}

// Cotangents of (hl, ql, wl, hr, qr, wr) from those of the edge-frame HLLC flux (fh, fq, fw).
__device__ void hllc_normal_vjp(double g, double hl, double ql, double wl, double hr, double qr,
                                double wr, double fhb, double fqb, double fwb, double &hlb,
                                double &qlb, double &wlb, double &hrb, double &qrb, double &wrb)
{
    hlb = qlb = wlb = hrb = qrb = wrb = 0.0;
    if (hl == 0.0 && hr == 0.0) return;
    const double cl = sqrt_nr(g * hl), cr = sqrt_nr(g * hr);
    double sl, sr, us = 0.0, cs = 0.0;
    bool sl_a = true, sr_a = true;
    if (hl == 0.0) {
        sl = qr - 2.0 * cr;
        sr = qr + cr;
    } else if (hr == 0.0) {
        sl = ql - cl;
        sr = ql + 2.0 * cl;
    } else {
        us = (ql + qr) / 2.0 + (cl - cr);
        cs = (cl + cr) / 2.0 + (ql - qr) / 4.0;
        sl_a = (ql - cl) <= (us - cs);
        sr_a = (qr + cr) >= (us + cs);
        sl = sl_a ? ql - cl : us - cs;
        sr = sr_a ? qr + cr : us + cs;
    }
    const double fhl = hl * ql, fql = hl * ql * ql + 0.5 * g * hl * hl;
    const double fhr = hr * qr, fqr = hr * qr * qr + 0.5 * g * hr * hr;
    double fhlb = 0.0, fqlb = 0.0, fhrb = 0.0, fqrb = 0.0, slb = 0.0, srb = 0.0;
    if (sl >= 0.0) {
        fhlb = fhb + fwb * wl;
        wlb += fwb * fhl;
        fqlb = fqb;
    } else if (sr <= 0.0) {
        fhrb = fhb + fwb * wr;
        wrb += fwb * fhr;
        fqrb = fqb;
    } else {
        const double den = sr - sl;
        const double dh = hr - hl, dq = hr * qr - hl * ql;
        const double rden = rcp_nr(den);
        const double fh = quot_nr((sr * fhl - sl * fhr) + sl * sr * dh, rden, den);
        const double fq = quot_nr((sr * fql - sl * fqr) + sl * sr * dq, rden, den);
        // the sign of the contact speed as the step takes it (den2 < 0 here: -num, unless the
        // quotient could underflow)
        const double num = sl * hr * (qr - sr) - sr * hl * (ql - sl);
        const double den2 = hr * (qr - sr) - hl * (ql - sl);
        const double sstar = fabs(num) < 0x1p-1000 * fabs(den2) ? div_nr(num, den2) : -num;
        const int sel = sstar > 0.0 ? 1 : (sstar < 0.0 ? 2 : 3);
        const double wup = sel == 1 ? wl : (sel == 2 ? wr : (wl + wr) / 2.0);
        const double fhtb = fhb + fwb * wup;
        const double wupb = fwb * fh;
        // both zero before this branch; set by value (a store through a chosen reference
        // would keep them in memory)
        wlb = sel == 1 ? wupb : (sel == 3 ? 0.5 * wupb : 0.0);
        wrb = sel == 2 ? wupb : (sel == 3 ? 0.5 * wupb : 0.0);
        const double nhb = fhtb * rden, nqb = fqb * rden;
        const double denb = -((fhtb * fh + fqb * fq) * rden);
        srb += nhb * (fhl + sl * dh) + nqb * (fql + sl * dq) + denb;
        slb += nhb * (-fhr + sr * dh) + nqb * (-fqr + sr * dq) - denb;
        fhlb += nhb * sr;
        fhrb -= nhb * sl;
        fqlb += nqb * sr;
        fqrb -= nqb * sl;
        hrb += nhb * sl * sr;
        hlb -= nhb * sl * sr;
        const double dqb = nqb * sl * sr;
        hrb += dqb * qr;
        qrb += dqb * hr;
        hlb -= dqb * ql;
        qlb -= dqb * hl;
    }
    hlb += fhlb * ql + fqlb * (ql * ql + g * hl);
    qlb += fhlb * hl + fqlb * 2.0 * hl * ql;
    hrb += fhrb * qr + fqrb * (qr * qr + g * hr);
    qrb += fhrb * hr + fqrb * 2.0 * hr * qr;
    double clb = 0.0, crb = 0.0;
    if (hl == 0.0) {
        qrb += slb + srb;
        crb += -2.0 * slb + srb;
    } else if (hr == 0.0) {
        qlb += slb + srb;
        clb += -slb + 2.0 * srb;
    } else {
        double usb = 0.0, csb = 0.0;
        if (sl_a) { qlb += slb; clb -= slb; } else { usb += slb; csb -= slb; }
        if (sr_a) { qrb += srb; crb += srb; } else { usb += srb; csb += srb; }
        qlb += 0.5 * usb;
        qrb += 0.5 * usb;
        clb += usb;
        crb -= usb;
        clb += 0.5 * csb;
        crb += 0.5 * csb;
        qlb += 0.25 * csb;
        qrb -= 0.25 * csb;
    }
    if (cl > 0.0) hlb += (0.5 * clb * g) * rcp_nr(cl);
    if (cr > 0.0) hrb += (0.5 * crb * g) * rcp_nr(cr);
}

// Cotangent of a cell's velocity pair (u, v) = (hu, hv)/h pulled back to (h, hu, hv).
__device__ __forceinline__ void vel_vjp(double h, double hu, double hv, double hd, double ub,
                                        double vb, Vjp3 &out)
{
    if (h > hd) {
        const double ih = rcp_nr(h);
        const double u = hu * ih, v = hv * ih;
        out.h -= (ub * u + vb * v) * ih;
        out.hu += ub * ih;
        out.hv += vb * ih;
    }
}

// Interior interface a-b (unit normal out of a, length l): cotangents of both sides' cells
// and beds from those of a's and b's contributions l (F + p n) and l (-F - p_b n).
__device__ void interface_vjp(double g, double hd, double ha, double hua, double hva, double za,
                              double hb, double hub, double hvb, double zb, double nx, double ny,
                              double l, const double *cab, const double *cbb, Vjp3 &ua_out,
                              double &za_out, Vjp3 &ub_out, double &zb_out)
{
    const double zs = fmax(za, zb);
    const double ra = ha - (zs - za), rb = hb - (zs - zb);
    double hsa = fmax(0.0, ra), hsb = fmax(0.0, rb);
    const bool act_a = ra > 0.0 && hsa > hd, act_b = rb > 0.0 && hsb > hd;
    if (hsa <= hd) hsa = 0.0;
    if (hsb <= hd) hsb = 0.0;
    const double ua = vel(ha, hua, hd), va = vel(ha, hva, hd);
    const double ubv = vel(hb, hub, hd), vbv = vel(hb, hvb, hd);
    const double qa = ua * nx + va * ny, wa = va * nx - ua * ny;
    const double qb = ubv * nx + vbv * ny, wb = vbv * nx - ubv * ny;
    const double fhb = l * (cab[0] - cbb[0]);
    const double fxb = l * (cab[1] - cbb[1]);
    const double fyb = l * (cab[2] - cbb[2]);
    const double pab = l * (cab[1] * nx + cab[2] * ny);
    const double pbb = -l * (cbb[1] * nx + cbb[2] * ny);
    const double fqb = fxb * nx + fyb * ny, fwb = -fxb * ny + fyb * nx;
    double hsab, qab, wab, hsbb, qbb, wbb;
    hllc_normal_vjp(g, hsa, qa, wa, hsb, qb, wb, fhb, fqb, fwb, hsab, qab, wab, hsbb, qbb, wbb);
    hsab -= pab * g * hsa;
    hsbb -= pbb * g * hsb;
    // the reconstructed depths' cotangents where h* = h - (z* - z) is active; all by value
    // selects (a store through a chosen reference would keep the outputs in memory)
    const double ta = act_a ? hsab : 0.0, tb = act_b ? hsbb : 0.0;
    ua_out = {pab * g * ha + ta, 0.0, 0.0};
    ub_out = {pbb * g * hb + tb, 0.0, 0.0};
    const double zsb = -ta - tb;
    // max(za, zb) at a tie: half to each side (the convention of the tangent model too)
    za_out = ta + (za > zb ? zsb : (zb > za ? 0.0 : 0.5 * zsb));
    zb_out = tb + (zb > za ? zsb : (za > zb ? 0.0 : 0.5 * zsb));
    vel_vjp(ha, hua, hva, hd, qab * nx - wab * ny, qab * ny + wab * nx, ua_out);
    vel_vjp(hb, hub, hvb, hd, qbb * nx - wbb * ny, qbb * ny + wbb * nx, ub_out);
}

// Reflective wall: cotangent of the cell from that of its contribution.
__device__ void wall_vjp(double g, double hd, double h, double hu, double hv, double nx,
                         double ny, double l, const double *cb, Vjp3 &out)
{
    const double u = vel(h, hu, hd), v = vel(h, hv, hd);
    const double q = u * nx + v * ny, w = v * nx - u * ny;
    const double hs = h > hd ? h : 0.0;
    const double fhb = l * cb[0], fxb = l * cb[1], fyb = l * cb[2];
    const double pb = l * (cb[1] * nx + cb[2] * ny);
    const double fqb = fxb * nx + fyb * ny, fwb = -fxb * ny + fyb * nx;
    double hlb, qlb, wlb, hrb, qrb, wrb;
    hllc_normal_vjp(g, hs, q, w, hs, -q, w, fhb, fqb, fwb, hlb, qlb, wlb, hrb, qrb, wrb);
    const double qb = qlb - qrb, wb = wlb + wrb;
    double hsb = hlb + hrb - pb * g * hs;
    out = {pb * g * h, 0.0, 0.0};
    if (h > hd) out.h += hsb;
    vel_vjp(h, hu, hv, hd, qb * nx - wb * ny, qb * ny + wb * nx, out);
}

// Inflow segment: the flux depends on the cell only through h_b = max(h, h_c).
__device__ void inflow_vjp(double g, double q_in, double h, double nx, double ny, double l,
                           const double *cb, Vjp3 &out)
{
    const double hc = cbrt_(div_nr(q_in * q_in, g));
    out = {0.0, 0.0, 0.0};
    if (h >= hc) {
        const double momb = l * (cb[1] * nx + cb[2] * ny);
        out.h = momb * (-div_nr(q_in * q_in, h * h) + g * h);
    }
}

struct AdjArgs {
    int64_t T;
    const int32_t *nbr;
    const int32_t *c2n;
    const double2 *xy;
    const double *z, *n, *area;
    const double *h, *hu, *hv;          // U^n
    const double *sh, *shu, *shv;       // U*^n before the clamp
    const double *lh, *lhu, *lhv;       // lambda^{n+1}
    double *lo, *lou, *lov;             // lambda^n
    double *mh, *mhu, *mhv;             // mu (per-cell kernels)
    double *gn, *gz;
    const double *dt_seq;
    int64_t step;
    double g, hd;
    double q[SWE_MAX_INFLOW];
};

// What the adjoint step reads of one cell: U^n, bed, U* before the clamp, lambda^{n+1},
// roughness and area.
struct CellIn {
    double h, hu, hv, z, sh, shu, shv, lh, lhu, lhv, n, area;
};

__device__ __forceinline__ CellIn load_cell(const AdjArgs &a, int64_t c)
{
    return {a.h[c],  a.hu[c],  a.hv[c],  a.z[c],  a.sh[c], a.shu[c],
            a.shv[c], a.lh[c], a.lhu[c], a.lhv[c], a.n[c],  a.area[c]};
}

// mu = (dU^{n+1}/dU*)^T lambda^{n+1} of a cell, and the roughness gradient's share
// (dU^{n+1}/dn_i)^T lambda^{n+1}; returns whether the cell is wet (the share exists).
__device__ __forceinline__ bool friction_vjp(double g, double hd, const CellIn &ci, double dt,
                                             Vjp3 &mu, double &gn)
{
    const double hraw = ci.sh, hus = ci.shu, hvs = ci.shv;
    const bool clamped = hraw < 0.0;
    const double hs = clamped ? 0.0 : hraw;
    const double lh = ci.lh, lhu = ci.lhu, lhv = ci.lhv;
    double mh = lh, mhu = 0.0, mhv = 0.0;
    gn = 0.0;
    if (hs > hd) {
        const double nm = ci.n;
        const double mag = sqrt_nr(hus * hus + hvs * hvs);
        const double c = cbrt_(hs);
        const double P = hs * hs * c;
        const double K = dt * g * nm * nm;
        const double rP = rcp_nr(P);   // every quotient by P as a product (within 1.5 ulp)
        const double D = 1.0 + (K * mag) * rP;
        const double rD = rcp_nr(D);
        const double hun = hus * rD, hvn = hvs * rD;
        const double Db = -(lhu * hun + lhv * hvn) * rD;
        mhu = lhu * rD;
        mhv = lhv * rD;
        if (mag > 0.0) {
            const double magb = (Db * K) * rP;
            const double rm = rcp_nr(mag);
            mhu += magb * hus * rm;
            mhv += magb * hvs * rm;
        }
        const double Pb = -((Db * K * mag) * rP) * rP;
        mh += Pb * (7.0 / 3.0) * hs * c;
        gn = ((Db * mag) * rP) * 2.0 * dt * g * nm;
    }
    if (clamped) mh = 0.0;
    mu = {mh, mhu, mhv};
    return hs > hd;
}

// mu of every cell into a.mh (the per-cell flux adjoint reads it); roughness gradient.
__global__ __launch_bounds__(256) void friction_adjoint_kernel(AdjArgs a)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= a.T) return;
    Vjp3 mu;
    double gn;
    if (friction_vjp(a.g, a.hd, load_cell(a, i), a.dt_seq[a.step], mu, gn)) a.gn[i] += gn;
    a.mh[i] = mu.h;
    a.mhu[i] = mu.hu;
    a.mhv[i] = mu.hv;
}

// lambda^n = mu + sum over the cell's edges of its share of the edge adjoints; bed gradient.
__global__ __launch_bounds__(256) void flux_adjoint_kernel(AdjArgs a)
{
    const int64_t T = a.T;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= T) return;
    const double dt = a.dt_seq[a.step], g = a.g, hd = a.hd;
    const double2 p[3] = {a.xy[a.c2n[i]], a.xy[a.c2n[T + i]], a.xy[a.c2n[2 * T + i]]};
    const double h = a.h[i], hu = a.hu[i], hv = a.hv[i], z = a.z[i];
    const double ri = dt * rcp_nr(a.area[i]);
    const double ci[3] = {-ri * a.mh[i], -ri * a.mhu[i], -ri * a.mhv[i]};
    double lh = a.mh[i], lhu = a.mhu[i], lhv = a.mhv[i], zb_sum = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double2 p0 = p[k], p1 = p[k == 2 ? 0 : k + 1];
        const double dx = p1.x - p0.x, dy = p1.y - p0.y;
        double nx, ny, l;
        edge_normal_nr(dx, dy, nx, ny, l);
        const int32_t j = a.nbr[k * T + i];
        Vjp3 u{0.0, 0.0, 0.0};
        if (j >= 0) {
            const double rj = dt * rcp_nr(a.area[j]);
            const double cj[3] = {-rj * a.mh[j], -rj * a.mhu[j], -rj * a.mhv[j]};
            Vjp3 uj;
            double zi_b, zj_b;
            interface_vjp(g, hd, h, hu, hv, z, a.h[j], a.hu[j], a.hv[j], a.z[j], nx, ny, l, ci, cj,
                          u, zi_b, uj, zj_b);
            zb_sum += zi_b;
        } else if (j == SWE_WALL) {
            wall_vjp(g, hd, h, hu, hv, nx, ny, l, ci, u);
        } else {
            inflow_vjp(g, a.q[-2 - j], h, nx, ny, l, ci, u);
        }
        lh += u.h;
        lhu += u.hu;
        lhv += u.hv;
    }
    a.lo[i] = lh;
    a.lou[i] = lhu;
    a.lov[i] = lhv;
    a.gz[i] += zb_sum;
}

// Tile lists of the mesh (as the tiled step uses them).
struct AdjTiles {
    const int32_t *halo_off, *halo, *edge_off;
    const uint32_t *edges;
    const uint16_t *slot;
    const double2 *edge_vec;
    int32_t n_tiles, max_halo, max_edges, pad;
};

// LDS of the tiled flux adjoint: 7 words per staged cell (h, hu, hv, z and the cotangent
// -dt/A mu of its contribution), 8 per edge-list entry (both sides' cotangents and bed terms).
// Tiles of TB cells with at most 2 TB entries use a shared layout: [8 rows of TB for entries
// 0..TB-1 | staged cells], the later entries written in 8 rows of TB over the staged cells
// once every interface has been differentiated; others [cells | 8 rows of M].
inline bool tile_adj_shared(int64_t tb, int64_t max_edges) { return max_edges <= 2 * tb; }

inline size_t tile_adj_lds_bytes(int64_t tb, int64_t max_halo, int64_t max_edges)
{
    const size_t cells = 7 * static_cast<size_t>(tb + max_halo);
    if (tile_adj_shared(tb, max_edges))
        return 8 * (8 * static_cast<size_t>(tb) + std::max(cells, 8 * static_cast<size_t>(tb)));
    return 8 * (cells + 8 * static_cast<size_t>(max_edges));
}

// The flux adjoint of flux_adjoint_kernel, tiled: each interface of a tile's edge list is
// differentiated once (both sides' cotangents at once) into LDS, then each cell gathers its
// three shares in local-edge order.  Same quantities as the per-cell kernel, up to rounding.
// Work-items take edge-list and halo positions as the tiled step does (the wave with one
// round of interfaces stages the halo; which wave it is turns with the tile).  Four waves per
// SIMD: 128 VGPRs, and the shared layout's LDS.
template <int TB, bool Shared>
__global__ __launch_bounds__(TB, 4) void tile_flux_adjoint_kernel(AdjArgs a, AdjTiles t)
{
    const int tile = blockIdx.x;
    if (tile >= t.n_tiles) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *const lds = reinterpret_cast<double *>(smem);
    const int ns = TB + t.max_halo;
    // staged cells at cbase; edge-list entry q of row j at ebase + j estride + q (+ bshift from
    // entry TB on)
    const int cbase = Shared ? 8 * TB : 0;
    const int ebase = Shared ? 0 : 7 * ns;
    const int estride = Shared ? TB : t.max_edges;
    const int bshift = Shared ? 7 * TB : 0;
    double *s_h = lds + cbase;
    double *s_hu = s_h + ns, *s_hv = s_hu + ns, *s_z = s_hv + ns;
    double *s_c0 = s_z + ns, *s_c1 = s_c0 + ns, *s_c2 = s_c1 + ns;
    const int64_t T = a.T, s0 = static_cast<int64_t>(tile) * TB;
    const int tid = threadIdx.x;
    const int pt = (tid + 64 * (tile % (TB / 64))) & (TB - 1);
    const int ph = TB - 1 - pt;
    const int64_t i = s0 + tid;
    const bool mine = i < T;
    const double dt = a.dt_seq[a.step], g = a.g, hd = a.hd;
    // the friction adjoint of every staged cell (halo cells' redone here rather than read):
    // mu and the contribution cotangent -dt/A mu; a tile cell keeps its mu and adds its
    // roughness gradient
    Vjp3 mu_own{0.0, 0.0, 0.0};
    double gn_own = 0.0;
    bool wet_own = false;
    auto stage = [&](int q, const CellIn &ci, bool own) {
        s_h[q] = ci.h;
        s_hu[q] = ci.hu;
        s_hv[q] = ci.hv;
        s_z[q] = ci.z;
        Vjp3 mu;
        double gn;
        const bool wet = friction_vjp(g, hd, ci, dt, mu, gn);
        if (own) {
            mu_own = mu;
            gn_own = gn;
            wet_own = wet;
        }
        const double r = dt * rcp_nr(ci.area);
        s_c0[q] = -r * mu.h;
        s_c1[q] = -r * mu.hu;
        s_c2[q] = -r * mu.hv;
    };
    // Global loads up front: the work-item's first halo index, then together that halo cell's
    // inputs, its own cell's and the first round's edge-list entry, so that one wait on the
    // index precedes one wait on all of them.
    const int hb = t.halo_off[tile], he = t.halo_off[tile + 1];
    const int j0 = hb + ph;
    const int32_t c0 = j0 < he ? t.halo[j0] : -1;
    const int eb = t.edge_off[tile], ee = t.edge_off[tile + 1];
    CellIn own{}, hal{};
    if (c0 >= 0) hal = load_cell(a, c0);
    if (mine) own = load_cell(a, i);
    uint32_t w = 0u;
    double2 d = {0.0, 0.0};
    if (eb + pt < ee) {
        w = t.edges[eb + pt];
        d = t.edge_vec[eb + pt];
    }
    if (mine) stage(tid, own, true);
    if (c0 >= 0) stage(TB + (j0 - hb), hal, false);
    for (int j = j0 + TB; j < he; j += TB) stage(TB + (j - hb), load_cell(a, t.halo[j]), false);
    __syncthreads();

    // side a's (h, hu, hv) cotangent and bed term, then side b's for interfaces inside the tile
    struct EdgeAdj {
        double v[8];
    };
    auto diff = [&](uint32_t w, double2 d, EdgeAdj &o) {
        const int ca = static_cast<int>(w & kEdgeA);
        const int cb = static_cast<int16_t>(w >> 16);
        const double dx = d.x, dy = d.y;
        double nx, ny, l;
        edge_normal_nr(dx, dy, nx, ny, l);
        const double ci[3] = {s_c0[ca], s_c1[ca], s_c2[ca]};
        Vjp3 u{0.0, 0.0, 0.0};
        double za_b = 0.0;
        bool inner = false;
        if (cb >= 0) {
            const double cj[3] = {s_c0[cb], s_c1[cb], s_c2[cb]};
            Vjp3 ub;
            double zb_b;
            interface_vjp(g, hd, s_h[ca], s_hu[ca], s_hv[ca], s_z[ca], s_h[cb], s_hu[cb],
                          s_hv[cb], s_z[cb], nx, ny, l, ci, cj, u, za_b, ub, zb_b);
            inner = cb < TB;
            o.v[4] = ub.h;
            o.v[5] = ub.hu;
            o.v[6] = ub.hv;
            o.v[7] = zb_b;
        } else if (cb == SWE_WALL) {
            wall_vjp(g, hd, s_h[ca], s_hu[ca], s_hv[ca], nx, ny, l, ci, u);
        } else {
            inflow_vjp(g, a.q[-2 - cb], s_h[ca], nx, ny, l, ci, u);
        }
        o.v[0] = u.h;
        o.v[1] = u.hu;
        o.v[2] = u.hv;
        o.v[3] = za_b;
        return inner;
    };
    auto put = [&](int q, const EdgeAdj &o, bool inner) {
        double *ed = lds + ebase + q + (q >= TB ? bshift : 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) ed[r * estride] = o.v[r];
        if (inner) {
#pragma unroll
            for (int r = 4; r < 8; ++r) ed[r * estride] = o.v[r];
        }
    };
    // one call site of diff: in the shared layout (two rounds at most) the second round's
    // result waits for the barrier after which the staged cells may be overwritten; each
    // round's successor entry is loaded before the round is differentiated
    EdgeAdj o;
    bool inner = false;
    int held = -1;
    for (int q = pt; eb + q < ee; q += TB) {
        uint32_t wn = 0u;
        double2 dn = {0.0, 0.0};
        if (eb + q + TB < ee) {
            wn = t.edges[eb + q + TB];
            dn = t.edge_vec[eb + q + TB];
        }
        inner = diff(w, d, o);
        if (Shared && q >= TB) {
            held = q;
            break;
        }
        put(q, o, inner);
        w = wn;
        d = dn;
    }
    if constexpr (Shared) {
        __syncthreads();   // every read of the staged cells is done
        if (held >= 0) put(held, o, inner);
    }
    // the cell's three edge-list slots, its roughness and bed gradients so far, loaded before
    // the wait for the other work-items' interfaces
    uint32_t sl[3] = {0u, 0u, 0u};
    double gn0 = 0.0, gz0 = 0.0;
    if (mine) {
#pragma unroll
        for (int k = 0; k < 3; ++k) sl[k] = t.slot[k * T + i];
        if (wet_own) gn0 = a.gn[i];
        gz0 = a.gz[i];
    }
    __syncthreads();
    if (!mine) return;
    double lh = mu_own.h, lhu = mu_own.hu, lhv = mu_own.hv, zb_sum = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int q = static_cast<int>(sl[k] & 0x7fffu);
        const double *ed = lds + ebase + q + (q >= TB ? bshift : 0) + ((sl[k] & 0x8000u) ? 4 * estride : 0);
        lh += ed[0];
        lhu += ed[estride];
        lhv += ed[2 * estride];
        zb_sum += ed[3 * estride];
    }
    a.lo[i] = lh;
    a.lou[i] = lhu;
    a.lov[i] = lhv;
    if (wet_own) a.gn[i] = gn0 + gn_own;
    a.gz[i] = gz0 + zb_sum;
}

// The tiled flux adjoint of a tile size and layout.
using AdjKernel = void (*)(AdjArgs, AdjTiles);

AdjKernel tile_adj_kernel(int tb, bool shared)
{
    switch (tb) {
    case 64: return shared ? tile_flux_adjoint_kernel<64, true> : tile_flux_adjoint_kernel<64, false>;
    case 128: return shared ? tile_flux_adjoint_kernel<128, true> : tile_flux_adjoint_kernel<128, false>;
    case 512: return shared ? tile_flux_adjoint_kernel<512, true> : tile_flux_adjoint_kernel<512, false>;
    default: return shared ? tile_flux_adjoint_kernel<256, true> : tile_flux_adjoint_kernel<256, false>;
    }
}

// Misfit at an observation (one workgroup of 64 work-items, a chunk of gauges at a time): its
// share of the loss, sum (h_g - obs_g)^2 in gauge order, into *part, and the adjoint's
// 2 (h_g - obs_g) added at the gauges (distinct cells) of lam.
__global__ void misfit_kernel(const double *h, const int32_t *gauges, int ng, const double *obs,
                              double *part, double *lam)
{
    __shared__ double sq[64];
    double acc = 0.0;
    for (int base = 0; base < ng; base += 64) {
        const int q = base + static_cast<int>(threadIdx.x);
        if (q < ng) {
            const double r = h[gauges[q]] - obs[q];
            sq[threadIdx.x] = r * r;
            lam[gauges[q]] += 2.0 * r;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = 0; k < 64 && base + k < ng; ++k) acc += sq[k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *part = acc;
}

// The loss: the observations' shares added in observation order.
__global__ void loss_sum_kernel(const double *part, int64_t n_obs, double *loss)
{
    double j = 0.0;
    for (int64_t m = 0; m < n_obs; ++m) j += part[m];
    *loss = j;
}

__global__ void fill_kernel(double *p, int64_t n, double v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Workspace layout of swe_adjoint (all double unless noted).
struct AdjLayout {
    int64_t T, n_ckpt, K;
    size_t ckpt, seg, segstar, lam, lam2, mu, loss, ctrl, work, total;
};

// K == 1 (every state stored): no recompute segment; U* of every step.
AdjLayout adj_layout(int64_t T, int64_t n_steps, int64_t K)
{
    AdjLayout L;
    L.T = T;
    L.K = K;
    L.n_ckpt = (n_steps + K - 1) / K + 1;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off = 0;
    const size_t st = 3 * static_cast<size_t>(T) * 8;
    L.ckpt = off; off += al(st * L.n_ckpt);
    L.seg = off; off += K == 1 ? 0 : al(st * (K + 1));
    L.segstar = off; off += al(st * (K == 1 ? n_steps : K));
    L.lam = off; off += al(st);
    L.lam2 = off; off += al(st);
    L.mu = off; off += al(st);
    L.loss = off; off += al(8 * (static_cast<size_t>(n_steps) + 1));   // J, then each observation's share
    L.ctrl = off; off += al(SWE_CTRL_BYTES);
    L.work = off; off += al(static_cast<size_t>(workspace_bytes(T)));
    L.total = off;
    return L;
}

}  // namespace
}  // namespace swe

using namespace swe;

namespace {

// Whether the tiled flux adjoint's dynamic LDS limit has been raised on a device (per layout:
// 0 not yet, 1 raised, -1 refused).
int g_adj_lds[64][4][2] = {};   // device, tile size (64 << index), layout
std::mutex g_adj_lds_mu;

int32_t afail(int32_t code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int32_t ahip(hipError_t e, const char *where)
{
    if (e == hipSuccess) return SWE_OK;
    return afail(SWE_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Events around the two passes of this thread's last swe_adjoint call.
struct Timing {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool recorded = false;
    hipError_t create()
    {
        for (hipEvent_t &e : ev)
            if (hipError_t r = hipEventCreate(&e)) return r;
        return hipSuccess;
    }
    void reset()
    {
        for (hipEvent_t &e : ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        recorded = false;
    }
    // no destructor: the runtime may be gone when thread-local objects die at exit
};
thread_local Timing g_timing;

}  // namespace

extern "C" {

int32_t swe_adjoint_workspace_bytes(const swe_mesh *mesh, int64_t n_steps, int32_t ckpt_every,
                                    int64_t *bytes)
{
    if (!mesh || !bytes || n_steps < 1 || ckpt_every < 1)
        return afail(SWE_EINVAL, "swe_adjoint_workspace_bytes: bad argument");
    *bytes = static_cast<int64_t>(adj_layout(mesh->info.n_cells, n_steps, ckpt_every).total);
    return SWE_OK;
}

int32_t swe_adjoint(const swe_mesh *mesh, const swe_dev_mesh *dm, const swe_params *p,
                    const swe_state *s, int64_t n_steps, const double *dt_seq,
                    const swe_loss *loss, int32_t ckpt_every, swe_grads *out, double *loss_out,
                    void *ws, int64_t ws_bytes, void *stream)
{
    const char *W = "swe_adjoint";
    if (!mesh || !dm || !p || !s || !dt_seq || !loss || !out || !ws)
        return afail(SWE_EINVAL, "swe_adjoint: null argument");
    if (p->dtype != SWE_F64) return afail(SWE_EUNSUPPORTED, "swe_adjoint: FP64 only");
    if (n_steps < 1 || ckpt_every < 1 || loss->every < 1 || loss->n_gauges < 0 ||
        (loss->n_gauges > 0 && (!loss->gauges || !loss->obs)))
        return afail(SWE_EINVAL, "swe_adjoint: bad steps, checkpoint interval or loss");
    if (!out->dn || !out->dz || !out->dh || !out->dhu || !out->dhv)
        return afail(SWE_EINVAL, "swe_adjoint: null gradient array");
    if (!(p->g > 0.0) || !(p->h_dry >= 0.0) || p->n_inflow < 0 || p->n_inflow > SWE_MAX_INFLOW ||
        (p->n_inflow > 0 && !p->inflow_q) || mesh->info.n_inflow_segments > p->n_inflow)
        return afail(SWE_EINVAL, "swe_adjoint: bad parameters");
    if (dm->n_cells != mesh->info.n_cells || !dm->nbr || !dm->c2n || !dm->xy || !dm->cell_geo)
        return afail(SWE_EINVAL, "swe_adjoint: bad device mesh");
    if (mesh->info.n_owned != mesh->info.n_cells || (p->flags & SWE_SHARD))
        return afail(SWE_EUNSUPPORTED, "swe_adjoint: not for shards");
    if (!s->h[s->cur] || !s->hu[s->cur] || !s->hv[s->cur] || !s->z || !s->n)
        return afail(SWE_EINVAL, "swe_adjoint: null state array");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return afail(SWE_EINVAL, "swe_adjoint: ws not 256-byte aligned");
    const int64_t T = mesh->info.n_cells, K = ckpt_every;
    const AdjLayout L = adj_layout(T, n_steps, K);
    if (ws_bytes < static_cast<int64_t>(L.total))
        return afail(SWE_EINVAL, "swe_adjoint: workspace needs " + std::to_string(L.total) + " bytes");
    const TileLayout *tl = nullptr;   // the step kernel of the forward and recompute passes
    int remap = 1;
    if (int32_t rc = choose_variant(mesh, dm, p, &tl, &remap, W)) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Timing &tm = g_timing;
    tm.reset();
    if (int32_t rc = ahip(tm.create(), W)) return rc;
    if (int32_t rc = ahip(hipEventRecord(tm.ev[0], st), W)) return rc;
    char *base = static_cast<char *>(ws);
    auto D = [&](size_t off) { return reinterpret_cast<double *>(base + off); };
    const size_t S = static_cast<size_t>(T);
    auto ck = [&](int64_t c, int f) { return D(L.ckpt) + (static_cast<size_t>(c) * 3 + f) * S; };
    auto sg = [&](int64_t n, int f) { return D(L.seg) + (static_cast<size_t>(n) * 3 + f) * S; };
    auto ss = [&](int64_t n, int f) { return D(L.segstar) + (static_cast<size_t>(n) * 3 + f) * S; };
    // lambda alternates between two buffers: a step reads lambda^{n+1} from one and writes
    // lambda^n to the other (neighbouring tiles still read the former)
    double *lamb[2] = {D(L.lam), D(L.lam2)};
    int lcur = 0;
    double *mu = D(L.mu), *lossd = D(L.loss), *obs_part = lossd + 1;
    const unsigned blocks = static_cast<unsigned>((T + 255) / 256);

    StepConfig cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.n_cells = T;
    cfg.n_owned = T;
    cfg.fast = (p->flags & SWE_EXACT) ? 0 : 1;
    cfg.tile = mesh->info.tile_cells;
    cfg.g = p->g;
    cfg.courant = p->courant > 0.0 && p->courant <= 1.0 ? p->courant : 0.7;
    cfg.h_dry = p->h_dry;
    cfg.n_inflow = p->n_inflow;
    for (int k = 0; k < p->n_inflow; ++k) cfg.inflow_q[k] = p->inflow_q[k];

    // a private state for the forward and recompute passes
    swe_state ps;
    memset(&ps, 0, sizeof(ps));
    ps.z = s->z;
    ps.n = s->n;
    ps.ctrl = base + L.ctrl;
    ps.work = base + L.work;
    auto view = [&](double *h0, double *hu0, double *hv0, double *h1, double *hu1, double *hv1) {
        swe_state v = ps;
        v.h[0] = h0; v.hu[0] = hu0; v.hv[0] = hv0;
        v.h[1] = h1; v.hu[1] = hu1; v.hv[1] = hv1;
        v.cur = 0;
        return v;
    };
    const size_t bytes3 = S * 8;
    auto copy3 = [&](double *dh, double *dhu, double *dhv, const void *sh, const void *shu,
                     const void *shv) -> int32_t {
        if (int32_t rc = ahip(hipMemcpyAsync(dh, sh, bytes3, hipMemcpyDeviceToDevice, st), W)) return rc;
        if (int32_t rc = ahip(hipMemcpyAsync(dhu, shu, bytes3, hipMemcpyDeviceToDevice, st), W)) return rc;
        return ahip(hipMemcpyAsync(dhv, shv, bytes3, hipMemcpyDeviceToDevice, st), W);
    };

    // forward pass: checkpoints (the loss is formed in the reverse pass, whose misfit launches
    // have every observed state at hand)
    if (int32_t rc = copy3(ck(0, 0), ck(0, 1), ck(0, 2), s->h[s->cur], s->hu[s->cur], s->hv[s->cur])) return rc;
    const bool record = K == 1;
    if (record) {
        // step n reads stored state n and writes state n + 1 and its U* in place
        for (int64_t nstep = 0; nstep < n_steps; ++nstep) {
            swe_state v = view(ck(nstep, 0), ck(nstep, 1), ck(nstep, 2), ck(nstep + 1, 0),
                               ck(nstep + 1, 1), ck(nstep + 1, 2));
            double *ustar[3] = {ss(nstep, 0), ss(nstep, 1), ss(nstep, 2)};
            if (int32_t rc = ahip(static_cast<hipError_t>(launch_step(SWE_F64, *dm, cfg, v, 0, dt_seq,
                                                                      n_steps, st, tl, nullptr, remap,
                                                                      ustar, dt_seq + nstep)), W))
                return rc;
        }
    } else {
    if (int32_t rc = copy3(sg(0, 0), sg(0, 1), sg(0, 2), ck(0, 0), ck(0, 1), ck(0, 2))) return rc;
    // the steps replay dt_seq directly: no control block, no dt reduction.  Segment slots 0
    // and 1 serve as ping-pong until the last segment, whose states and U* the pass stores
    // as the reverse pass's recompute would (so that segment is not recomputed).
    const int64_t s_last = ((n_steps + K - 1) / K - 1) * K;
    swe_state fw = view(sg(0, 0), sg(0, 1), sg(0, 2), sg(1, 0), sg(1, 1), sg(1, 2));
    int cur = 0;
    for (int64_t nstep = 0; nstep < n_steps; ++nstep) {
        const int64_t q = nstep - s_last;
        if (q == 0 && cur != 0)   // the last segment starts in slot 0
            if (int32_t rc = copy3(sg(0, 0), sg(0, 1), sg(0, 2), sg(1, 0), sg(1, 1), sg(1, 2))) return rc;
        double *un[3];
        if (q < 0) {
            if (int32_t rc = ahip(static_cast<hipError_t>(launch_step(SWE_F64, *dm, cfg, fw, cur, dt_seq,
                                                                      n_steps, st, tl, nullptr, remap,
                                                                      nullptr, dt_seq + nstep)), W))
                return rc;
            cur ^= 1;
            for (int f = 0; f < 3; ++f) un[f] = sg(cur, f);
        } else {
            swe_state v = view(sg(q, 0), sg(q, 1), sg(q, 2), sg(q + 1, 0), sg(q + 1, 1), sg(q + 1, 2));
            double *ustar[3] = {ss(q, 0), ss(q, 1), ss(q, 2)};
            if (int32_t rc = ahip(static_cast<hipError_t>(launch_step(SWE_F64, *dm, cfg, v, 0, dt_seq,
                                                                      n_steps, st, tl, nullptr, remap,
                                                                      ustar, dt_seq + nstep)), W))
                return rc;
            for (int f = 0; f < 3; ++f) un[f] = sg(q + 1, f);
        }
        if ((nstep + 1) % K == 0) {
            const int64_t c = (nstep + 1) / K;
            if (int32_t rc = copy3(ck(c, 0), ck(c, 1), ck(c, 2), un[0], un[1], un[2])) return rc;
        }
    }
    }

    // reverse pass
    if (int32_t rc = ahip(hipEventRecord(tm.ev[1], st), W)) return rc;
    AdjArgs a;
    memset(&a, 0, sizeof(a));
    a.T = T;
    a.nbr = dm->nbr;
    a.c2n = dm->c2n;
    a.xy = reinterpret_cast<const double2 *>(dm->xy);
    a.z = static_cast<const double *>(s->z);
    a.n = static_cast<const double *>(s->n);
    a.area = dm->cell_geo;   // the cell areas A_i, first T entries
    a.mh = mu; a.mhu = mu + S; a.mhv = mu + 2 * S;
    a.gn = out->dn;
    a.gz = out->dz;
    a.dt_seq = dt_seq;
    a.g = p->g;
    a.hd = p->h_dry;
    for (int k = 0; k < p->n_inflow; ++k) a.q[k] = p->inflow_q[k];
    // the tiled flux adjoint where the step is tiled and its LDS fits a workgroup
    AdjTiles at;
    memset(&at, 0, sizeof(at));
    size_t adj_lds = 0;
    bool adj_shared = false;
    const int adj_tb = tl ? tl->tile : 0;
    if (tl && SWE_TILE_ADJOINT) {
        const size_t need = tile_adj_lds_bytes(adj_tb, tl->max_halo, tl->max_edges);
        adj_shared = tile_adj_shared(adj_tb, tl->max_edges);
        int dev = 0, max_lds = 65536;
        if (int32_t rc = ahip(hipGetDevice(&dev), W)) return rc;
        if (int32_t rc = ahip(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), W))
            return rc;
        bool fits = need <= static_cast<size_t>(max_lds);
        if (fits && need > 65536) {   // beyond the default dynamic LDS limit
            // raised once per device and layout to the device's limit (the kernel has no static
            // LDS), so that calls on other meshes, from other threads too, never lower it
            fits = false;
            if (dev >= 0 && dev < 64) {
                std::lock_guard<std::mutex> lk(g_adj_lds_mu);
                const int ti = adj_tb == 64 ? 0 : adj_tb == 128 ? 1 : adj_tb == 256 ? 2 : 3;
                int &state = g_adj_lds[dev][ti][adj_shared ? 1 : 0];
                if (state == 0) {
                    const void *k = reinterpret_cast<const void *>(tile_adj_kernel(adj_tb, adj_shared));
                    state = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds) ==
                                    hipSuccess
                                ? 1
                                : -1;
                    if (state < 0) (void)hipGetLastError();   // the per-cell kernel then; clear it
                }
                fits = state > 0;
            }
        }
        if (fits) {
            adj_lds = need;
            at.halo_off = dm->halo_off;
            at.halo = dm->halo;
            at.edge_off = dm->edge_off;
            at.edges = dm->edges;
            at.slot = dm->slot;
            at.edge_vec = reinterpret_cast<const double2 *>(dm->edge_vec);
            at.n_tiles = static_cast<int32_t>(tl->n_tiles);
            at.max_halo = tl->max_halo;
            at.max_edges = tl->max_edges;
        }
    }
    fill_kernel<<<(3 * S + 255) / 256, 256, 0, st>>>(lamb[0], 3 * T, 0.0);
    fill_kernel<<<blocks, 256, 0, st>>>(out->dn, T, 0.0);
    fill_kernel<<<blocks, 256, 0, st>>>(out->dz, T, 0.0);
    // one adjoint step: lambda^{n+1} (plus the misfit at n + 1) -> lambda^n, from the state
    // U^n and U* of step n
    // (the tiled kernel does the friction adjoint of the cells it stages itself)
    auto adjoint_step = [&](int64_t nstep, const double *const *un, const double *const *us1,
                            const double *const *ustar) {
        double *lin = lamb[lcur], *lout = lamb[lcur ^ 1];
        if ((nstep + 1) % loss->every == 0 && loss->n_gauges > 0) {
            const int64_t m = (nstep + 1) / loss->every - 1;   // the observation
            misfit_kernel<<<1, 64, 0, st>>>(us1[0], loss->gauges, loss->n_gauges,
                                            loss->obs + m * loss->n_gauges, obs_part + m, lin);
        }
        a.step = nstep;
        a.sh = ustar[0]; a.shu = ustar[1]; a.shv = ustar[2];
        a.lh = lin; a.lhu = lin + S; a.lhv = lin + 2 * S;
        a.lo = lout; a.lou = lout + S; a.lov = lout + 2 * S;
        a.h = un[0]; a.hu = un[1]; a.hv = un[2];
        if (adj_lds) {
            tile_adj_kernel(adj_tb, adj_shared)
                <<<dim3(static_cast<unsigned>(at.n_tiles)), dim3(adj_tb), adj_lds, st>>>(a, at);
        } else {
            friction_adjoint_kernel<<<blocks, 256, 0, st>>>(a);
            flux_adjoint_kernel<<<blocks, 256, 0, st>>>(a);
        }
        lcur ^= 1;
    };
    if (record) {
        for (int64_t nstep = n_steps - 1; nstep >= 0; --nstep) {
            const double *un[3] = {ck(nstep, 0), ck(nstep, 1), ck(nstep, 2)};
            const double *u1[3] = {ck(nstep + 1, 0), ck(nstep + 1, 1), ck(nstep + 1, 2)};
            const double *us[3] = {ss(nstep, 0), ss(nstep, 1), ss(nstep, 2)};
            adjoint_step(nstep, un, u1, us);
        }
        if (int32_t rc = ahip(hipGetLastError(), W)) return rc;
    }
    const int64_t n_seg = record ? 0 : (n_steps + K - 1) / K;
    for (int64_t sgi = n_seg - 1; sgi >= 0; --sgi) {
        const int64_t s0 = sgi * K, s1 = std::min(n_steps, s0 + K);
        // the last segment is in the slots already (forward pass)
        if (sgi < n_seg - 1)
            if (int32_t rc = copy3(sg(0, 0), sg(0, 1), sg(0, 2), ck(sgi, 0), ck(sgi, 1), ck(sgi, 2))) return rc;
        for (int64_t nstep = sgi < n_seg - 1 ? s0 : s1; nstep < s1; ++nstep) {
            const int64_t q = nstep - s0;
            swe_state v = view(sg(q, 0), sg(q, 1), sg(q, 2), sg(q + 1, 0), sg(q + 1, 1), sg(q + 1, 2));
            double *ustar[3] = {ss(q, 0), ss(q, 1), ss(q, 2)};
            if (int32_t rc = ahip(static_cast<hipError_t>(launch_step(SWE_F64, *dm, cfg, v, 0, dt_seq + s0,
                                                                      s1 - s0, st, tl, nullptr,
                                                                      remap, ustar, dt_seq + nstep)), W))
                return rc;
        }
        for (int64_t nstep = s1 - 1; nstep >= s0; --nstep) {
            const int64_t q = nstep - s0;
            const double *un[3] = {sg(q, 0), sg(q, 1), sg(q, 2)};
            const double *u1[3] = {sg(q + 1, 0), sg(q + 1, 1), sg(q + 1, 2)};
            const double *us[3] = {ss(q, 0), ss(q, 1), ss(q, 2)};
            adjoint_step(nstep, un, u1, us);
        }
        if (int32_t rc = ahip(hipGetLastError(), W)) return rc;
    }
    if (loss->n_gauges > 0)
        loss_sum_kernel<<<1, 1, 0, st>>>(obs_part, n_steps / loss->every, lossd);
    else
        fill_kernel<<<1, 256, 0, st>>>(lossd, 1, 0.0);
    double *lam = lamb[lcur];   // lambda^0
    if (int32_t rc = copy3(out->dh, out->dhu, out->dhv, lam, lam + S, lam + 2 * S)) return rc;
    if (int32_t rc = ahip(hipEventRecord(tm.ev[2], st), W)) return rc;
    tm.recorded = true;
    if (loss_out) {
        if (int32_t rc = ahip(hipMemcpyAsync(loss_out, lossd, 8, hipMemcpyDeviceToHost, st), W)) return rc;
        if (int32_t rc = ahip(hipStreamSynchronize(st), W)) return rc;
    }
    return ahip(hipGetLastError(), W);
}

int32_t swe_adjoint_timings(double *forward_ms, double *reverse_ms)
{
    if (!forward_ms || !reverse_ms) return afail(SWE_EINVAL, "swe_adjoint_timings: null argument");
    Timing &tm = g_timing;
    if (!tm.recorded) return afail(SWE_EINVAL, "swe_adjoint_timings: no completed swe_adjoint call");
    const char *W = "swe_adjoint_timings";
    if (int32_t rc = ahip(hipEventSynchronize(tm.ev[2]), W)) return rc;
    float f = 0.0f, r = 0.0f;
    if (int32_t rc = ahip(hipEventElapsedTime(&f, tm.ev[0], tm.ev[1]), W)) return rc;
    if (int32_t rc = ahip(hipEventElapsedTime(&r, tm.ev[1], tm.ev[2]), W)) return rc;
    *forward_ms = f;
    *reverse_ms = r;
    return SWE_OK;
}

}  // extern "C"
