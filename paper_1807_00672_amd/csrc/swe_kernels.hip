// HIP kernels of libswe for gfx950: the tiled and the per-cell step, the dt reductions, the
// initial-dt pass, the shard helpers and the flux test hook.
//
// Cells are in Morton order.  The tiled step (the default) stages a tile of cells (64, 128, 256
// or 512, the mesh's tile size) and its halo in LDS and evaluates each interface of the tile
// once; the per-cell step has each cell
// gather its three neighbours and evaluate its three interface fluxes itself (section 2.2: HLLC
// with hydrostatic reconstruction).  Both accumulate a cell's contributions in local-edge
// order, apply the explicit Euler update of eq. 4, clamp negative depths, apply semi-implicit
// Manning friction and compute the cell's CFL bound for the next step.  The flux is written so
// that the two sides' evaluations of an interface are exact negatives of each other, so both
// kernels give the same bits and mass is conserved up to the rounding of the cell sums, with
// no atomics.
//
// Every product and sum is rounded on its own (the library is built with contraction off),
// in the order written here.  This file is compiled twice: into swe::exact with correctly
// rounded FP64 division and square root, and (swe_kernels_fast.hip) into swe::fast with their
// hardware-seeded Newton forms; FP32 is the same in both.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "swe_device_math.h"
#include "swe_internal.h"

#ifndef SWE_MATH_NS
#define SWE_MATH_NS exact
#endif

namespace swe {
namespace SWE_MATH_NS {
namespace {

constexpr double kInf = __builtin_huge_val();

// Minimum waves per SIMD the compiler must allow for (register budget) in the two step
// kernels; 1 leaves the choice to the compiler.  Six holds the FP64 tiled kernels to 80
// VGPRs (the correctly rounded one needs 81 unconstrained), which the shared LDS layout
// lets six tiles per CU use; FP32 needs fewer anyway.
#ifndef SWE_CELL_WAVES
#define SWE_CELL_WAVES 1
#endif
#ifndef SWE_TILE_WAVES
#define SWE_TILE_WAVES 6
#endif
#ifndef SWE_F32_FAST
#define SWE_F32_FAST 1
#endif
// 1: the workgroups of a single mesh's step merge their dt partials into one slot per
// kSlotTiles tiles with relaxed device-scope atomics (min of the bound's bits, clamp count,
// status bits), and one workgroup folds the slots after the step (dt_group_fold_kernel); 0:
// they write per-tile partials, which dt_fold_kernel folds over many workgroups.
#ifndef SWE_GROUP_ATOMIC
#define SWE_GROUP_ATOMIC 1
#endif
// Single-mesh steps of at most this many tiles finish their dt reduction themselves (the last
// workgroup to arrive folds the partials) instead of launching the fold kernel.  Each
// workgroup's release then writes back its XCD's L2, which costs more than the fold launch
// beyond a few hundred workgroups (measured: 10,000 cells 14.4 -> 12.4 us per step, 250,000
// cells 21.4 -> 40.4 us).
#ifndef SWE_FUSE_TILES
#define SWE_FUSE_TILES 128
#endif
// 1: the tiled kernel addresses arrays below 4 GiB by 32-bit byte offsets; 0: always 64-bit.
#ifndef SWE_OFF32
#define SWE_OFF32 1
#endif
// 1: tiles whose LDS limits occupancy write their second round of interface results over
// the states (tile_alias); 0: never.
#ifndef SWE_TILE_ALIAS
#define SWE_TILE_ALIAS 1
#endif
// Division and square root of the step.  FP64: the correctly rounded operations (the same
// results as the CPU oracle's), or with SWE_F64_FAST their Newton forms.  FP32: the hardware
// reciprocal and square root (about 1 ulp), a fraction of the instructions of the correctly
// rounded sequences.  All are odd in their sign arguments, so interface fluxes stay exact
// negatives of each other.
template <typename R>
__device__ __forceinline__ R div_(R a, R b)
{
    return a / b;
}
template <typename R>
__device__ __forceinline__ R sqrt_(R a)
{
    return sqrt(a);
}
#ifndef SWE_F64_FAST
#define SWE_F64_FAST 0
#endif
#if SWE_F64_FAST
// Newton forms of swe_device_math.h (within an ulp, odd in their sign arguments).
template <>
__device__ __forceinline__ double div_<double>(double a, double b)
{
    return div_nr(a, b);
}
template <>
__device__ __forceinline__ double sqrt_<double>(double a)
{
    return sqrt_nr(a);
}
#endif
#if SWE_F32_FAST
template <>
__device__ __forceinline__ float div_<float>(float a, float b)
{
    return a * __builtin_amdgcn_rcpf(b);
}
template <>
__device__ __forceinline__ float sqrt_<float>(float a)
{
    return __builtin_amdgcn_sqrtf(a);
}
#endif

// Fast forms (FP32, and FP64 outside SWE_EXACT): quotients by one divisor share its
// reciprocal; an edge's length and reciprocal length come from one reciprocal square root; the
// friction factor and the CFL bound are rearranged to one quotient each.  A velocity is the
// momentum times the depth's reciprocal (within 1.5 ulp), and so are a cell's dt/A, friction
// factor and CFL bound; the HLL fluxes and the unit normals, where cancellation would magnify
// that, refine each product by one residual step (quot,
// within an ulp, nearly always the correctly rounded quotient).  Every form is odd in the
// arguments whose sign a mirrored interface flips, so the two sides of an interface still give
// exact negatives.  SWE_EXACT keeps the plain definitions with correctly rounded division and
// square root (the oracle's bits).
template <typename R>
constexpr bool kFastForms = sizeof(R) == 4 || SWE_F64_FAST;

template <typename R>
__device__ __forceinline__ R rcp_(R b);
template <>
__device__ __forceinline__ double rcp_<double>(double b)
{
    return rcp_nr(b);
}
template <>
__device__ __forceinline__ float rcp_<float>(float b)
{
    return __builtin_amdgcn_rcpf(b);
}

// a / b from ir, the reciprocal of b: the product and, in FP64, one residual correction;
// odd in a, and in b with ir.
template <typename R>
__device__ __forceinline__ R quot(R a, R ir, R b)
{
    if constexpr (sizeof(R) == 8) {
        return quot_nr(a, ir, b);
    } else {
        return a * ir;   // as div_<float>
    }
}

// ------------------------------------------------------------------------ flux pieces

// Velocities of a cell: zero at or below the dry threshold.
template <typename R>
__device__ __forceinline__ void velocities(R h, R hu, R hv, R h_dry, R &u, R &v)
{
    if (h > h_dry) {
        if constexpr (kFastForms<R>) {
            const R ih = rcp_(h);
            u = hu * ih;
            v = hv * ih;
        } else {
            u = div_(hu, h);
            v = div_(hv, h);
        }
    } else {
        u = R(0);
        v = R(0);
    }
}

// Quotients with |num| below this fraction of |den| may round to zero; larger ones keep the
// sign of num / den.
template <typename R>
__device__ __forceinline__ R tiny_ratio();
template <>
__device__ __forceinline__ double tiny_ratio<double>() { return 0x1p-1000; }
template <>
__device__ __forceinline__ float tiny_ratio<float>() { return 0x1p-100f; }

// HLLC flux in the edge frame (section 2.2, ref. [6]).  Reconstructed depths (already zero
// when dry), normal (q) and tangential (w) velocities of both sides; outputs the mass,
// normal-momentum and tangential-momentum flux.  Two-rarefaction wave speeds with the dry-bed
// speeds; mass and normal momentum from the HLL average; tangential momentum carried by the
// mass flux with the tangential velocity upwind of the contact speed S*.
template <typename R>
__device__ __forceinline__ void hllc_normal(R g, R hl, R ql, R wl, R hr, R qr, R wr, R &fh,
                                            R &fq, R &fw)
{
    if (hl == R(0) && hr == R(0)) {
        fh = R(0); fq = R(0); fw = R(0);
        return;
    }
    const R cl = sqrt_(g * hl), cr = sqrt_(g * hr);
    R sl, sr;
    if (hl == R(0)) {
        sl = qr - R(2) * cr;
        sr = qr + cr;
    } else if (hr == R(0)) {
        sl = ql - cl;
        sr = ql + R(2) * cl;
    } else {
        const R us = (ql + qr) / R(2) + (cl - cr);
        const R cs = (cl + cr) / R(2) + (ql - qr) / R(4);
        sl = fmin(ql - cl, us - cs);
        sr = fmax(qr + cr, us + cs);
    }
    const R fhl = hl * ql, fql = hl * ql * ql + R(0.5) * g * hl * hl;
    const R fhr = hr * qr, fqr = hr * qr * qr + R(0.5) * g * hr * hr;
    if (sl >= R(0)) {
        fh = fhl; fq = fql; fw = fh * wl;
    } else if (sr <= R(0)) {
        fh = fhr; fq = fqr; fw = fh * wr;
    } else {
        const R den = sr - sl;
        const R nh = (sr * fhl - sl * fhr) + sl * sr * (hr - hl);
        const R nq = (sr * fql - sl * fqr) + sl * sr * (hr * qr - hl * ql);
        if constexpr (kFastForms<R>) {
            const R rden = rcp_(den);
            fh = quot(nh, rden, den);
            fq = quot(nq, rden, den);
        } else {
            fh = div_(nh, den);
            fq = div_(nq, den);
        }
        // Only the sign of the contact speed S* = num / den is used.  In this branch a side is
        // wet, S_L < q_L and S_R > q_R, so den < 0 and S* has the sign of -num; the quotient
        // is formed only where it could underflow to zero.
        const R num = sl * hr * (qr - sr) - sr * hl * (ql - sl);
        const R den2 = hr * (qr - sr) - hl * (ql - sl);
        const R sstar = fabs(num) < tiny_ratio<R>() * fabs(den2) ? div_(num, den2) : -num;
        const R wup = sstar > R(0) ? wl : (sstar < R(0) ? wr : (wl + wr) / R(2));
        fw = fh * wup;
    }
}

// Flux through an interior edge from side a to side b (unit normal (nx, ny) out of a) with the
// hydrostatic reconstruction of the bed (z* = max, h* = max(0, h - (z* - z)), velocities
// kept) and both side terms p = g/2 (h^2 - h*^2).  (fx, fy) are the momentum fluxes in (x, y).
template <typename R>
__device__ __forceinline__ void interface_flux_uv(R g, R hd, R hl, R ul, R vl, R zl, R hr, R ur,
                                                  R vr, R zr, R nx, R ny, R &fh, R &fx, R &fy,
                                                  R &pl, R &pr)
{
    const R zs = fmax(zl, zr);
    R hsl = fmax(R(0), hl - (zs - zl));
    R hsr = fmax(R(0), hr - (zs - zr));
    if (hsl <= hd) hsl = R(0);
    if (hsr <= hd) hsr = R(0);
    const R ql = ul * nx + vl * ny, wl = vl * nx - ul * ny;
    const R qr = ur * nx + vr * ny, wr = vr * nx - ur * ny;
    R fq, fw;
    hllc_normal(g, hsl, ql, wl, hsr, qr, wr, fh, fq, fw);
    fx = fq * nx - fw * ny;
    fy = fq * ny + fw * nx;
    pl = R(0.5) * g * (hl * hl - hsl * hsl);
    pr = R(0.5) * g * (hr * hr - hsr * hsr);
}

// The same seen from cell l with the right state in conserved variables.
template <typename R>
__device__ __forceinline__ void interface_flux(R g, R hd, R hl, R ul, R vl, R zl, R hr, R hur,
                                               R hvr, R zr, R nx, R ny, R &fh, R &fx, R &fy,
                                               R &p)
{
    R pr, ur, vr;
    velocities(hr, hur, hvr, hd, ur, vr);
    interface_flux_uv(g, hd, hl, ul, vl, zl, hr, ur, vr, zr, nx, ny, fh, fx, fy, p, pr);
}

// Reflective wall (section 3): mirror ghost built in the edge frame (q -> -q, w kept), so the
// mass flux is exactly zero.
template <typename R>
__device__ __forceinline__ void wall_flux(R g, R hd, R h, R u, R v, R nx, R ny, R &fh, R &fx,
                                          R &fy, R &p)
{
    const R q = u * nx + v * ny, w = v * nx - u * ny;
    const R hs = h > hd ? h : R(0);
    R fq, fw;
    hllc_normal(g, hs, q, w, hs, -q, w, fh, fq, fw);
    fx = fq * nx - fw * ny;
    fy = fq * ny + fw * nx;
    p = R(0.5) * g * (h * h - hs * hs);
}

// Inflow segment: discharge q_in per unit length enters through the edge; boundary depth
// h_b = max(h, (q_in^2/g)^(1/3)).  Returns the boundary wave speed q_in/h_b + sqrt(g h_b).
template <typename R>
__device__ __forceinline__ R inflow_flux(R g, R q_in, R h, R nx, R ny, R &fh, R &fx, R &fy)
{
    const R hc = cbrt_(div_(q_in * q_in, g));
    const R hb = fmax(h, hc);
    const R mom = div_(q_in * q_in, hb) + R(0.5) * g * hb * hb;
    fh = -q_in;
    fx = mom * nx;
    fy = mom * ny;
    return div_(q_in, hb) + sqrt_(g * hb);
}

// Semi-implicit Manning friction (eq. 1's S_f, section 2.2) of a wet cell after the flux
// update: D = 1 + dt g n^2 |q*| / (h*^2 cbrt(h*)), q = q* / D.
template <typename R>
__device__ __forceinline__ void friction(R g, R dt, R nm, R hs, R hus, R hvs, R &hun, R &hvn)
{
    const R mag = sqrt_(hus * hus + hvs * hvs);
    const R x = dt * g * nm * nm * mag;
    const R y = hs * hs * cbrt_(hs);
    if constexpr (kFastForms<R>) {
        // 1 / D = y / (y + x) as y times the reciprocal (within 1.5 ulp), for both
        // components; D = 1 exactly when x = 0
        const R rd = x > R(0) ? y * rcp_(y + x) : R(1);
        hun = hus * rd;
        hvn = hvs * rd;
    } else {
        const R d = R(1) + div_(x, y);
        hun = div_(hus, d);
        hvn = div_(hvs, d);
    }
}

template <typename R>
__device__ __forceinline__ R inflow_speed(R g, R q_in, R h)
{
    const R hc = cbrt_(div_(q_in * q_in, g));
    const R hb = fmax(h, hc);
    return div_(q_in, hb) + sqrt_(g * hb);
}

// ------------------------------------------------------------------------ geometry

// Local edge k of a counter-clockwise triangle runs from node k to node k+1; its outward
// unit normal is (dy, -dx) / l (section 2.2, eq. 3, Fig. 1).  Coordinates are double for both
// precisions; the edge vector is rounded to R after the subtraction.  The cell's area and
// inradius come from the mesh (SWE_ARR_CELL_GEO).
template <typename R>
struct CellGeom {
    R nx[3], ny[3], l[3];
};

// Length and outward unit normal (dy, -dx) / l of an edge vector; odd in (dx, dy).
template <typename R>
__device__ __forceinline__ void edge_normal(R dx, R dy, R &nx, R &ny, R &l)
{
    if constexpr (sizeof(R) == 8 && kFastForms<R>) {
        R il;
        len_rcp_nr(dx * dx + dy * dy, l, il);
        nx = quot(dy, il, l);
        ny = quot(-dx, il, l);
    } else {
        l = sqrt_(dx * dx + dy * dy);
        nx = div_(dy, l);
        ny = div_(-dx, l);
    }
}

template <typename R>
__device__ __forceinline__ void cell_geometry(const double2 *__restrict__ xy, int32_t n0,
                                              int32_t n1, int32_t n2, CellGeom<R> &gm)
{
    const double2 p0 = xy[n0], p1 = xy[n1], p2 = xy[n2];
    const double ex[3] = {p1.x - p0.x, p2.x - p1.x, p0.x - p2.x};
    const double ey[3] = {p1.y - p0.y, p2.y - p1.y, p0.y - p2.y};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        edge_normal<R>(static_cast<R>(ex[k]), static_cast<R>(ey[k]), gm.nx[k], gm.ny[k],
                       gm.l[k]);
    }
}

// ------------------------------------------------------------------------ reductions

// A lane's double from another lane of its row of 16 by a DPP move (Ctrl: a quad permutation
// or a row mirror), as two 32-bit moves; every lane of the wave active.
template <int Ctrl>
__device__ __forceinline__ double dpp_double(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = static_cast<int>(b), hi = static_cast<int>(b >> 32);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, Ctrl, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, Ctrl, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(static_cast<unsigned>(hi2)) << 32) |
                                static_cast<unsigned>(lo2));
}

// Minimum over the wave (fmin: a NaN counts only where every value is one), on every lane and
// with every lane active: within each row of 16 lanes by DPP moves (lane xor 1, lane xor 2,
// the half-row mirror, the row mirror), then the four rows' minima read from one lane each.
// No LDS traffic, unlike a shuffle through ds_bpermute.
__device__ __forceinline__ double wave_min(double v)
{
    v = fmin(v, dpp_double<0xB1>(v));    // quad_perm [1, 0, 3, 2]
    v = fmin(v, dpp_double<0x4E>(v));    // quad_perm [2, 3, 0, 1]
    v = fmin(v, dpp_double<0x141>(v));   // row_half_mirror
    v = fmin(v, dpp_double<0x140>(v));   // row_mirror
    const long long b = __double_as_longlong(v);
    const int lo = static_cast<int>(b), hi = static_cast<int>(b >> 32);
    double r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned l = static_cast<unsigned>(__builtin_amdgcn_readlane(lo, 16 * q));
        const unsigned h = static_cast<unsigned>(__builtin_amdgcn_readlane(hi, 16 * q));
        r[q] = __longlong_as_double((static_cast<long long>(h) << 32) | l);
    }
    return fmin(fmin(r[0], r[1]), fmin(r[2], r[3]));
}

// Minimum over the wave of unsigned words, on every lane and with every lane active: DPP
// steps within each row of 16 lanes (as wave_min), then the four rows' minima read from one
// lane each.
template <int Ctrl>
__device__ __forceinline__ unsigned dpp_min_u32(unsigned v)
{
    // all lanes active and in range: the old value (the min's identity) is never taken
    const unsigned o = static_cast<unsigned>(__builtin_amdgcn_update_dpp(
        static_cast<int>(0xffffffffu), static_cast<int>(v), Ctrl, 0xF, 0xF, false));
    return min(v, o);
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned v)
{
    v = dpp_min_u32<0xB1>(v);
    v = dpp_min_u32<0x4E>(v);
    v = dpp_min_u32<0x141>(v);
    v = dpp_min_u32<0x140>(v);
    const unsigned r0 = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 0));
    const unsigned r1 = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 16));
    const unsigned r2 = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 32));
    const unsigned r3 = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 48));
    return min(min(r0, r1), min(r2, r3));
}

// Minimum over the wave of CFL bounds, as a double on every lane.  A bound is positive or
// +inf (never negative, -0 or NaN: cell_dt divides a positive length by a positive speed, or
// gives +inf), and such numbers order as their bit patterns read as unsigned integers; so the
// minimum is an unsigned one: of the 32-bit patterns in FP32 (then widened, exactly), of the
// high words in FP64 and then of the low words of the lanes that hold the high minimum.
__device__ __forceinline__ double wave_min_bound(float v)
{
    return static_cast<double>(__uint_as_float(wave_min_u32(__float_as_uint(v))));
}

__device__ __forceinline__ double wave_min_bound(double v)
{
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned hi = static_cast<unsigned>(b >> 32), lo = static_cast<unsigned>(b);
    const unsigned mh = wave_min_u32(hi);
    const unsigned ml = wave_min_u32(hi == mh ? lo : 0xffffffffu);
    return __longlong_as_double(
        static_cast<long long>((static_cast<unsigned long long>(mh) << 32) | ml));
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}

// Block-wide (TB work-items) min of the CFL bounds (bound: a work-item's, in the step's
// precision), count of clamps and status of a step, on thread 0 (dtc).  A work-item's flag is
// 0 or kStatusNonFinite and its clamp 0 or 1: a wave counts its clamps and flags from ballots,
// and one integer sum across the waves carries both, clamps in the low 16 bits, flagged waves
// above them.
template <int TB, typename R>
__device__ __forceinline__ void block_reduce(R bound, double &dtc, int clamp, int flag, int &cf)
{
    static_assert(TB < (1 << 16), "clamp count must fit 16 bits");
    __shared__ double s_dt[TB / 64];
    __shared__ int s_cf[TB / 64];
    dtc = wave_min_bound(bound);
    cf = __popcll(__ballot(clamp != 0)) + (__ballot(flag != 0) ? (1 << 16) : 0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        s_dt[wv] = dtc;
        s_cf[wv] = cf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < TB / 64; ++w) {
            dtc = fmin(dtc, s_dt[w]);
            cf += s_cf[w];
        }
    }
}

// The block's partials written as partials[slot] (thread 0).
template <int TB, typename R>
__device__ __forceinline__ void block_partials_at(R bound, int clamp, int flag,
                                                  const Partials &part, int slot)
{
    int cf;
    double dtc;
    block_reduce<TB>(bound, dtc, clamp, flag, cf);
    if (threadIdx.x == 0) {
        part.dt[slot] = dtc;
        part.clamps[slot] = cf & 0xffff;
        part.flags[slot] = (cf >> 16) != 0 ? kStatusNonFinite : 0;
    }
}

// The block's partials merged into slot tile / kSlotTiles (thread 0): the bound by an unsigned
// min of its bits (the order of non-negative doubles, with +inf and the NaNs above every
// number, as fmin ignores a NaN), the clamps by an add and the status by an or (both only when
// non-zero); relaxed device-scope atomics, read after the step by dt_group_fold_kernel.  A
// slot takes few workgroups' atomics: one address taking hundreds per step serialises them.
template <int TB, typename R>
__device__ __forceinline__ void block_partials_group(R bound, int clamp, int flag,
                                                     const Partials &part, int slot)
{
    int cf;
    double dtc;
    block_reduce<TB>(bound, dtc, clamp, flag, cf);
    if (threadIdx.x == 0) {
        const int q = slot / kSlotTiles;
        __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(part.dt) + q,
                               static_cast<unsigned long long>(__double_as_longlong(dtc)),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cf & 0xffff)
            __hip_atomic_fetch_add(part.clamps + q, cf & 0xffff, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (cf >> 16)
            __hip_atomic_fetch_or(part.flags + q, static_cast<int32_t>(kStatusNonFinite),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int TB, typename R>
__device__ __forceinline__ void block_partials(R bound, int clamp, int flag, const Partials &part)
{
    block_partials_at<TB>(bound, clamp, flag, part, blockIdx.x);
}

// Account for the step just taken (m: min CFL bound over the cells, cl: clamps, fl: status
// bits of the new state), then set the next step's dt: CFL, replayed from dt_seq, or cut at
// t_end (section 2.2, Courant number).
__device__ void advance_ctrl(Ctrl *ctrl, double m, long long cl, int fl, double courant,
                             const double *dt_seq, int64_t n_seq, int shard)
{
    Ctrl c = *ctrl;
    c.t = c.last ? c.t_end : c.t + c.dt;
    c.dt_min = c.steps == 0 ? c.dt : fmin(c.dt_min, c.dt);
    c.dt_max = c.steps == 0 ? c.dt : fmax(c.dt_max, c.dt);
    c.dt_sum = c.dt_sum + c.dt;
    c.steps += 1;
    c.run_step += 1;
    c.clamps += cl;
    if (c.last) c.done = 1;
    if (fl & kStatusNonFinite) {
        c.status |= kStatusNonFinite;
        c.done = 1;
    }
    if (shard) {
        // a shard keeps its candidate; the all-reduce over shards decides dt and last
        c.dt_cfl = courant * m;
    } else if (!c.done) {
        double dt = courant * m;
        if (dt_seq) dt = c.run_step < n_seq ? dt_seq[c.run_step] : c.dt;
        c.last = 0;
        if (!(dt < kInf)) {
            c.status |= kStatusDry;
            c.done = 1;
        } else if (!(dt > 0.0)) {
            c.status |= kStatusBadDt;
            c.done = 1;
        } else {
            if (c.t_end > 0.0 && dt >= c.t_end - c.t) {
                dt = c.t_end - c.t;
                c.last = 1;
            }
            c.dt = dt;
        }
    }
    *ctrl = c;
}

// How a small single-mesh step finishes its dt reduction itself (ctrl == nullptr: a fold
// kernel follows the step instead).
struct Advance {
    Ctrl *ctrl;
    const double *dt_seq;
    int64_t n_seq;
    double courant;
    int32_t shard;
    int32_t pad;
};

// Block partials of tile `slot`: merged into its slot (group: a single mesh's step with a fold
// kernel after it) or written as the tile's partials; with Fuse and adv.ctrl, the last
// workgroup to arrive (a release increment by each, an acquire before reading) folds all
// n_tiles partials and advances the control block.  No workgroup waits for another; every one
// read the control block before it arrived.
// Fuse selects this at compile time: the kernels without it run measurably faster on large
// grids even though the branch is never taken there.
template <int TB, bool Fuse, typename R>
__device__ __forceinline__ void finish_step(R bound, int clamp, int flag, const Partials &part,
                                            int slot, int n_tiles, const Advance &adv, bool group)
{
    if (!Fuse && group) {
        block_partials_group<TB>(bound, clamp, flag, part, slot);
        return;
    }
    block_partials_at<TB>(bound, clamp, flag, part, slot);
    if constexpr (Fuse) {
    if (!adv.ctrl || threadIdx.x >= 64) return;
    // wave 0 only; work-item 0 wrote the partial
    uint32_t old = 0;
    if (threadIdx.x == 0)
        old = __hip_atomic_fetch_add(part.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0, 64);
    if (old != static_cast<uint32_t>(n_tiles - 1)) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double m = kInf;
    long long cl = 0;
    int fl = 0;
    for (int b = static_cast<int>(threadIdx.x); b < n_tiles; b += 64) {
        m = fmin(m, part.dt[b]);
        cl += part.clamps[b];
        fl |= part.flags[b];
    }
    m = wave_min(m);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cl += __shfl_xor(cl, off, 64);
    fl = wave_or(fl);
    if (threadIdx.x == 0) {
        part.count[0] = 0;
        advance_ctrl(adv.ctrl, m, cl, fl, adv.courant, adv.dt_seq, adv.n_seq, adv.shard);
    }
    }
}

// CFL bound r / (|u| + sqrt(g h)) of a cell (inflow edges add their boundary speed);
// +inf for a dry cell without inflow.  qtab: the scenario's inflow discharges (nullptr: cfg's).
// A function of the cell's state alone, the same in a step's epilogue and in the initial pass,
// so that a run restarted from a saved state takes the uninterrupted run's dt.
template <typename R>
__device__ __forceinline__ R cell_dt(R g, R hd, R h, R hu, R hv, R inradius, const int32_t *nb,
                                     const StepConfig &cfg, const double *qtab = nullptr)
{
    if constexpr (kFastForms<R>) {
        // r / (|u| + sqrt(g h)) as r h / (|(hu, hv)| + h sqrt(g h)): one quotient; the
        // inflow speeds compare scaled by h alike
        const bool wet = h > hd;
        R num = inradius, s = R(0);
        if (wet) {
            num = inradius * h;
            s = sqrt_(hu * hu + hv * hv) + h * sqrt_(g * h);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (nb[k] < SWE_WALL) {
                const double q = qtab ? qtab[-2 - nb[k]] : cfg.inflow_q[-2 - nb[k]];
                R sb = inflow_speed(g, static_cast<R>(q), h);
                if (wet) sb = sb * h;
                if (sb > s) s = sb;
            }
        return s > R(0) ? num * rcp_(s) : static_cast<R>(kInf);   // within 1.5 ulp
    } else {
        R s = R(0);
        if (h > hd) {
            const R u = div_(hu, h), v = div_(hv, h);
            s = sqrt_(u * u + v * v) + sqrt_(g * h);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (nb[k] < SWE_WALL) {
                const double q = qtab ? qtab[-2 - nb[k]] : cfg.inflow_q[-2 - nb[k]];
                const R sb = inflow_speed(g, static_cast<R>(q), h);
                if (sb > s) s = sb;
            }
        return s > R(0) ? div_(inradius, s) : static_cast<R>(kInf);
    }
}

// The positivity clamp, the semi-implicit friction and the next CFL bound of one cell after its
// flux update U* = (hs, hus, hvs) (eq. 4 and the source treatments of section 2.2).  Outputs
// U^{n+1} = (hs, hun, hvn) (hs clamped in place), the cell's CFL bound (+inf with Cfl false: a
// step whose dt is replayed forms none) and whether it clamped.
template <typename R, bool Cfl = true>
__device__ __forceinline__ void cell_finish(R g, R hd, R dt, R nm, R inradius, R &hs, R hus,
                                            R hvs, const int32_t *nb, const StepConfig &cfg,
                                            const double *qtab, R &hun, R &hvn, R &dtc,
                                            int &clamp)
{
    clamp = 0;
    if (hs < R(0)) {
        clamp = 1;
        hs = R(0);
    }
    if (hs > hd) {
        friction(g, dt, nm, hs, hus, hvs, hun, hvn);
    } else {
        hun = R(0);
        hvn = R(0);
    }
    if constexpr (Cfl)
        dtc = cell_dt<R>(g, hd, hs, hun, hvn, inradius, nb, cfg, qtab);
    else
        dtc = static_cast<R>(kInf);
}

// Where a workgroup's cells live when several meshes (scenarios) are stepped together: tile t
// holds cells [tile_start[t], tile_start[t+1]) of scenario tile_scen[t], whose control block
// is ctrl + tile_scen[t] * SWE_CTRL_BYTES and inflow discharges q_table[16 s ..].  A single
// mesh leaves tile_start null: tile t holds cells [TB t, TB t + TB) (TB its tile size).
struct Batch {
    const int32_t *tile_start;
    const int32_t *tile_scen;
    const int32_t *scen_tile_off;   // [n_scen + 1] tiles of each scenario (dt pass)
    const double *q_table;
    int32_t n_scen;
    int32_t remap;       // 1: XCD-contiguous tile order
    int32_t n_tiles;
    int32_t pad;
};

// Workgroups are handed to the eight XCDs in turn; give each XCD a contiguous run of tiles
// so that a tile's neighbours were recently read into the same XCD's L2 by its neighbour
// tiles (remap == 0 keeps the hardware order).
__device__ __forceinline__ int xcd_tile(int b, int n_tiles, int remap)
{
    if (!remap) return b;
    const int per = (n_tiles + 7) / 8;
    return (b % 8) * per + b / 8;
}

__device__ __forceinline__ const Ctrl *ctrl_of(const Ctrl *base, int scen)
{
    return reinterpret_cast<const Ctrl *>(reinterpret_cast<const unsigned char *>(base) +
                                          static_cast<size_t>(scen) * SWE_CTRL_BYTES);
}

// ------------------------------------------------------------------------ kernels

template <typename R>
struct StepArgs {
    const int32_t *__restrict__ nbr;
    const int32_t *__restrict__ c2n;
    const double2 *__restrict__ xy;
    const R *__restrict__ cell_geo;        // [2T]: area, inradius (mesh, in R)
    const R *__restrict__ z;
    const R *__restrict__ n;
    const R *__restrict__ h;
    const R *__restrict__ hu;
    const R *__restrict__ hv;
    R *__restrict__ ho;
    R *__restrict__ huo;
    R *__restrict__ hvo;
    const Ctrl *ctrl;
    Partials part;
    R *us_h, *us_hu, *us_hv;   // optional: U* before clamp and friction (adjoint recompute)
    const double *dt_direct;   // optional: this step's dt; then no control block, no partials
    Advance adv;               // small grids: the step folds its own partials
};

// One explicit step for every cell (eq. 4 with the source treatments of section 2.2).
template <typename R, int TB, bool Fuse>
__global__ __launch_bounds__(TB, SWE_CELL_WAVES) void step_kernel(StepArgs<R> a, StepConfig cfg,
                                                                   Batch bt)
{
    const int tile = xcd_tile(blockIdx.x, bt.n_tiles, bt.remap);
    if (tile >= bt.n_tiles) return;
    const bool batched = bt.tile_start != nullptr;
    const int scen = batched ? bt.tile_scen[tile] : 0;
    const Ctrl *ctrl = ctrl_of(a.ctrl, scen);
    const double *qtab = batched ? bt.q_table + scen * SWE_MAX_INFLOW : nullptr;
    if (!a.dt_direct && ctrl->done) return;   // uniform over the workgroup: its state stopped
    const int64_t T = cfg.n_cells;
    const int64_t s0 = batched ? bt.tile_start[tile] : static_cast<int64_t>(tile) * TB;
    const int64_t s1 = batched ? bt.tile_start[tile + 1] : s0 + TB;
    const int64_t i = s0 + threadIdx.x;
    const R g = static_cast<R>(cfg.g), hd = static_cast<R>(cfg.h_dry);
    const R dt = static_cast<R>(a.dt_direct ? *a.dt_direct : ctrl->dt);
    R dtc = static_cast<R>(kInf);
    int clamp = 0, flag = 0;
    if (i < s1 && i < T) {
        CellGeom<R> gm;
        cell_geometry<R>(a.xy, a.c2n[i], a.c2n[T + i], a.c2n[2 * T + i], gm);
        const R h = a.h[i], hu = a.hu[i], hv = a.hv[i], z = a.z[i];
        R u, v;
        velocities(h, hu, hv, hd, u, v);
        int32_t nb[3];
        R acc0 = R(0), acc1 = R(0), acc2 = R(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            nb[k] = a.nbr[k * T + i];
            const int32_t j = nb[k];
            R fh, fx, fy, p;
            if (j >= 0) {
                interface_flux<R>(g, hd, h, u, v, z, a.h[j], a.hu[j], a.hv[j], a.z[j], gm.nx[k],
                                  gm.ny[k], fh, fx, fy, p);
            } else if (j == SWE_WALL) {
                wall_flux<R>(g, hd, h, u, v, gm.nx[k], gm.ny[k], fh, fx, fy, p);
            } else {
                inflow_flux<R>(g, static_cast<R>(qtab ? qtab[-2 - j] : cfg.inflow_q[-2 - j]), h,
                               gm.nx[k], gm.ny[k],
                               fh, fx, fy);
                p = R(0);
            }
            const R c0 = gm.l[k] * fh;
            const R c1 = gm.l[k] * (fx + p * gm.nx[k]);
            const R c2 = gm.l[k] * (fy + p * gm.ny[k]);
            if (k == 0) {
                acc0 = c0; acc1 = c1; acc2 = c2;
            } else {
                acc0 = acc0 + c0; acc1 = acc1 + c1; acc2 = acc2 + c2;
            }
        }
        // explicit Euler update, positivity clamp, semi-implicit friction
        const R area = a.cell_geo[i], inradius = a.cell_geo[T + i];
        const R r = kFastForms<R> ? dt * rcp_(area) : div_(dt, area);   // dt / A
        R hs = h - r * acc0;
        const R hus = hu - r * acc1;
        const R hvs = hv - r * acc2;
        if (a.us_h) {
            a.us_h[i] = hs;
            a.us_hu[i] = hus;
            a.us_hv[i] = hvs;
        }
        R hun, hvn;
        cell_finish<R>(g, hd, dt, a.n[i], inradius, hs, hus, hvs, nb, cfg, qtab, hun, hvn, dtc,
                       clamp);
        a.ho[i] = hs;
        a.huo[i] = hun;
        a.hvo[i] = hvn;
        if (!isfinite(hs) || !isfinite(hun) || !isfinite(hvn)) flag = kStatusNonFinite;
        if (i >= cfg.n_owned) {   // a shard's halo cell: refreshed by its owner
            dtc = static_cast<R>(kInf);
            clamp = 0;
            flag = 0;
        }
    }
    if (a.dt_direct) return;   // uniform: a replay that needs no dt reduction
    finish_step<TB, Fuse>(dtc, clamp, flag, a.part, tile, bt.n_tiles, a.adv,
                          SWE_GROUP_ATOMIC && !batched);
}

// ------------------------------------------------------------------------ tiled step

// Element i of an array: with O32 (every array the kernel indexes spans less than 4 GiB,
// checked at launch) addressed by a 32-bit byte offset from its base, which the hardware adds
// to the scalar base itself; else by 64-bit index arithmetic.
template <bool O32, typename T>
__device__ __forceinline__ T ld(const T *p, int64_t i)
{
    if constexpr (O32)
        return *reinterpret_cast<const T *>(
            reinterpret_cast<const char *>(p) +
            static_cast<uint32_t>(static_cast<uint32_t>(i) * static_cast<uint32_t>(sizeof(T))));
    else
        return p[i];
}

template <bool O32, typename T>
__device__ __forceinline__ void st(T *p, int64_t i, T v)
{
    if constexpr (O32)
        *reinterpret_cast<T *>(
            reinterpret_cast<char *>(p) +
            static_cast<uint32_t>(static_cast<uint32_t>(i) * static_cast<uint32_t>(sizeof(T)))) = v;
    else
        p[i] = v;
}

// (dx, dy) pairs of the mesh's edge vectors in the step's precision.
template <typename R>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double2;
};
template <>
struct Vec2<float> {
    using type = float2;
};

template <typename R>
struct TileArgs {
    StepArgs<R> s;
    const int32_t *__restrict__ halo_off;
    const int32_t *__restrict__ halo;
    const int32_t *__restrict__ edge_off;
    const uint32_t *__restrict__ edges;
    const typename Vec2<R>::type *__restrict__ edge_vec;   // per edge-list entry (mesh, in R)
    // FP64 with node lists (else null): each tile's node coordinates and, per edge-list entry,
    // the tile-local ids of the two nodes whose difference is its edge vector
    const int32_t *__restrict__ tile_node_off;
    const double2 *__restrict__ tile_nodes;
    const uint16_t *__restrict__ edge_nodes;
    int32_t n_tiles, max_halo, max_edges, max_nodes;
};

// LDS of the tiled step: the tile + halo states ((h, u, v, z) interleaved per cell) and five
// values per edge-list entry (side a's contribution and side b's momentum contribution; side
// b's mass part is -a's).
// Plain layout: [states | 5 rows of max_edges].  Shared layout (at most 2 TB entries, TB the
// tile's cells): [5 rows of TB for entries 0..TB-1 | states], the entries from TB on written in
// 5 rows of TB over the states once every interface of the tile has been evaluated.  An FP64
// step with node lists (shared layout only: a tile of at most 256 nodes has at most 511
// interfaces) appends the tile's nodes, (x, y) each; the layout's words before them are even.
inline size_t tile_lds_nodes(size_t word, int64_t max_nodes)
{
    return word == 8 && max_nodes > 0 ? 16 * static_cast<size_t>(max_nodes) : 0;
}

inline size_t tile_lds_plain(size_t word, int64_t tb, int64_t max_halo, int64_t max_edges)
{
    return 4 * word * static_cast<size_t>(tb + max_halo) +
           5 * word * static_cast<size_t>(max_edges);
}

inline size_t tile_lds_shared(size_t word, int64_t tb, int64_t max_halo, int64_t max_nodes)
{
    return word * (5 * static_cast<size_t>(tb) +
                   std::max(4 * static_cast<size_t>(tb + max_halo), 5 * static_cast<size_t>(tb))) +
           tile_lds_nodes(word, max_nodes);
}

// Static LDS of the tiled step besides: its slot table and the block reduction's partials.
constexpr size_t tile_static_lds(int64_t tb) { return 3 * static_cast<size_t>(tb) * sizeof(uint16_t) + 64; }
static_assert(tile_static_lds(kTileMax) <= kTileStaticLdsMax, "static LDS beyond the allowance");

// The shared layout costs one more barrier per tile; take it only where the plain layout
// limits a CU (160 KiB of LDS) to fewer than eight waves per SIMD and the shared one fits
// more workgroups.  FP64 only: FP32 tiles of the meshes built here reach eight waves in the
// plain layout.
inline bool tile_alias(size_t word, int64_t tb, int64_t max_halo, int64_t max_edges,
                       int64_t max_nodes)
{
    if (!SWE_TILE_ALIAS || word != 8 || max_edges > 2 * tb) return false;
    constexpr size_t kLdsPerCu = 160 * 1024;
    const size_t st = tile_static_lds(tb);
    const size_t plain = kLdsPerCu / (tile_lds_plain(word, tb, max_halo, max_edges) + st);
    const size_t shared = kLdsPerCu / (tile_lds_shared(word, tb, max_halo, max_nodes) + st);
    // waves per SIMD: workgroups per CU x (tb / 64) waves over 4 SIMDs
    return plain * static_cast<size_t>(tb) < 8 * 256 && shared > plain;
}

inline size_t tile_lds_bytes(size_t word, int64_t tb, int64_t max_halo, int64_t max_edges,
                             int64_t max_nodes)
{
    return tile_alias(word, tb, max_halo, max_edges, max_nodes)
               ? tile_lds_shared(word, tb, max_halo, max_nodes)
               : tile_lds_plain(word, tb, max_halo, max_edges);
}

// One explicit step, tiled.  Every global load of the workgroup is issued up front: the own
// cell (state, bed, Manning, area, inradius), the halo states, and the first two rounds of
// edge-list entries with their edge vectors (Nodes: their node ids, and the tile's node
// coordinates, one per work-item), all from the mesh's arrays, so no load waits on another's
// index but the halo list's.  Phase 1 stages the tile's cells and its halo in LDS as
// (h, u, v, z), each velocity computed once.  Phase 2 also records, for each tile cell's local
// edge, its entry in the edge list (the entries carry both sides' local edges).  Phase 2
// evaluates every interface of the edge list once (section 2.3's interface loop, restricted
// to the tile) and stores the contributions l (F + p n) to eq. 3 of both sides, computed
// exactly as the per-cell form computes them; with the shared layout (Shared) the second
// round's results wait in registers until every work-item has read the states they replace.
// Phase 3 sums each cell's three contributions in local-edge order and applies the update of
// eq. 4, the clamp, the friction and the next CFL bound, as the per-cell kernel does.
// Replay: a step whose dt is given (a.dt_direct) forms no CFL bound and reads no inradius; the
// other instances replay too when a.dt_direct is set, forming the bound and discarding it.
template <typename R, int TB, bool O32, bool Fuse, bool Shared, bool Nodes, bool Replay = false>
__global__ __launch_bounds__(TB, SWE_TILE_WAVES) void tile_step_kernel(TileArgs<R> ta, StepConfig cfg,
                                                                       Batch bt)
{
    static_assert(!Nodes || (sizeof(R) == 8 && Shared), "node lists serve the shared FP64 layout");
    const StepArgs<R> &a = ta.s;
    const int tile = xcd_tile(blockIdx.x, ta.n_tiles, bt.remap);
    if (tile >= ta.n_tiles) return;
    const bool batched = bt.tile_start != nullptr;
    const int scen = batched ? bt.tile_scen[tile] : 0;
    const Ctrl *ctrl = ctrl_of(a.ctrl, scen);
    const double *qtab = batched ? bt.q_table + scen * SWE_MAX_INFLOW : nullptr;
    if (!a.dt_direct && ctrl->done) return;   // uniform over the workgroup: its scenario stopped
    extern __shared__ __align__(16) unsigned char smem[];
    R *const lds = reinterpret_cast<R *>(smem);
    const int ns = TB + ta.max_halo;
    // word offsets: states, and edge-list entry q of row j at ebase + j estride + q (+ bshift
    // from entry TB on)
    constexpr bool alias = Shared;
    const int sbase = alias ? 5 * TB : 0;
    const int ebase = alias ? 0 : 4 * ns;
    const int estride = alias ? TB : ta.max_edges;
    const int bshift = alias ? 4 * TB : 0;
    // staged cells' (h, u, v, z) interleaved: one cell in two 16-byte LDS accesses (FP64)
    struct alignas(16) St {
        R h, u, v, z;
    };
    St *const s_st = reinterpret_cast<St *>(lds + sbase);
    // Nodes (FP64 with node lists): the tile's nodes after the layout's other words (an even
    // count, so 16-byte aligned), each entry's edge vector formed from them
    constexpr bool nodes = Nodes;
    double2 *const s_nd = reinterpret_cast<double2 *>(lds + 5 * TB + max(4 * ns, 5 * TB));
    // each tile cell's local edge k -> its edge-list entry (bit 15: the cell is side b),
    // filled from the edge list in phase 2
    __shared__ uint16_t s_slot[3 * TB];

    const int64_t T = cfg.n_cells;
    const int64_t s0 = batched ? bt.tile_start[tile] : static_cast<int64_t>(tile) * TB;
    const int64_t s1 = batched ? bt.tile_start[tile + 1] : s0 + TB;
    const int tid = threadIdx.x;
    const int64_t i = s0 + tid;
    const bool mine = i < s1 && i < T;
    const R g = static_cast<R>(cfg.g), hd = static_cast<R>(cfg.h_dry);
    const R dt = static_cast<R>(a.dt_direct ? *a.dt_direct : ctrl->dt);
    // Work-item positions in the edge list (pt) and the halo list (ph).  About 1.7 interfaces
    // per cell leave some waves a single round of phase 2; the halo loads go to those waves,
    // and which waves they are turns with the tile, so that no SIMD idles through a round.
    const int pt = (tid + 64 * (tile % (TB / 64))) & (TB - 1);
    const int ph = TB - 1 - pt;

    // global loads: own cell
    R h = R(0), hu = R(0), hv = R(0), zc = R(0), nm = R(0), area = R(0), inradius = R(1);
    if (mine) {
        h = ld<O32>(a.h, i); hu = ld<O32>(a.hu, i); hv = ld<O32>(a.hv, i);
        zc = ld<O32>(a.z, i); nm = ld<O32>(a.n, i);
        area = ld<O32>(a.cell_geo, i);
        if constexpr (!Replay) inradius = ld<O32>(a.cell_geo, T + i);   // for the CFL bound
    }
    // global loads: the edge-list entries of the first two rounds and their edge vectors (or
    // their node ids, and the tile's nodes, one per work-item)
    const int eb = ta.edge_off[tile], ee = ta.edge_off[tile + 1];
    uint32_t ew[2] = {0u, 0u}, en[2] = {0u, 0u};
    typename Vec2<R>::type ev[2] = {{R(0), R(0)}, {R(0), R(0)}};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int e = eb + pt + it * TB;
        if (e < ee) {
            ew[it] = ld<O32>(ta.edges, e);
            if (nodes)
                en[it] = ld<O32>(ta.edge_nodes, e);
            else
                ev[it] = ld<O32>(ta.edge_vec, e);
        }
    }
    double2 nd = {0.0, 0.0};
    const int nb0 = nodes ? ta.tile_node_off[tile] : 0;
    const bool node_mine = nodes && tid < ta.tile_node_off[tile + 1] - nb0;
    if (node_mine) nd = ld<O32>(ta.tile_nodes, nb0 + tid);
    // phase 1: halo and own cell into LDS
    const int hb = ta.halo_off[tile], he = ta.halo_off[tile + 1];
    for (int j = hb + ph; j < he; j += TB) {
        const int32_t c = ld<O32>(ta.halo, j);
        const R hh = ld<O32>(a.h, c);
        const int q = TB + (j - hb);
        R uu, vv;
        velocities(hh, ld<O32>(a.hu, c), ld<O32>(a.hv, c), hd, uu, vv);
        s_st[q] = St{hh, uu, vv, ld<O32>(a.z, c)};
    }
    if (mine) {
        R uu, vv;
        velocities(h, hu, hv, hd, uu, vv);
        s_st[tid] = St{h, uu, vv, zc};
    }
    if (node_mine) s_nd[tid] = nd;
    __syncthreads();
    // an entry's edge vector: node k+1 minus node k of its owning cell, the same subtraction
    // (and bits) as the mesh's edge vectors
    auto node_vec = [&](uint32_t p, R &dx, R &dy) {
        const double2 p0 = s_nd[p & 0xffu], p1 = s_nd[(p >> 8) & 0xffu];
        dx = static_cast<R>(p1.x - p0.x);
        dy = static_cast<R>(p1.y - p0.y);
    };
    R edx[2] = {ev[0].x, ev[1].x}, edy[2] = {ev[0].y, ev[1].y};
    if (nodes) {
        node_vec(en[0], edx[0], edy[0]);
        node_vec(en[1], edx[1], edy[1]);
    }

    // phase 2: the tile's interfaces, each once
    struct EdgeOut {
        R a0, a1, a2, b1, b2;
    };
    // returns whether side b is a cell (its momentum parts b1, b2 set)
    auto flux = [&](uint32_t w, R dx, R dy, EdgeOut &o) {
        const int ca = static_cast<int>(w & kEdgeA);
        const int cb = static_cast<int16_t>(w >> 16);
        R nx, ny, l;
        edge_normal<R>(dx, dy, nx, ny, l);
        const St A = s_st[ca];
        const R ha = A.h, ua = A.u, va = A.v;
        R fh, fx, fy, pa, pb;
        if (cb >= 0) {
            const St B = s_st[cb];
            interface_flux_uv<R>(g, hd, ha, ua, va, A.z, B.h, B.u, B.v, B.z, nx, ny, fh, fx, fy,
                                 pa, pb);
            // side b's contributions are l (-f_h) = -(l f_h) and l (-f + p_b (-n)) =
            // -(l (f + p_b n)), exactly; its momentum parts are stored as they are added
            o.b1 = -(l * (fx + pb * nx));
            o.b2 = -(l * (fy + pb * ny));
        } else if (cb == SWE_WALL) {
            wall_flux<R>(g, hd, ha, ua, va, nx, ny, fh, fx, fy, pa);
        } else {
            const double qin = qtab ? qtab[-2 - cb] : cfg.inflow_q[-2 - cb];
            inflow_flux<R>(g, static_cast<R>(qin), ha, nx, ny, fh, fx, fy);
            pa = R(0);
        }
        o.a0 = l * fh;
        o.a1 = l * (fx + pa * nx);
        o.a2 = l * (fy + pa * ny);
        return cb >= 0;
    };
    auto put = [&](int q, uint32_t w, const EdgeOut &o, bool two) {
        R *e = lds + ebase + q + (q >= TB ? bshift : 0);
        e[0] = o.a0;
        e[estride] = o.a1;
        e[2 * estride] = o.a2;
        if (two) {
            e[3 * estride] = o.b1;
            e[4 * estride] = o.b2;
        }
        s_slot[3 * (w & kEdgeA) + ((w >> kEdgeKa) & 3u)] = static_cast<uint16_t>(q);
        const int cb = static_cast<int16_t>(w >> 16);
        if (cb >= 0 && cb < TB) s_slot[3 * cb + ((w >> kEdgeKb) & 3u)] = static_cast<uint16_t>(q | 0x8000);
    };
    {
        EdgeOut o;
        if (eb + pt < ee) put(pt, ew[0], o, flux(ew[0], edx[0], edy[0], o));
        const bool has1 = eb + pt + TB < ee;
        bool two1 = false;
        if (has1) two1 = flux(ew[1], edx[1], edy[1], o);
        if constexpr (alias) __syncthreads();   // every read of the states is done
        if (has1) put(pt + TB, ew[1], o, two1);
    }
    for (int e = eb + pt + 2 * TB; e < ee; e += TB) {   // plain layout only
        const uint32_t w = ld<O32>(ta.edges, e);
        const auto d = ld<O32>(ta.edge_vec, e);
        EdgeOut o;
        put(e - eb, w, o, flux(w, d.x, d.y, o));
    }
    __syncthreads();

    // phase 3: per-cell sum, update, clamp, friction, next CFL bound
    R dtc = static_cast<R>(kInf);
    int clamp = 0, flag = 0;
    if (mine) {
        const uint32_t sl[3] = {s_slot[3 * tid], s_slot[3 * tid + 1], s_slot[3 * tid + 2]};
        R acc0 = R(0), acc1 = R(0), acc2 = R(0);
        int32_t nb[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int q = static_cast<int>(sl[k] & 0x7fffu);
            const bool side_b = (sl[k] & 0x8000u) != 0;
            const R *e = lds + ebase + q + (q >= TB ? bshift : 0);
            const R *m = e + (side_b ? 3 * estride : estride);   // the side's momentum rows
            const R c0 = side_b ? -e[0] : e[0];
            const R c1 = m[0];
            const R c2 = m[estride];
            nb[k] = 0;
            if (!Replay && (cfg.n_inflow > 0 || batched) && !side_b)   // for the CFL bound
                nb[k] = static_cast<int16_t>(ld<O32>(ta.edges, eb + q) >> 16);
            if (k == 0) {
                acc0 = c0; acc1 = c1; acc2 = c2;
            } else {
                acc0 = acc0 + c0; acc1 = acc1 + c1; acc2 = acc2 + c2;
            }
        }
        const R r = kFastForms<R> ? dt * rcp_(area) : div_(dt, area);   // dt / A
        R hs = h - r * acc0;
        const R hus = hu - r * acc1;
        const R hvs = hv - r * acc2;
        if (a.us_h) {
            st<O32>(a.us_h, i, hs);
            st<O32>(a.us_hu, i, hus);
            st<O32>(a.us_hv, i, hvs);
        }
        R hun, hvn;
        cell_finish<R, !Replay>(g, hd, dt, nm, inradius, hs, hus, hvs, nb, cfg, qtab, hun, hvn, dtc,
                                clamp);
        st<O32>(a.ho, i, hs);
        st<O32>(a.huo, i, hun);
        st<O32>(a.hvo, i, hvn);
        if (!isfinite(hs) || !isfinite(hun) || !isfinite(hvn)) flag = kStatusNonFinite;
        if (i >= cfg.n_owned) {   // a shard's halo cell: refreshed by its owner
            dtc = static_cast<R>(kInf);
            clamp = 0;
            flag = 0;
        }
    }
    if (Replay || a.dt_direct) return;   // uniform: a replay that needs no dt reduction
    finish_step<TB, Fuse>(dtc, clamp, flag, a.part, tile, ta.n_tiles, a.adv,
                          SWE_GROUP_ATOMIC && !batched);
}

// CFL bounds of the initial state.
template <typename R, int TB>
__global__ __launch_bounds__(TB) void init_kernel(StepArgs<R> a, StepConfig cfg, Batch bt)
{
    const int64_t T = cfg.n_cells;
    const bool batched = bt.tile_start != nullptr;
    const int64_t s0 = batched ? bt.tile_start[blockIdx.x] : static_cast<int64_t>(blockIdx.x) * TB;
    const int64_t s1 = batched ? bt.tile_start[blockIdx.x + 1] : s0 + TB;
    const double *qtab = batched ? bt.q_table + bt.tile_scen[blockIdx.x] * SWE_MAX_INFLOW : nullptr;
    const int64_t i = s0 + threadIdx.x;
    const R g = static_cast<R>(cfg.g), hd = static_cast<R>(cfg.h_dry);
    R dtc = static_cast<R>(kInf);
    int flag = 0;
    if (i < s1 && i < T) {
        const int32_t nb[3] = {a.nbr[i], a.nbr[T + i], a.nbr[2 * T + i]};
        const R h = a.h[i], hu = a.hu[i], hv = a.hv[i];
        if (!isfinite(h) || !isfinite(hu) || !isfinite(hv)) flag = kStatusNonFinite;
        dtc = cell_dt<R>(g, hd, h, hu, hv, a.cell_geo[T + i], nb, cfg, qtab);
        if (i >= cfg.n_owned) {
            dtc = static_cast<R>(kInf);
            flag = 0;
        }
    }
    block_partials<TB>(dtc, 0, flag, a.part);
}

constexpr int kPassThreads = 1024;

// Min, sum and or over the kPassThreads work-items of a workgroup, the result on work-item 0;
// every work-item calls it (one barrier).
__device__ __forceinline__ void pass_reduce(double &m, long long &cl, int &fl)
{
    __shared__ double s_dt[kPassThreads / 64];
    __shared__ long long s_cl[kPassThreads / 64];
    __shared__ int s_fl[kPassThreads / 64];
    m = wave_min(m);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cl += __shfl_xor(cl, off, 64);
    fl = wave_or(fl);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        s_dt[wv] = m;
        s_cl[wv] = cl;
        s_fl[wv] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kPassThreads / 64; ++w) {
            m = fmin(m, s_dt[w]);
            cl += s_cl[w];
            fl |= s_fl[w];
        }
}

// Reduce the per-block partials into the control block: account for the step just taken
// (mode 1) or start the state (mode 0, which also clears the arrival counter of
// dt_fold_kernel), then set the next step's dt (CFL, replayed, or cut at t_end).
__global__ __launch_bounds__(kPassThreads) void dt_pass_kernel(Ctrl *ctrl_base, Partials part,
                                                               int64_t nb, double courant,
                                                               const double *dt_seq,
                                                               int64_t n_seq, int mode,
                                                               double t0, double t_end,
                                                               int cur0, Batch bt, int shard)
{
    // workgroup s reduces scenario s's tiles (a single mesh: all nb partials)
    Ctrl *ctrl = const_cast<Ctrl *>(ctrl_of(ctrl_base, blockIdx.x));
    const int64_t b_lo = bt.scen_tile_off ? bt.scen_tile_off[blockIdx.x] : 0;
    const int64_t b_hi = bt.scen_tile_off ? bt.scen_tile_off[blockIdx.x + 1] : nb;
    if (mode == 0 && blockIdx.x == 0)
        for (int64_t q = threadIdx.x; q <= (nb + kGroup - 1) / kGroup; q += kPassThreads)
            part.count[q] = 0;
    if (mode == 1 && ctrl->done) return;
    double m = kInf;
    long long cl = 0;
    int fl = 0;
    // kUnroll independent loads per work-item in flight: the partials are few, so latency,
    // not bandwidth, bounds this loop
    constexpr int kUnroll = 16;
    for (int64_t b0 = b_lo + threadIdx.x; b0 < b_hi; b0 += kPassThreads * kUnroll) {
        double v[kUnroll];
        int c[kUnroll], f[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t b = b0 + static_cast<int64_t>(u) * kPassThreads;
            const bool in = b < b_hi;
            v[u] = in ? part.dt[b] : kInf;
            c[u] = in ? part.clamps[b] : 0;
            f[u] = in ? part.flags[b] : 0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            m = fmin(m, v[u]);
            cl += c[u];
            fl |= f[u];
        }
    }
    pass_reduce(m, cl, fl);
    if (mode == 0 && !bt.scen_tile_off) {
        // a single mesh's first step merges its partials into the slots (dt_group_fold_kernel
        // resets them after each step): they start reset, now that the partials are read
        for (int64_t q = threadIdx.x; q < n_slots(nb); q += kPassThreads) {
            reinterpret_cast<unsigned long long *>(part.dt)[q] = kInfBits;
            part.clamps[q] = 0;
            part.flags[q] = 0;
        }
    }
    if (threadIdx.x != 0) return;
    if (mode == 1) {
        advance_ctrl(ctrl, m, cl, fl, courant, dt_seq, n_seq, shard);
        return;
    }
    Ctrl c = *ctrl;
    c.t = t0;
    c.dt = 0.0;
    c.t_end = t_end;
    c.dt_min = 0.0; c.dt_max = 0.0; c.dt_sum = 0.0;
    c.steps = 0; c.run_step = 0; c.clamps = 0;
    c.status = 0; c.done = 0; c.last = 0;
    c.cur0 = cur0;
    if (t_end > 0.0 && t0 >= t_end) c.done = 1;
    if (fl & kStatusNonFinite) {
        c.status |= kStatusNonFinite;
        c.done = 1;
    }
    c.dt_cfl = courant * m;
    if (!c.done && !shard) {
        double dt = courant * m;
        if (!(dt < kInf)) {
            c.status |= kStatusDry;
            c.done = 1;
        } else if (!(dt > 0.0)) {
            c.status |= kStatusBadDt;
            c.done = 1;
        } else {
            if (c.t_end > 0.0 && dt >= c.t_end - c.t) {
                dt = c.t_end - c.t;
                c.last = 1;
            }
            c.dt = dt;
        }
    }
    *ctrl = c;
}

// Fold kGroup work-items' (min, sum, or) into work-item 0's values.
__device__ __forceinline__ void fold_group(double &m, long long &cl, int &fl)
{
    __shared__ double s_dt[kGroup / 64];
    __shared__ long long s_cl[kGroup / 64];
    __shared__ int s_fl[kGroup / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    m = wave_min(m);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cl += __shfl_xor(cl, off, 64);
    fl = wave_or(fl);
    if (lane == 0) {
        s_dt[wv] = m;
        s_cl[wv] = cl;
        s_fl[wv] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kGroup / 64; ++w) {
            m = fmin(m, s_dt[w]);
            cl += s_cl[w];
            fl |= s_fl[w];
        }
    __syncthreads();
}

// The dt pass of a single mesh after a step whose workgroups merged their partials into the
// slots: one workgroup folds the ns slots, resets them for the next step (+inf, 0, 0) and
// advances the control block.  A step skipped as done merged nothing: the slots stay reset.
__global__ __launch_bounds__(kPassThreads) void dt_group_fold_kernel(Ctrl *ctrl, Partials part,
                                                                    int64_t ns, double courant,
                                                                    const double *dt_seq,
                                                                    int64_t n_seq, int shard)
{
    if (ctrl->done) return;   // uniform
    unsigned long long *const bits = reinterpret_cast<unsigned long long *>(part.dt);
    double m = kInf;
    long long cl = 0;
    int fl = 0;
    // kUnroll independent loads per work-item in flight: latency, not bandwidth, bounds this
    constexpr int kUnroll = 4;
    for (int64_t q0 = threadIdx.x; q0 < ns; q0 += kPassThreads * kUnroll) {
        unsigned long long v[kUnroll];
        int c[kUnroll], f[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t q = q0 + static_cast<int64_t>(u) * kPassThreads;
            const bool in = q < ns;
            v[u] = in ? bits[q] : kInfBits;
            c[u] = in ? part.clamps[q] : 0;
            f[u] = in ? part.flags[q] : 0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t q = q0 + static_cast<int64_t>(u) * kPassThreads;
            if (q < ns) {
                bits[q] = kInfBits;
                part.clamps[q] = 0;
                part.flags[q] = 0;
            }
            m = fmin(m, __longlong_as_double(static_cast<long long>(v[u])));
            cl += c[u];
            fl |= f[u];
        }
    }
    pass_reduce(m, cl, fl);
    if (threadIdx.x == 0) advance_ctrl(ctrl, m, cl, fl, courant, dt_seq, n_seq, shard);
}

// The dt pass of a single mesh, spread over the chip: workgroup q folds the partials of tiles
// [kGroup q, kGroup q + kGroup) into group partial q; the last workgroup to finish folds the
// groups and advances the control block.  Nothing waits: arrivals are counted with a release
// increment, and only the last arrival (acquire) reads what the others wrote.
__global__ __launch_bounds__(kGroup) void dt_fold_kernel(Ctrl *ctrl, Partials part, int64_t nb,
                                                        double courant, const double *dt_seq,
                                                        int64_t n_seq, int shard)
{
    __shared__ int s_last;
    // uniform; the control block changes only after every workgroup has arrived
    if (ctrl->done) return;
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kGroup + threadIdx.x;
    double m = b < nb ? part.dt[b] : kInf;
    long long cl = b < nb ? part.clamps[b] : 0;
    int fl = b < nb ? part.flags[b] : 0;
    fold_group(m, cl, fl);
    if (threadIdx.x == 0) {
        part.gdt[blockIdx.x] = m;
        part.gclamps[blockIdx.x] = static_cast<int32_t>(cl);
        part.gflags[blockIdx.x] = fl;
        const uint32_t old = __hip_atomic_fetch_add(part.count, 1u, __ATOMIC_RELEASE,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        s_last = old == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    m = kInf;
    cl = 0;
    fl = 0;
    for (int q = threadIdx.x; q < static_cast<int>(gridDim.x); q += kGroup) {
        m = fmin(m, part.gdt[q]);
        cl += part.gclamps[q];
        fl |= part.gflags[q];
    }
    fold_group(m, cl, fl);
    if (threadIdx.x == 0) {
        part.count[0] = 0;
        advance_ctrl(ctrl, m, cl, fl, courant, dt_seq, n_seq, shard);
    }
}

// Control blocks of the shards of one mesh (swe_shard_dt_combine).
struct ShardCtrls {
    Ctrl *c[kMaxShards];
};

// The dt all-reduce of a sharded run: the minimum of the shards' CFL candidates, cut at t_end,
// becomes every shard's next dt; a shard that stopped stops them all.
__global__ void shard_combine_kernel(ShardCtrls sc, int n)
{
    if (threadIdx.x != 0) return;
    double m = kInf;
    int32_t status = 0, done = 0;
    for (int p = 0; p < n; ++p) {
        m = fmin(m, sc.c[p]->dt_cfl);
        status |= sc.c[p]->status;
        done |= sc.c[p]->done;
    }
    for (int p = 0; p < n; ++p) {
        Ctrl c = *sc.c[p];
        c.status |= status;
        c.last = 0;
        if (done) {
            c.done = 1;
        } else if (!(m < kInf)) {
            c.status |= kStatusDry;
            c.done = 1;
        } else if (!(m > 0.0)) {
            c.status |= kStatusBadDt;
            c.done = 1;
        } else {
            double dt = m;
            if (c.t_end > 0.0 && dt >= c.t_end - c.t) {
                dt = c.t_end - c.t;
                c.last = 1;
            }
            c.dt = dt;
        }
        *sc.c[p] = c;
    }
}

// Halo exchange of a sharded run: gather rows idx of (h, hu, hv) into a buffer of 3n values
// (pack), or scatter such a buffer into rows idx (unpack).
template <typename R>
__global__ void halo_kernel(int64_t n, const int32_t *__restrict__ idx, int pack,
                            const R *__restrict__ buf_in, R *__restrict__ buf_out,
                            const R *__restrict__ h, const R *__restrict__ hu,
                            const R *__restrict__ hv, R *__restrict__ ho, R *__restrict__ huo,
                            R *__restrict__ hvo)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t r = idx[k];
    if (pack) {
        buf_out[k] = h[r];
        buf_out[n + k] = hu[r];
        buf_out[2 * n + k] = hv[r];
    } else {
        ho[r] = buf_in[k];
        huo[r] = buf_in[n + k];
        hvo[r] = buf_in[2 * n + k];
    }
}

// Start a run: restart the dt_seq index and, when replaying, take dt_seq[0] (cut at t_end).
__global__ void run_begin_kernel(Ctrl *ctrl, const double *dt_seq)
{
    if (threadIdx.x != 0) return;
    Ctrl c = *ctrl;
    c.run_step = 0;
    if (dt_seq && !c.done) {
        double dt = dt_seq[0];
        c.last = 0;
        if (!(dt > 0.0) || !(dt < kInf)) {
            c.status |= kStatusBadDt;
            c.done = 1;
        } else {
            if (c.t_end > 0.0 && dt >= c.t_end - c.t) {
                dt = c.t_end - c.t;
                c.last = 1;
            }
            c.dt = dt;
        }
    }
    *ctrl = c;
}

// Test hook: interface or wall fluxes on independent edges.
template <typename R>
__global__ void flux_eval_kernel(int64_t n, R g, R hd, const R *hl, const R *hul, const R *hvl,
                                 const R *zl, const R *hr, const R *hur, const R *hvr,
                                 const R *zr, const R *nx, const R *ny, R *f, R *p)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const R h = hl[i];
    R u, v;
    velocities(h, hul[i], hvl[i], hd, u, v);
    R fh, fx, fy, pp;
    if (hr)
        interface_flux<R>(g, hd, h, u, v, zl[i], hr[i], hur[i], hvr[i], zr[i], nx[i], ny[i], fh,
                          fx, fy, pp);
    else
        wall_flux<R>(g, hd, h, u, v, nx[i], ny[i], fh, fx, fy, pp);
    f[3 * i] = fh;
    f[3 * i + 1] = fx;
    f[3 * i + 2] = fy;
    p[i] = pp;
}

template <typename R>
StepArgs<R> make_args(const swe_dev_mesh &dm, const swe_state &s, int cur)
{
    StepArgs<R> a;
    a.nbr = dm.nbr;
    a.c2n = dm.c2n;
    a.xy = reinterpret_cast<const double2 *>(dm.xy);
    if constexpr (sizeof(R) == 8)
        a.cell_geo = dm.cell_geo;
    else
        a.cell_geo = dm.cell_geo32;
    a.z = static_cast<const R *>(s.z);
    a.n = static_cast<const R *>(s.n);
    a.h = static_cast<const R *>(s.h[cur]);
    a.hu = static_cast<const R *>(s.hu[cur]);
    a.hv = static_cast<const R *>(s.hv[cur]);
    a.ho = static_cast<R *>(s.h[1 - cur]);
    a.huo = static_cast<R *>(s.hu[1 - cur]);
    a.hvo = static_cast<R *>(s.hv[1 - cur]);
    a.ctrl = static_cast<const Ctrl *>(s.ctrl);
    a.part = Partials{};   // set by the launcher, for the launch's tiles
    a.us_h = a.us_hu = a.us_hv = nullptr;
    a.dt_direct = nullptr;
    a.adv = Advance{nullptr, nullptr, 0, 0.0, 0, 0};
    return a;
}

template <typename R>
TileArgs<R> make_tile_args(const swe_dev_mesh &dm, const swe_state &s, int cur,
                           const TileLayout &tl)
{
    TileArgs<R> t;
    t.s = make_args<R>(dm, s, cur);
    t.halo_off = dm.halo_off;
    t.halo = dm.halo;
    t.edge_off = dm.edge_off;
    t.edges = dm.edges;
    t.tile_node_off = nullptr;
    t.tile_nodes = nullptr;
    t.edge_nodes = nullptr;
    t.max_nodes = 0;
    if constexpr (sizeof(R) == 8) {
        t.edge_vec = reinterpret_cast<const double2 *>(dm.edge_vec);
        if (tl.max_nodes > 0 && dm.tile_node_off && dm.tile_nodes && dm.edge_nodes) {
            t.tile_node_off = dm.tile_node_off;
            t.tile_nodes = reinterpret_cast<const double2 *>(dm.tile_nodes);
            t.edge_nodes = dm.edge_nodes;
            t.max_nodes = tl.max_nodes;
        }
    } else {
        t.edge_vec = reinterpret_cast<const float2 *>(dm.edge_vec32);
    }
    t.n_tiles = static_cast<int32_t>(tl.n_tiles);
    t.max_halo = tl.max_halo;
    t.max_edges = tl.max_edges;
    return t;
}

}  // namespace

namespace {

Batch batch_view(const BatchLaunch *b)
{
    Batch v;
    v.tile_start = b ? b->tile_start : nullptr;
    v.tile_scen = b ? b->tile_scen : nullptr;
    v.scen_tile_off = b ? b->scen_tile_off : nullptr;
    v.q_table = b ? b->q_table : nullptr;
    v.n_scen = b ? b->n_scen : 1;
    v.remap = 1;
    v.n_tiles = 0;
    v.pad = 0;
    return v;
}

}  // namespace

// Kernels are instantiated for every tile size; with_tile(tile, f) calls f with it as a
// compile-time constant.
template <typename F>
int with_tile(int tile, F &&f)
{
    switch (tile) {
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    default: return static_cast<int>(hipErrorInvalidValue);
    }
}

int launch_init(int dtype, const swe_dev_mesh &dm, const StepConfig &cfg, const swe_state &s,
                double t0, double t_end, void *stream, const BatchLaunch *batch)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nb = batch ? batch->n_tiles : n_tiles_of(cfg.n_cells, cfg.tile);
    const Batch bv = batch_view(batch);
    const Partials part = partials_for(s.work, nb);
    const int e = with_tile(cfg.tile, [&](auto tb) {
        constexpr int TB = decltype(tb)::value;
        if (dtype == SWE_F64) {
            StepArgs<double> a = make_args<double>(dm, s, s.cur);
            a.part = part;
            init_kernel<double, TB><<<dim3(nb), dim3(TB), 0, st>>>(a, cfg, bv);
        } else {
            StepArgs<float> a = make_args<float>(dm, s, s.cur);
            a.part = part;
            init_kernel<float, TB><<<dim3(nb), dim3(TB), 0, st>>>(a, cfg, bv);
        }
        return static_cast<int>(hipGetLastError());
    });
    if (e != hipSuccess) return e;
    dt_pass_kernel<<<dim3(bv.n_scen), kPassThreads, 0, st>>>(
        static_cast<Ctrl *>(s.ctrl), part, nb, cfg.courant, nullptr, 0, 0, t0, t_end, s.cur, bv,
        cfg.shard);
    return static_cast<int>(hipGetLastError());
}

// The tiled kernel for a launch (FP32 has no shared-layout, node-list or replay instances; an
// FP32 replay takes the plain instance, which checks a.dt_direct).
template <typename R>
using TileKernel = void (*)(TileArgs<R>, StepConfig, Batch);

template <typename R, int TB, bool Shared, bool Nodes>
TileKernel<R> tile_kernel_of(bool o32, bool fuse, bool replay)
{
    if constexpr (sizeof(R) == 8) {
        if (replay)
            return o32 ? tile_step_kernel<R, TB, true, false, Shared, Nodes, true>
                       : tile_step_kernel<R, TB, false, false, Shared, Nodes, true>;
    }
    return o32 ? (fuse ? tile_step_kernel<R, TB, true, true, Shared, Nodes>
                       : tile_step_kernel<R, TB, true, false, Shared, Nodes>)
               : (fuse ? tile_step_kernel<R, TB, false, true, Shared, Nodes>
                       : tile_step_kernel<R, TB, false, false, Shared, Nodes>);
}

template <typename R, int TB>
TileKernel<R> tile_kernel(bool o32, bool fuse, bool shared, bool nodes, bool replay = false)
{
    if constexpr (sizeof(R) == 8) {
        if (shared)
            return nodes ? tile_kernel_of<R, TB, true, true>(o32, fuse, replay)
                         : tile_kernel_of<R, TB, true, false>(o32, fuse, replay);
    }
    return tile_kernel_of<R, TB, false, false>(o32, fuse, replay);
}

size_t tile_lds_bytes_for(int dtype, const TileLayout &tl)
{
    return tile_lds_bytes(dtype == SWE_F64 ? 8 : 4, tl.tile, tl.max_halo, tl.max_edges,
                          tl.max_nodes);
}

int prepare_tile_kernels(size_t max_lds)
{
    for (int tile = kTileMin; tile <= kTileMax; tile *= 2) {
        const int e = with_tile(tile, [&](auto tb) {
            constexpr int TB = decltype(tb)::value;
            const void *k[22];
            int n = 0;
            for (int o32 = 0; o32 < 2; ++o32) {
                for (int fuse = 0; fuse < 2; ++fuse) {
                    k[n++] = reinterpret_cast<const void *>(tile_kernel<double, TB>(o32, fuse, false, false));
                    k[n++] = reinterpret_cast<const void *>(tile_kernel<double, TB>(o32, fuse, true, false));
                    k[n++] = reinterpret_cast<const void *>(tile_kernel<double, TB>(o32, fuse, true, true));
                    k[n++] = reinterpret_cast<const void *>(tile_kernel<float, TB>(o32, fuse, false, false));
                }
                k[n++] = reinterpret_cast<const void *>(tile_kernel<double, TB>(o32, false, false, false, true));
                k[n++] = reinterpret_cast<const void *>(tile_kernel<double, TB>(o32, false, true, false, true));
                k[n++] = reinterpret_cast<const void *>(tile_kernel<double, TB>(o32, false, true, true, true));
            }
            for (const void *f : k) {
                const hipError_t e = hipFuncSetAttribute(
                    f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(max_lds));
                if (e != hipSuccess) return static_cast<int>(e);
            }
            return static_cast<int>(hipSuccess);
        });
        if (e != hipSuccess) return e;
    }
    return static_cast<int>(hipSuccess);
}

namespace {

// Whether every array the tiled kernel indexes spans less than 4 GiB (32-bit byte offsets).
bool offsets_fit_32(const swe_dev_mesh &dm, int64_t n_cells, const TileLayout &tl)
{
    const int64_t lim = int64_t{1} << 32;
    return SWE_OFF32 && 16 * n_cells < lim && 16 * dm.n_nodes < lim &&
           16 * tl.n_tiles * static_cast<int64_t>(tl.max_edges) < lim &&
           4 * tl.n_tiles * static_cast<int64_t>(tl.max_halo) < lim &&
           16 * tl.n_tiles * static_cast<int64_t>(tl.max_nodes) < lim;
}

}  // namespace

int launch_step(int dtype, const swe_dev_mesh &dm, const StepConfig &cfg, const swe_state &s,
                int cur, const double *dt_seq, int64_t n_seq, void *stream, const TileLayout *tl,
                const BatchLaunch *batch, int remap, double *const *ustar,
                const double *dt_direct)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nb = batch ? batch->n_tiles : n_tiles_of(cfg.n_cells, cfg.tile);
    Batch bv = batch_view(batch);
    bv.remap = remap;
    bv.n_tiles = static_cast<int32_t>(nb);
    const int64_t grid = remap ? 8 * ((nb + 7) / 8) : nb;
    const Partials part = partials_for(s.work, nb);
    const bool fuse = batch == nullptr && dt_direct == nullptr && nb <= SWE_FUSE_TILES;
    const Advance adv{fuse ? static_cast<Ctrl *>(s.ctrl) : nullptr, dt_seq, n_seq, cfg.courant,
                      cfg.shard, 0};
    const int e = with_tile(cfg.tile, [&](auto tb) {
        constexpr int TB = decltype(tb)::value;
        if (tl) {
            const size_t lds = SWE_MATH_NS::tile_lds_bytes_for(dtype, *tl);
            const bool o32 = !cfg.index64 && offsets_fit_32(dm, dm.n_cells, *tl);
            if (dtype == SWE_F64) {
                TileArgs<double> ta = make_tile_args<double>(dm, s, cur, *tl);
                ta.s.part = part;
                ta.s.dt_direct = dt_direct;
                ta.s.adv = adv;
                if (ustar) {
                    ta.s.us_h = ustar[0];
                    ta.s.us_hu = ustar[1];
                    ta.s.us_hv = ustar[2];
                }
                const bool shared = tile_alias(sizeof(double), TB, tl->max_halo, tl->max_edges,
                                               tl->max_nodes);
                const bool nodes = shared && ta.edge_nodes != nullptr;
                tile_kernel<double, TB>(o32, fuse, shared, nodes, dt_direct != nullptr)
                    <<<dim3(grid), dim3(TB), lds, st>>>(ta, cfg, bv);
            } else {
                TileArgs<float> ta = make_tile_args<float>(dm, s, cur, *tl);
                ta.s.part = part;
                ta.s.dt_direct = dt_direct;
                ta.s.adv = adv;
                tile_kernel<float, TB>(o32, fuse, false, false)<<<dim3(grid), dim3(TB), lds, st>>>(
                    ta, cfg, bv);
            }
        } else if (dtype == SWE_F64) {
            StepArgs<double> a = make_args<double>(dm, s, cur);
            a.part = part;
            a.dt_direct = dt_direct;
            a.adv = adv;
            if (ustar) {
                a.us_h = ustar[0];
                a.us_hu = ustar[1];
                a.us_hv = ustar[2];
            }
            (fuse ? step_kernel<double, TB, true> : step_kernel<double, TB, false>)<<<dim3(grid), dim3(TB), 0, st>>>(
                a, cfg, bv);
        } else {
            StepArgs<float> a = make_args<float>(dm, s, cur);
            a.part = part;
            a.dt_direct = dt_direct;
            a.adv = adv;
            (fuse ? step_kernel<float, TB, true> : step_kernel<float, TB, false>)<<<dim3(grid), dim3(TB), 0, st>>>(
                a, cfg, bv);
        }
        return static_cast<int>(hipGetLastError());
    });
    if (e != hipSuccess) return e;
    if (dt_direct || fuse) return static_cast<int>(hipSuccess);   // nothing more to launch
    if (batch == nullptr && SWE_GROUP_ATOMIC)
        dt_group_fold_kernel<<<1, dim3(kPassThreads), 0, st>>>(
            static_cast<Ctrl *>(s.ctrl), part, n_slots(nb), cfg.courant, dt_seq, n_seq, cfg.shard);
    else if (batch == nullptr)
        dt_fold_kernel<<<dim3(n_groups(nb)), dim3(kGroup), 0, st>>>(
            static_cast<Ctrl *>(s.ctrl), part, nb, cfg.courant, dt_seq, n_seq, cfg.shard);
    else
        dt_pass_kernel<<<dim3(bv.n_scen), kPassThreads, 0, st>>>(
            static_cast<Ctrl *>(s.ctrl), part, nb, cfg.courant, dt_seq, n_seq, 1, 0.0, 0.0, 0, bv,
            cfg.shard);
    return static_cast<int>(hipGetLastError());
}

int launch_run_begin(const swe_state &s, const double *dt_seq, void *stream)
{
    run_begin_kernel<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(static_cast<Ctrl *>(s.ctrl),
                                                                      dt_seq);
    return static_cast<int>(hipGetLastError());
}

int launch_halo(int dtype, bool pack, int64_t n, const int32_t *idx, const void *buf_in,
                void *buf_out, const void *h, const void *hu, const void *hv, void *ho, void *huo,
                void *hvo, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    if (dtype == SWE_F64) {
        using R = double;
        halo_kernel<R><<<grid, 256, 0, st>>>(n, idx, pack ? 1 : 0, (const R *)buf_in, (R *)buf_out,
                                             (const R *)h, (const R *)hu, (const R *)hv, (R *)ho,
                                             (R *)huo, (R *)hvo);
    } else {
        using R = float;
        halo_kernel<R><<<grid, 256, 0, st>>>(n, idx, pack ? 1 : 0, (const R *)buf_in, (R *)buf_out,
                                             (const R *)h, (const R *)hu, (const R *)hv, (R *)ho,
                                             (R *)huo, (R *)hvo);
    }
    return static_cast<int>(hipGetLastError());
}

int launch_shard_combine(void *const *ctrls, int n, void *stream)
{
    ShardCtrls sc;
    for (int p = 0; p < kMaxShards; ++p) sc.c[p] = p < n ? static_cast<Ctrl *>(ctrls[p]) : nullptr;
    shard_combine_kernel<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(sc, n);
    return static_cast<int>(hipGetLastError());
}

int launch_flux_eval(int dtype, int64_t n, double g, double h_dry, const void *hl,
                     const void *hul, const void *hvl, const void *zl, const void *hr,
                     const void *hur, const void *hvr, const void *zr, const void *nx,
                     const void *ny, void *f, void *p, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nb = (n + 255) / 256;
    if (dtype == SWE_F64) {
        using R = double;
        flux_eval_kernel<R><<<dim3(nb), dim3(256), 0, st>>>(
            n, g, h_dry, (const R *)hl, (const R *)hul, (const R *)hvl, (const R *)zl,
            (const R *)hr, (const R *)hur, (const R *)hvr, (const R *)zr, (const R *)nx,
            (const R *)ny, (R *)f, (R *)p);
    } else {
        using R = float;
        flux_eval_kernel<R><<<dim3(nb), dim3(256), 0, st>>>(
            n, (R)g, (R)h_dry, (const R *)hl, (const R *)hul, (const R *)hvl, (const R *)zl,
            (const R *)hr, (const R *)hur, (const R *)hvr, (const R *)zr, (const R *)nx,
            (const R *)ny, (R *)f, (R *)p);
    }
    return static_cast<int>(hipGetLastError());
}

}  // namespace SWE_MATH_NS
}  // namespace swe
