// Device math shared by the step and adjoint kernels of libswe.
#pragma once

#include <hip/hip_runtime.h>

namespace swe {

// FP64 division by the hardware reciprocal refined by two Newton steps, the quotient by one
// residual correction: within an ulp of the correctly rounded quotient for normal operands,
// odd in each argument.
__device__ __forceinline__ double div_nr(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    const double q = a * r;
    const double rem = fma(-b, q, a);
    return fma(rem, r, q);
}

// FP64 reciprocal by the hardware reciprocal refined by two Newton steps, for several
// quotients by one divisor (each then a single product, within about an ulp); odd in b.
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}

// a / b from ir = rcp_nr(b): the product refined by one residual step, within an ulp of the
// quotient (nearly always the correctly rounded one); odd in a, and in b with ir.
__device__ __forceinline__ double quot_nr(double a, double ir, double b)
{
    const double q = a * ir;
    return fma(fma(-b, q, a), ir, q);
}

// Length l = sqrt(s) (within an ulp, residual-corrected as sqrt_nr) and its reciprocal
// il = 1/l (within about an ulp) of a positive normal s, both from one hardware reciprocal
// square root refined by Goldschmidt's iteration, g -> sqrt(s) and h -> 1/(2 sqrt(s)), and one
// more step of h against the corrected root.
__device__ __forceinline__ void len_rcp_nr(double s, double &l, double &il)
{
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, s);
    l = fma(d, h, g);
    const double r2 = fma(-l, h, 0.5);
    h = fma(h, r2, h);
    il = h + h;
}

// FP64 square root by the hardware reciprocal square root refined by Goldschmidt's iteration
// and one residual correction: within an ulp of the correctly rounded root; sqrt(0) = 0.
__device__ __forceinline__ double sqrt_nr(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, a);
    g = fma(d, h, g);
    return a > 0.0 ? g : a;   // rsq(0) is inf
}

// Cube root of a positive normal argument by Newton's iteration for r = x^(-1/3), which needs
// no division: r <- r + r (1 - x r^3) / 3, from the single-precision seed 2^(-log2(x) / 3) (the
// hardware log2 and exp2, relative error a few 1e-6 over the range taken here).  A seed error
// e becomes -2 e^2 (about 1e-10) after one step; cbrt(x) = x r^2 with one residual correction
// c <- c - (c^3 - x) r^2 / 3, which squares the error again, below the double rounding.  Zero,
// tiny, huge and non-finite arguments take the library cbrt.
__device__ __forceinline__ double cbrt_(double x)
{
    if (!(x > 0x1p-120 && x < 0x1p120)) return cbrt(x);
    double r = static_cast<double>(
        __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(static_cast<float>(x)) * (-1.0f / 3.0f)));
    const double third = 1.0 / 3.0;
    {
        const double e = fma(-x * r, r * r, 1.0);
        r = fma(r * third, e, r);
    }
    const double r2 = r * r;
    const double c = x * r2;
    const double t = fma(c * c, c, -x);
    return fma(-t * third, r2, c);
}

__device__ __forceinline__ float cbrt_(float x)
{
    if (!(x > 0x1p-100f && x < 0x1p100f)) return cbrtf(x);
    float r = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (-1.0f / 3.0f));
    const float e = fmaf(-x * r, r * r, 1.0f);
    r = fmaf(r * (1.0f / 3.0f), e, r);
    const float r2 = r * r;
    const float c = x * r2;
    const float t = fmaf(c * c, c, -x);
    return fmaf(-t * (1.0f / 3.0f), r2, c);
}

}  // namespace swe
