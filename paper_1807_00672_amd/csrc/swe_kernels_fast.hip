// The kernels of swe_kernels.hip compiled a second time, into swe::fast: FP64 division by the
// hardware reciprocal with two Newton steps and a residual correction, FP64 square root by the
// hardware reciprocal square root with Goldschmidt's iteration and a residual correction (both
// within an ulp of the correctly rounded result, and odd in their sign arguments, so interface
// fluxes stay exact negatives of each other).
#define SWE_F64_FAST 1
#define SWE_MATH_NS fast
#include "swe_kernels.hip"
