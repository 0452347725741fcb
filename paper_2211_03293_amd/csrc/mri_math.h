// mri_math.h -- device math shared by the fast-stage kernels.
#pragma once

// 2^t for finite |t| < 1022.
//
// Method: t = n + f with n = rint(t) and |f| <= 1/2; 2^f from the degree-11
// polynomial interpolating 2^f at the 12 Chebyshev nodes of [-1/2, 1/2]
// (near-minimax; interpolation error below 3e-18 relative), evaluated by
// Horner's rule with fused multiply-adds; 2^n applied exactly with ldexp.
// Error <= ~1 ulp over the domain.  The coefficients were obtained by solving
// the interpolation conditions in 40-digit decimal arithmetic and rounding to
// double.  There are no range clamps: the kernels' exponents are bounded by
// construction (checked at mechanism creation for T >= 200 K); a NaN argument
// returns NaN and very large |t| saturate through the integer conversion to
// inf or 0.
__device__ __forceinline__ double mri_exp2(double t)
{
    const double n = __builtin_rint(t);
    const double f = t - n;                      // exact
    double p = fma(f, 0x1.e9ec1fcb69a7fp-32, 0x1.e6228acd1c6e5p-28);
    p = fma(p, f, 0x1.b524ebd13a55fp-24);
    p = fma(p, f, 0x1.62bfc2c86d700p-20);
    p = fma(p, f, 0x1.ffcbfc6da6ed1p-17);
    p = fma(p, f, 0x1.430913112c61bp-13);
    p = fma(p, f, 0x1.5d87fe78a3f9cp-10);
    p = fma(p, f, 0x1.3b2ab6fb9f1a5p-7);
    p = fma(p, f, 0x1.c6b08d704a0c6p-5);
    p = fma(p, f, 0x1.ebfbdff82c5aep-3);
    p = fma(p, f, 0x1.62e42fefa39efp-1);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)n);
}
