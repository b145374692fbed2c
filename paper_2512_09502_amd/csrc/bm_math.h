// Double-precision pieces of the Box-Muller normal for 32-bit uniform words,
// written for the arguments that occur there (usable on host and device):
// ln(v / 2^32) for integer v in [1, 2^32] and cos(2 pi w / 2^32) for a word w.
// Both reduce their argument exactly with integer operations, so only short
// polynomials remain (Taylor series of atanh, sin and cos, truncated below
// 2^-56 on the reduced ranges).
#pragma once

#include <cmath>
#include <cstdint>

#ifndef __HIPCC__
#define SNNC_HD inline
#else
#define SNNC_HD __host__ __device__ __forceinline__
#endif

namespace snnc {

// ln(v / 2^32), v in [1, 2^32].  v = m 2^e with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716; ln 2 in two parts
// so that e ln2_hi is exact.
SNNC_HD double log_u32_frac(uint64_t v) {
    const double ln2_hi = 0.6931471803691238;      // ln 2 with 32 significant bits
    const double ln2_lo = 1.9082149292705877e-10;  // ln 2 - ln2_hi
    int e = 63 - __builtin_clzll(v);               // v >= 1
    double m = ldexp((double)v, -e);               // exact
    if (m > 1.4142135623730951) {
        m *= 0.5;
        e += 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    // atanh(s) / s = sum z^k / (2k + 1), k = 0 .. 11
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    const double ln_m = 2.0 * s + 2.0 * s * (z * p);
    const double k = (double)(e - 32);
    return k * ln2_hi + (k * ln2_lo + ln_m);
}

// sin and cos of b in [0, pi/4] by their Taylor series (b^2 <= 0.617)
SNNC_HD double sin_quarter(double b) {
    const double z = b * b;
    // sin b = b - b^3/3! + b^5/5! - ... (to b^19)
    double q = -1.0 / 121645100408832000.0;        // -1/19!
    q = q * z + 1.0 / 355687428096000.0;           //  1/17!
    q = q * z - 1.0 / 1307674368000.0;             // -1/15!
    q = q * z + 1.0 / 6227020800.0;                //  1/13!
    q = q * z - 1.0 / 39916800.0;                  // -1/11!
    q = q * z + 1.0 / 362880.0;                    //  1/9!
    q = q * z - 1.0 / 5040.0;                      // -1/7!
    q = q * z + 1.0 / 120.0;                       //  1/5!
    q = q * z - 1.0 / 6.0;                         // -1/3!
    return b + b * (z * q);
}

SNNC_HD double cos_quarter(double b) {
    const double z = b * b;
    // cos b = 1 - b^2/2! + b^4/4! - ... (to b^18)
    double p = 1.0 / 6402373705728000.0;           //  1/18!
    p = p * z - 1.0 / 20922789888000.0;            // -1/16!
    p = p * z + 1.0 / 87178291200.0;               //  1/14!
    p = p * z - 1.0 / 479001600.0;                 // -1/12!
    p = p * z + 1.0 / 3628800.0;                   //  1/10!
    p = p * z - 1.0 / 40320.0;                     // -1/8!
    p = p * z + 1.0 / 720.0;                       //  1/6!
    p = p * z - 1.0 / 24.0;                        // -1/4!
    p = p * z + 1.0 / 2.0;                         //  1/2!
    return 1.0 - z * p;
}

// cos(x) for x = fl(2pi_d * w / 2^32), the argument as a double product
// (2pi_d = 2 pi rounded to double), as Box-Muller in double precision forms
// it.  theta = 2 pi w / 2^32 is reduced exactly: quadrant q = w >> 30, the
// offset r inside it folded to [0, pi/4] (cos a = sin(pi/2 - a)); then
// x = theta + corr with corr = (2pi_d - 2 pi) u + (the product's rounding
// error, exact by a fused multiply-add), so cos x = cos theta - corr sin theta
// (corr <= 1e-15: the next term is below 1e-30).
SNNC_HD double cos_2pi_u32(uint32_t w) {
    const double two_pi_over_2_32 = 1.4629180792671596e-09;   // 2 pi / 2^32
    const double two_pi_d = 6.283185307179586;                 // 2 pi rounded to double
    const double two_pi_err = -2.4492935982947064e-16;         // two_pi_d - 2 pi
    const uint32_t q = w >> 30;
    const uint32_t r = w & 0x3fffffffu;
    const bool low = r < (1u << 29);
    const uint32_t g = low ? r : (1u << 30) - r;
    const double b = (double)g * two_pi_over_2_32;
    const double cb = cos_quarter(b), sb = sin_quarter(b);
    const double ca = low ? cb : sb;   // cos a, a = 2 pi r / 2^32
    const double sa = low ? sb : cb;   // sin a
    double ct, st;                     // cos theta, sin theta
    switch (q) {
    case 0: ct = ca; st = sa; break;
    case 1: ct = -sa; st = ca; break;
    case 2: ct = -ca; st = -sa; break;
    default: ct = sa; st = -ca; break;
    }
    const double u = (double)w * (1.0 / 4294967296.0);
    const double x = two_pi_d * u;
    const double corr = two_pi_err * u - fma(two_pi_d, u, -x);   // x - 2 pi u
    return ct - st * corr;
}

}  // namespace snnc
