// Binary64 logarithm, cosine of 2 pi u and exponential for the
// secondary-uncertainty draws (x = exp(m + s sqrt(-2 ln u1) cos(2 pi u2))).
//
// Written out rather than taken from the device math library: the library's
// versions serve every argument (double-double steps, a Payne-Hanek path for
// huge angles) and carry a few dozen binary64 constants, which in the draw
// loop cost as many instructions as the rest of the draw and the registers
// that hold them.  Here each function is a Cody-Waite argument reduction
// (W. J. Cody and W. Waite, Software Manual for the Elementary Functions,
// 1980) and a Taylor polynomial in Horner form, with the terms taken until
// the first omitted one is below 2^-55 of the result on the reduced range:
//   log x    x = m 2^e, m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
//            ln m = 2 atanh s = 2 (s + s^3/3 + ... + s^19/19), |s| <= 0.1716;
//   cos 2pu  a = fl(2 pi u) (the rounded product the definition names),
//            a = k pi/2 + r, |r| <= pi/4 (pi/2 in three parts, the first two
//            of 33 bits, so k * part is exact for k <= 4), then +-cos r or
//            +-sin r by the quadrant k, cos to r^16, sin to r^17;
//   exp y    y = n ln2 + r, |r| <= ln2/2 (ln 2 in two parts, the first of 32
//            bits), e^r to r^13, times 2^n.
// Every step is an IEEE operation (fma, division, frexp, ldexp, rint), so
// the same code compiled for the host gives the device's results bit for
// bit; a host test measures the error against the C library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace ara {

namespace sumath {
constexpr double kTwoPi = 0x1.921fb54442d18p+2;      // binary64 nearest 2 pi
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;  // binary64 nearest 2 / pi
constexpr double kPio2A = 0x1.921fb544p+0;           // pi/2 = A + B + C
constexpr double kPio2B = 0x1.0b4611a6p-34;
constexpr double kPio2C = 0x1.3198a2e037073p-69;
constexpr double kLn2Hi = 0x1.62e42feep-1;           // ln 2 = Hi + Lo
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kLog2e = 0x1.71547652b82fep+0;      // binary64 nearest 1 / ln 2
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;   // binary64 nearest sqrt(1/2)
}  // namespace sumath

// Natural logarithm of a positive normal x.
__host__ __device__ inline double su_log(double x) {
    using namespace sumath;
    int e;
    double m = std::frexp(x, &e);   // x = m 2^e, m in [1/2, 1)
    if (m < kSqrtHalf) {
        m += m;
        --e;
    }
    const double f = m - 1.0;       // exact (Sterbenz)
    const double s = f / (2.0 + f);
    const double z = s * s;
    // (atanh(s) - s) / s^3 = 1/3 + z/5 + ... + z^8/19
    double p = 1.0 / 19.0;
    p = std::fma(p, z, 1.0 / 17.0);
    p = std::fma(p, z, 1.0 / 15.0);
    p = std::fma(p, z, 1.0 / 13.0);
    p = std::fma(p, z, 1.0 / 11.0);
    p = std::fma(p, z, 1.0 / 9.0);
    p = std::fma(p, z, 1.0 / 7.0);
    p = std::fma(p, z, 1.0 / 5.0);
    p = std::fma(p, z, 1.0 / 3.0);
    const double lm = 2.0 * std::fma(s * z, p, s);   // ln m
    const double de = static_cast<double>(e);
    return std::fma(de, kLn2Hi, std::fma(de, kLn2Lo, lm));
}

// cos(fl(2 pi u)) for u in [0, 1].
__host__ __device__ inline double su_cos_2pi(double u) {
    using namespace sumath;
    const double a = kTwoPi * u;
    const double k = std::rint(a * kTwoOverPi);   // quadrant, 0 .. 4
    double r = std::fma(-k, kPio2A, a);
    r = std::fma(-k, kPio2B, r);
    r = std::fma(-k, kPio2C, r);
    const double r2 = r * r;
    double c = 1.0 / 20922789888000.0;            // 1/16!
    c = std::fma(c, r2, -1.0 / 87178291200.0);    // 1/14!
    c = std::fma(c, r2, 1.0 / 479001600.0);       // 1/12!
    c = std::fma(c, r2, -1.0 / 3628800.0);        // 1/10!
    c = std::fma(c, r2, 1.0 / 40320.0);           // 1/8!
    c = std::fma(c, r2, -1.0 / 720.0);            // 1/6!
    c = std::fma(c, r2, 1.0 / 24.0);
    c = std::fma(c, r2, -0.5);
    c = std::fma(c, r2, 1.0);                     // cos r
    double sn = 1.0 / 355687428096000.0;          // 1/17!
    sn = std::fma(sn, r2, -1.0 / 1307674368000.0);   // 1/15!
    sn = std::fma(sn, r2, 1.0 / 6227020800.0);    // 1/13!
    sn = std::fma(sn, r2, -1.0 / 39916800.0);     // 1/11!
    sn = std::fma(sn, r2, 1.0 / 362880.0);        // 1/9!
    sn = std::fma(sn, r2, -1.0 / 5040.0);         // 1/7!
    sn = std::fma(sn, r2, 1.0 / 120.0);
    sn = std::fma(sn, r2, -1.0 / 6.0);
    sn = std::fma(r * r2, sn, r);                 // sin r
    const int q = static_cast<int>(k) & 3;        // cos(r + q pi/2) = cos r, -sin r, -cos r, sin r
    const double v = (q & 1) ? sn : c;
    return (q == 1 || q == 2) ? -v : v;
}

// e^y (0 below -760, infinity above 720).
__host__ __device__ inline double su_exp(double y) {
    using namespace sumath;
    y = std::fmin(std::fmax(y, -760.0), 720.0);
    const double n = std::rint(y * kLog2e);
    double r = std::fma(-n, kLn2Hi, y);
    r = std::fma(-n, kLn2Lo, r);
    double p = 1.0 / 6227020800.0;                // 1/13!
    p = std::fma(p, r, 1.0 / 479001600.0);        // 1/12!
    p = std::fma(p, r, 1.0 / 39916800.0);         // 1/11!
    p = std::fma(p, r, 1.0 / 3628800.0);          // 1/10!
    p = std::fma(p, r, 1.0 / 362880.0);           // 1/9!
    p = std::fma(p, r, 1.0 / 40320.0);            // 1/8!
    p = std::fma(p, r, 1.0 / 5040.0);             // 1/7!
    p = std::fma(p, r, 1.0 / 720.0);              // 1/6!
    p = std::fma(p, r, 1.0 / 120.0);
    p = std::fma(p, r, 1.0 / 24.0);
    p = std::fma(p, r, 1.0 / 6.0);
    p = std::fma(p, r, 0.5);
    p = std::fma(p, r, 1.0);
    p = std::fma(p, r, 1.0);
    return std::ldexp(p, static_cast<int>(n));
}

}  // namespace ara
