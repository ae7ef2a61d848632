// Shared definitions of the cfmm HIP library: complex arithmetic and limits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#define CFMM_HD __host__ __device__ inline

namespace cfmm {

constexpr int kPMax2D = 63;          // 2D expansions hold 2P+1 <= 127 coefficients
constexpr int kNCoef2DMax = 2 * kPMax2D + 1;
constexpr int kPMax3D = 40;          // 3D expansions hold (P+1)^2 coefficients
constexpr int kPMaxH3 = 50;          // 3D Helmholtz expansion length limit
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEuler = 0.57721566490153286060651209008240243;
constexpr int kGHHalf = 24;          // 48-point Gauss-Hermite rule, positive half

struct cplx {
    double re, im;
};

CFMM_HD cplx mk(double r, double i) { return cplx{r, i}; }
CFMM_HD cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
CFMM_HD cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
CFMM_HD cplx operator-(cplx a) { return cplx{-a.re, -a.im}; }
CFMM_HD cplx operator*(cplx a, cplx b)
{
    return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
CFMM_HD cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
CFMM_HD cplx operator*(cplx a, double s) { return cplx{s * a.re, s * a.im}; }
CFMM_HD cplx& operator+=(cplx& a, cplx b) { a.re += b.re; a.im += b.im; return a; }
CFMM_HD cplx& operator-=(cplx& a, cplx b) { a.re -= b.re; a.im -= b.im; return a; }
CFMM_HD cplx& operator*=(cplx& a, cplx b) { a = a * b; return a; }
CFMM_HD cplx& operator*=(cplx& a, double s) { a.re *= s; a.im *= s; return a; }
// acc += a * b as four fused multiply-adds (no separate product rounding)
CFMM_HD void cfma(cplx& acc, cplx a, cplx b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
CFMM_HD double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
CFMM_HD double cabs1(cplx a) { return hypot(a.re, a.im); }
CFMM_HD cplx conj(cplx a) { return cplx{a.re, -a.im}; }
CFMM_HD cplx times_i(cplx a) { return cplx{-a.im, a.re}; }

// a / b with scaling (Smith's algorithm)
CFMM_HD cplx cdiv(cplx a, cplx b)
{
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return cplx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    double r = b.re / b.im, d = b.re * r + b.im;
    return cplx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
CFMM_HD cplx cinv(cplx b) { return cdiv(cplx{1.0, 0.0}, b); }

// principal square root, Re >= 0
CFMM_HD cplx csqrt_p(cplx a)
{
    if (a.re == 0.0 && a.im == 0.0) return cplx{0.0, 0.0};
    double m = hypot(a.re, a.im);
    if (a.re >= 0.0) {
        double t = sqrt(0.5 * (m + a.re));
        return cplx{t, a.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (m - a.re));
    return cplx{fabs(a.im) / (2.0 * t), copysign(t, a.im)};
}

// principal logarithm
CFMM_HD cplx clog_p(cplx a) { return cplx{log(hypot(a.re, a.im)), atan2(a.im, a.re)}; }

CFMM_HD cplx cexp_(cplx a)
{
    double e = exp(a.re), s, c;
    sincos(a.im, &s, &c);
    return cplx{e * c, e * s};
}

// sin and cos of x for |x| < 2^20 (the phases of near fields and radial
// functions, which the expansion-length limit keeps far below that):
// Cody-Waite reduction x = k pi/2 + t with pi/2 split into a 33-bit head
// (k * head is exact) and its tail, |t| <= pi/4, then the Taylor series of
// sin t to t^17 and of cos t to t^18 (truncation below 1e-19 relative), and
// the quadrant k mod 4.  The constants are pi/2 and its head and tail,
// computed from pi to 60 digits; the series coefficients are 1/n!.
__device__ inline void sincos_cw(double x, double* sn, double* cs)
{
    const double two_over_pi = 0.6366197723675814;
    const double pio2_hi = 1.5707963267341256;
    const double pio2_lo = 6.077100506506192e-11;
    double k = rint(x * two_over_pi);
    double t = fma(-k, pio2_lo, fma(-k, pio2_hi, x));
    double t2 = t * t;
    double ps = 1.0 / 355687428096000.0;                    // 1/17!
    ps = fma(ps, t2, -1.0 / 1307674368000.0);               // -1/15!
    ps = fma(ps, t2, 1.0 / 6227020800.0);
    ps = fma(ps, t2, -1.0 / 39916800.0);
    ps = fma(ps, t2, 1.0 / 362880.0);
    ps = fma(ps, t2, -1.0 / 5040.0);
    ps = fma(ps, t2, 1.0 / 120.0);
    ps = fma(ps, t2, -1.0 / 6.0);
    double st = fma(ps * t2, t, t);
    double pc = 1.0 / 6402373705728000.0;                   // 1/18!
    pc = fma(pc, t2, -1.0 / 20922789888000.0);              // -1/16!
    pc = fma(pc, t2, 1.0 / 87178291200.0);
    pc = fma(pc, t2, -1.0 / 479001600.0);
    pc = fma(pc, t2, 1.0 / 3628800.0);
    pc = fma(pc, t2, -1.0 / 40320.0);
    pc = fma(pc, t2, 1.0 / 720.0);
    pc = fma(pc, t2, -1.0 / 24.0);
    pc = fma(pc, t2, 0.5);
    double ct = fma(-pc, t2, 1.0);
    int q = (int)k & 3;
    double s0 = (q & 1) ? ct : st, c0 = (q & 1) ? st : ct;
    *sn = (q & 2) ? -s0 : s0;
    *cs = ((q + 1) & 2) ? -c0 : c0;
}

// exp(y): y = k ln2 + t with ln 2 split as pi/2 above, |t| <= ln2/2, the
// Taylor series of e^t to t^13 (truncation below 5e-18 relative), times 2^k
// (which gives 0 and inf beyond the double range, as exp does).
__device__ inline double exp_cw(double y)
{
    const double inv_ln2 = 1.4426950408889634;
    const double ln2_hi = 0.6931471804855391;
    const double ln2_lo = 7.440617110012397e-11;
    double k = rint(y * inv_ln2);
    double t = fma(-k, ln2_lo, fma(-k, ln2_hi, y));
    double p = 1.0 / 6227020800.0;                          // 1/13!
    p = fma(p, t, 1.0 / 479001600.0);
    p = fma(p, t, 1.0 / 39916800.0);
    p = fma(p, t, 1.0 / 3628800.0);
    p = fma(p, t, 1.0 / 362880.0);
    p = fma(p, t, 1.0 / 40320.0);
    p = fma(p, t, 1.0 / 5040.0);
    p = fma(p, t, 1.0 / 720.0);
    p = fma(p, t, 1.0 / 120.0);
    p = fma(p, t, 1.0 / 24.0);
    p = fma(p, t, 1.0 / 6.0);
    p = fma(p, t, 0.5);
    p = fma(p, t, 1.0);
    p = fma(p, t, 1.0);
    return ldexp(p, (int)k);
}

// e^a for complex a with |Im a| < 2^20.
__device__ inline cplx cexp_cw(cplx a)
{
    double s, c;
    sincos_cw(a.im, &s, &c);
    double e = exp_cw(a.re);
    return cplx{e * c, e * s};
}

// Workgroup i of a grid of n is dispatched to XCD i mod 8; this returns a
// work index such that each XCD takes one contiguous range of [0, n), so that
// neighbouring work items (which share their inputs) share one L2.
__device__ inline int xcd_contiguous(int i, int n)
{
    int q = n >> 3, r = n & 7, x = i & 7;
    return x * q + (x < r ? x : r) + (i >> 3);
}

}  // namespace cfmm
