// Host-side plan-time mathematics of the 3D Helmholtz path.
#include "h3d_host.hpp"

#include <math.h>

#include <algorithm>
#include <vector>

namespace cfmm {

namespace {

// j_n for n <= nmax by the power series j_n(x) = x^n/(2n+1)!! sum_k (-x^2/2)^k
// / (k! prod_{i<=k} (2n+2i+1)) at the two top orders, then downward
// recurrence (stable for the regular solution); valid while x^2 is small
// next to 2(2 nmax + 5), so the series has no cancellation.
template <class T>
void jn_series_down(int nmax, T x, T* j)
{
    auto series = [&](int n) {
        T pref = 1.0;
        for (int i = 1; i <= n; ++i) pref *= x / (T)(2.0 * i + 1.0);
        T term = 1.0, sum = 1.0, q = -(T)0.5 * x * x;
        for (int k = 1; k < 200; ++k) {
            term *= q / (T)((double)k * (2.0 * n + 2.0 * k + 1.0));
            sum += term;
            if (fabsl(term) < 1e-18L * fabsl(sum)) break;
        }
        return pref * sum;
    };
    j[nmax] = series(nmax);
    if (nmax == 0) return;
    j[nmax - 1] = series(nmax - 1);
    for (int n = nmax - 1; n >= 1; --n) j[n - 1] = (T)(2.0 * n + 1.0) / x * j[n] - j[n + 1];
}

// j_n by Miller's backward recurrence normalised on j_0 and j_1 (least squares
// on both, so a zero of either costs nothing).
template <class T>
void jn_miller(int nmax, T x, T* j)
{
    int start = nmax + 20 + (int)(x);
    std::vector<T> t(start + 2, 0.0);
    t[start + 1] = 0.0;
    t[start] = 1e-30;
    for (int n = start; n >= 1; --n) {
        t[n - 1] = (T)(2.0 * n + 1.0) / x * t[n] - t[n + 1];
        if (fabsl(t[n - 1]) > 1e250L) {
            for (int k = n - 1; k <= start; ++k) t[k] *= (T)1e-250L;
        }
    }
    T j0 = sinl(x) / x, j1 = sinl(x) / (x * x) - cosl(x) / x;
    T nrm = std::max(fabsl(t[0]), fabsl(t[1]));
    T a0 = t[0] / nrm, a1 = t[1] / nrm;
    T s = (j0 * a0 + j1 * a1) / (a0 * a0 + a1 * a1) / nrm;
    for (int n = 0; n <= nmax; ++n) j[n] = s * t[n];
}

// j_n and y_n for n <= nmax + 1 in the arithmetic T
template <class T>
void sph_jy(int nmax, T x, T* jj, T* yy)
{
    if (x * x < (T)(2.0 * (2.0 * (nmax + 1) + 5.0))) jn_series_down<T>(nmax + 1, x, jj);
    else jn_miller<T>(nmax + 1, x, jj);
    yy[0] = -cosl(x) / x;
    if (nmax + 1 >= 1) yy[1] = -cosl(x) / (x * x) - sinl(x) / x;
    for (int n = 1; n <= nmax; ++n) yy[n + 1] = (T)(2.0 * n + 1.0) / x * yy[n] - yy[n - 1];
}

}  // namespace

void sph_bessel_real(int nmax, double x, double* j, double* y, double* jd, double* yd)
{
    std::vector<long double> jj(nmax + 2), yy(nmax + 2);
    sph_jy<long double>(nmax, x, jj.data(), yy.data());
    for (int n = 0; n <= nmax; ++n) {
        if (j) j[n] = (double)jj[n];
        if (y) y[n] = (double)yy[n];
        if (jd) jd[n] = (double)(n / (long double)x * jj[n] - jj[n + 1]);
        if (yd) yd[n] = (double)(n / (long double)x * yy[n] - yy[n + 1]);
    }
}

void gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

int h3d_nterms(double kappa, double w, int sep, double eps, int pmax)
{
    // in x87 extended precision: at small kappa w, |h_n(kR)| ~ (2n-1)!!/(kR)^(n+1)
    // and j_n(kr) ~ (kr)^n/(2n+1)!! leave the FP64 range long before n = pmax
    double R = (0.5 + sep) * w, r = sqrt(3.0) * 0.5 * w;
    std::vector<long double> jR(pmax + 4), yR(pmax + 4), jr(pmax + 4), yr(pmax + 4);   // orders 0 .. pmax + 3
    sph_jy<long double>(pmax + 2, (long double)kappa * R, jR.data(), yR.data());
    sph_jy<long double>(pmax + 2, (long double)kappa * r, jr.data(), yr.data());
    auto crit = [&](int n) { return sqrtl(jR[n] * jR[n] + yR[n] * yR[n]) * fabsl(jr[n]); };
    for (int n = 1; n <= pmax; ++n)
        if (crit(n) <= eps && crit(n + 1) <= eps) return n;
    return pmax + 1;
}

// Column recurrence of the Schmidt-normalised solid harmonics at a unit vector
// with w = x + iy real (y = 0): S_m^m = c_m x^m, then
// S_n^m = ((2n-1) z S_{n-1}^m - sqrt((n+m-1)(n-m-1)) S_{n-2}^m) / sqrt((n-m)(n+m)).
void schmidt_column_table(int P, double cth, double sth, double* out)
{
    double d = 1.0;
    for (int m = 0; m <= P; ++m) {
        if (m > 0) d *= sth * sqrt((2.0 * m - 1.0) / (2.0 * m));
        double a = d;
        out[m * (m + 1) / 2 + m] = a;
        if (m + 1 > P) continue;
        double b = sqrt(2.0 * m + 1.0) * cth * d;
        out[(m + 1) * (m + 2) / 2 + m] = b;
        for (int n = m + 2; n <= P; ++n) {
            double c = ((2.0 * n - 1.0) * cth * b - sqrt((double)(n + m - 1) * (n - m - 1)) * a) /
                       sqrt((double)(n - m) * (n + m));
            out[n * (n + 1) / 2 + m] = c;
            a = b;
            b = c;
        }
    }
}

// At e_x: z = 0, w = 1; along v = (0, 0, -1): dw = 0, dz = -1 (tangent, so r^2
// is constant to first order).
void equator_table(int P, double* p0, double* d0)
{
    double d = 1.0;
    for (int m = 0; m <= P; ++m) {
        if (m > 0) d *= sqrt((2.0 * m - 1.0) / (2.0 * m));
        double q0 = 1.0, dq0 = 0.0;
        p0[m * (m + 1) / 2 + m] = d * q0;
        d0[m * (m + 1) / 2 + m] = d * dq0;
        if (m + 1 > P) continue;
        double q1 = 0.0, dq1 = -sqrt(2.0 * m + 1.0);
        p0[(m + 1) * (m + 2) / 2 + m] = d * q1;
        d0[(m + 1) * (m + 2) / 2 + m] = d * dq1;
        for (int n = m + 2; n <= P; ++n) {
            double e = sqrt((double)(n + m - 1) * (n - m - 1)), f = sqrt((double)(n - m) * (n + m));
            double q2 = (0.0 - e * q0) / f;
            double dq2 = ((2.0 * n - 1.0) * (-1.0 * q1 + 0.0 * dq1) - e * dq0) / f;
            p0[n * (n + 1) / 2 + m] = d * q2;
            d0[n * (n + 1) / 2 + m] = d * dq2;
            q0 = q1; q1 = q2; dq0 = dq1; dq1 = dq2;
        }
    }
}

}  // namespace cfmm
