// Host-side construction of quadrature rules used by the kernels.
#pragma once
#include <math.h>

namespace cfmm {

// Positive half of the n-point Gauss-Hermite rule (weight e^{-x^2}), n even:
// nodes are the roots of the orthonormal Hermite function h_n, bracketed by
// sign changes on a fine grid and refined by bisection; weights are the
// Christoffel numbers 1 / sum_{k<n} h_k(x)^2.
inline void gauss_hermite_half(int n, double* x, double* w)
{
    auto eval = [n](double t, double* sumsq) {
        double p0 = pow(M_PI, -0.25), p1 = sqrt(2.0) * t * p0;
        double s = p0 * p0 + p1 * p1;
        double pm = p0, pk = p1;
        for (int k = 1; k < n; ++k) {
            double pn = sqrt(2.0 / (k + 1)) * t * pk - sqrt((double)k / (k + 1)) * pm;
            pm = pk;
            pk = pn;
            if (k + 1 < n) s += pk * pk;
        }
        if (sumsq) *sumsq = s;
        return pk;   // orthonormal h_n(t) up to the weight factor
    };
    int half = n / 2, found = 0;
    double step = 1e-3, hi = sqrt(2.0 * n + 1.0) + 1.0;
    double a = 1e-9, fa = eval(a, nullptr);
    for (double b = a + step; b < hi && found < half; b += step) {
        double fb = eval(b, nullptr);
        if ((fa < 0) != (fb < 0)) {
            double lo = a, up = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + up);
                if (mid == lo || mid == up) break;
                double fm = eval(mid, nullptr);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else up = mid;
            }
            double r = 0.5 * (lo + up), ss;
            eval(r, &ss);
            x[found] = r;
            w[found] = 1.0 / ss;
            ++found;
        }
        a = b;
        fa = fb;
    }
}

}  // namespace cfmm
