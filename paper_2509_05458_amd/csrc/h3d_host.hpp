// Host-side plan-time mathematics of the 3D Helmholtz path: spherical Bessel
// functions of real argument, Gauss-Legendre rules and the per-level tables of
// the sampled translations (Sec. 5.3, the point-and-shoot translations).
#pragma once

#include <vector>

namespace cfmm {

// j_n(x), y_n(x) and their derivatives for n = 0..nmax, real x > 0.
void sph_bessel_real(int nmax, double x, double* j, double* y, double* jd, double* yd);

// n-point Gauss-Legendre rule on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, double* x, double* w);

// Smallest n >= 1 with |h_n(kR) j_n(kr)| <= eps at n and n+1, R = (0.5+k) w,
// r = sqrt(3)/2 w (Sec. 6.3); pmax + 1 if none up to pmax qualifies.
int h3d_nterms(double kappa, double w, int sep, double eps, int pmax);

// Schmidt-normalised S_n^m at the unit vector (sin t, 0, cos t) for n <= P,
// 0 <= m <= n, indexed n(n+1)/2 + m (real).
void schmidt_column_table(int P, double cth, double sth, double* out);

// Equator constants: S_n^m(e_x) and its derivative along (0, 0, -1),
// indexed n(n+1)/2 + m for n <= P.
void equator_table(int P, double* p0, double* d0);

}  // namespace cfmm
