/*
 * ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct FP64 direct evaluation of the discrete
 * single-layer sum the complex-coordinate FMM approximates:
 *
 *     u(x_i) = sum_j G(x_i, y_j) sigma_j                    (Sec. 2.3, eq. for
 *                                                            the M-body sum)
 *
 * at complex points x, y in C^d, with the complexified distance
 * r = sqrt(sum_d (x_d - y_d)^2) on the principal branch (Sec. 2.1 and the
 * complex polar / spherical coordinates of Sec. 3.1: Re r > 0 under the
 * Lipschitz assumptions of Sec. 4.1 / 5.1).  Kernels, with the constants of
 * the standard free-space Green's functions:
 *
 *     2D Helmholtz  G = (i/4) H0^(1)(kappa r)          (Sec. 2.1, Sec. 4.3)
 *     2D Laplace    G = -(1/(2 pi)) log r              (Sec. 4.2)
 *     3D Laplace    G = 1/(4 pi r)                     (Sec. 5.2)
 *     3D Helmholtz  G = exp(i kappa r)/(4 pi r)        (Sec. 5.3)
 *
 * Self pairs (the target is the source itself) are skipped; a pair whose
 * squared distance is exactly zero contributes nothing.
 *
 * Each target is summed over sources in index order with Neumaier
 * compensated summation of the real and the imaginary parts.
 *
 * The complex Hankel function H0^(1) is this file's own:
 *   |z| <= 2.5 : power series of J0 and Y0 (DLMF 10.2.2, 10.8.2);
 *   |z| >= 25  : Hankel's asymptotic expansion (DLMF 10.17.5);
 *   otherwise  : Taylor-series continuation of Bessel's equation
 *                z^2 w'' + z w' + z^2 w = 0 from the asymptotic region,
 *                along a vertical path on which H0^(1) is the dominant
 *                solution (Im z decreasing), so the continuation is stable.
 * Valid for Re z > 0, |arg z| <= 60 degrees.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
 * file.  It shares no code with the HIP library.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_PI 3.14159265358979323846264338327950288
#define OR_EULER 0.57721566490153286060651209008240243

enum { OR_LAPLACE = 0, OR_HELMHOLTZ = 1 };

/* ---------------------------------------------------------------- Bessel */

/* J0, Y0 power series, H0 = J0 + i Y0.  q = z^2/4,
 * J0 = sum (-q)^k/(k!)^2,  Y0 = (2/pi)[(log(z/2)+gamma) J0 - sum_{k>=1} H_k (-q)^k/(k!)^2]
 * with H_k the harmonic numbers. */
static cplx h0_series(cplx z)
{
    cplx q = z * z * 0.25;
    cplx t = 1.0, j0 = 1.0, s = 0.0;
    double hk = 0.0;
    for (int k = 1; k < 200; ++k) {
        t *= -q / ((double)k * (double)k);
        hk += 1.0 / k;
        j0 += t;
        s += hk * t;
        if (cabs(t) * hk < 1e-18 * (cabs(j0) + cabs(s)) && k > cabs(q)) break;
    }
    cplx y0 = (2.0 / OR_PI) * ((clog(z * 0.5) + OR_EULER) * j0 - s);
    return j0 + I * y0;
}

/* Hankel's expansion for H_nu^(1), nu = 0 and 1:
 * H_nu ~ sqrt(2/(pi z)) exp(i(z - nu pi/2 - pi/4)) sum_k i^k a_k(nu) / z^k,
 * a_0 = 1, a_k = a_{k-1} (4 nu^2 - (2k-1)^2) / (8k). */
static void h01_asym(cplx z, cplx* h0, cplx* h1)
{
    cplx pre = csqrt(2.0 / (OR_PI * z));
    cplx e0 = cexp(I * (z - 0.25 * OR_PI));
    cplx e1 = cexp(I * (z - 0.75 * OR_PI));
    cplx s0 = 1.0, s1 = 1.0, t0 = 1.0, t1 = 1.0;
    double last0 = 1.0, last1 = 1.0;
    for (int k = 1; k < 200; ++k) {
        double m = (2.0 * k - 1.0) * (2.0 * k - 1.0);
        cplx f = I / (8.0 * k * z);
        cplx n0 = t0 * f * (0.0 - m);
        cplx n1 = t1 * f * (4.0 - m);
        double a0 = cabs(n0), a1 = cabs(n1);
        if (a0 > last0 && a1 > last1) break;   /* asymptotic: stop at the smallest term */
        t0 = n0; t1 = n1;
        s0 += t0; s1 += t1;
        last0 = a0; last1 = a1;
        if (a0 < 1e-18 * cabs(s0) && a1 < 1e-18 * cabs(s1)) break;
    }
    *h0 = pre * e0 * s0;
    *h1 = pre * e1 * s1;
}

#define OR_RASYM 25.0

/* Continue (w, w') = (H0, -H1) from z0 to z0 + h with the Taylor series of
 * Bessel's equation (order 0) about z0:  with w(z0+h) = sum a_k h^k,
 *   z0 (k+1)(k+2) a_{k+2} + (k+1)^2 a_{k+1} + z0 a_k + a_{k-1} = 0. */
static void bessel0_taylor_step(cplx z0, cplx h, cplx* w, cplx* dw)
{
    cplx am1 = 0.0, a0 = *w, a1 = *dw;
    cplx hp = h;                  /* h^k for the current a_k, k = 1 */
    cplx sw = a0 + a1 * h, sd = a1;
    double scale = cabs(a0) + cabs(a1) * cabs(h);
    for (int k = 0; k < 400; ++k) {
        cplx a2 = -(((double)(k + 1) * (k + 1)) * a1 + z0 * a0 + am1) /
                  (z0 * ((double)(k + 1) * (k + 2)));
        cplx dterm = (double)(k + 2) * a2 * hp;   /* derivative term uses h^(k+1) */
        hp *= h;                                  /* now h^(k+2) */
        cplx term = a2 * hp;
        sw += term;
        sd += dterm;
        am1 = a0; a0 = a1; a1 = a2;
        if (k > 4 && cabs(term) < 1e-19 * scale && cabs(dterm) * cabs(h) < 1e-19 * scale) break;
    }
    *w = sw;
    *dw = sd;
}

static cplx h0_ode(cplx z)
{
    double x = creal(z);
    double y1 = sqrt(OR_RASYM * OR_RASYM - x * x);
    cplx zc = x + I * y1;
    cplx h0, h1;
    h01_asym(zc, &h0, &h1);
    cplx w = h0, dw = -h1;        /* d/dz H0 = -H1 */
    double yt = cimag(z);
    while (cimag(zc) > yt) {
        double step = 0.3 * cabs(zc);
        double remain = cimag(zc) - yt;
        if (step > remain) step = remain;
        cplx h = -I * step;
        bessel0_taylor_step(zc, h, &w, &dw);
        zc = (cimag(zc) - step <= yt) ? z : zc + h;
        if (cimag(zc) <= yt) break;
    }
    return w;
}

cplx oracle_hankel0_c(cplx z)
{
    double a = cabs(z);
    if (a <= 2.5) return h0_series(z);
    if (a >= OR_RASYM) {
        cplx h0, h1;
        h01_asym(z, &h0, &h1);
        return h0;
    }
    return h0_ode(z);
}

/* ------------------------------------------------------------ kernels */

/* G for one complexified pair; s = sum_d (x_d - y_d)^2. */
static cplx green(int dim, int kernel, double kappa, cplx s)
{
    cplx r = csqrt(s);                   /* principal branch, Re r >= 0 */
    if (dim == 2) {
        if (kernel == OR_HELMHOLTZ) return 0.25 * I * oracle_hankel0_c(kappa * r);
        return -(1.0 / (2.0 * OR_PI)) * clog(r);
    }
    if (kernel == OR_HELMHOLTZ) return cexp(I * kappa * r) / (4.0 * OR_PI * r);
    return 1.0 / (4.0 * OR_PI * r);
}

typedef struct { double s, c; } neum_t;

static inline void neum_add(neum_t* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/*
 * u[i] = sum_j G(trg_i, src_j) sigma_j for i < n_trg.
 *   trg, src : complex128 [n][dim], interleaved (re, im) doubles
 *   sigma    : complex128 [n_src]
 *   self_idx : if non-NULL, self_idx[i] is the source index equal to target i
 *              (that pair is skipped); -1 for none
 *   out      : complex128 [n_trg]
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_direct(int dim, int kernel, double kappa,
                  int64_t n_trg, const double* trg,
                  int64_t n_src, const double* src,
                  const double* sigma, const int64_t* self_idx,
                  double* out, int nthreads)
{
    if ((dim != 2 && dim != 3) || (kernel != OR_LAPLACE && kernel != OR_HELMHOLTZ))
        return -1;
    if (kernel == OR_HELMHOLTZ && !(kappa > 0.0)) return -1;
    if (n_trg < 0 || n_src < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const cplx* T = (const cplx*)trg;
    const cplx* S = (const cplx*)src;
    const cplx* Q = (const cplx*)sigma;
    cplx* U = (cplx*)out;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n_trg; ++i) {
        neum_t re = {0.0, 0.0}, im = {0.0, 0.0};
        int64_t skip = self_idx ? self_idx[i] : -1;
        for (int64_t j = 0; j < n_src; ++j) {
            if (j == skip) continue;
            cplx s = 0.0;
            for (int d = 0; d < dim; ++d) {
                cplx dd = T[i * dim + d] - S[j * dim + d];
                s += dd * dd;
            }
            if (creal(s) == 0.0 && cimag(s) == 0.0) continue;
            cplx g = green(dim, kernel, kappa, s) * Q[j];
            neum_add(&re, creal(g));
            neum_add(&im, cimag(g));
        }
        U[i] = (re.s + re.c) + I * (im.s + im.c);
    }
    return 0;
}

/* Vector wrappers over this file's special functions, for the pins. */
void oracle_hankel0(int64_t n, const double* z, double* out)
{
    const cplx* Z = (const cplx*)z;
    cplx* O = (cplx*)out;
    for (int64_t i = 0; i < n; ++i) O[i] = oracle_hankel0_c(Z[i]);
}

void oracle_green(int dim, int kernel, double kappa, int64_t n, const double* s, double* out)
{
    const cplx* S = (const cplx*)s;
    cplx* O = (cplx*)out;
    for (int64_t i = 0; i < n; ++i) O[i] = green(dim, kernel, kappa, S[i]);
}

/*
 * Layer potentials with charges and dipoles, potential and gradient (Sec. 2.1:
 * the single and double layer potentials S[sigma], D[tau] and their normal
 * derivatives at the targets; a dipole vector v_j = tau_j nu_j carries the
 * double-layer density and the source normal):
 *
 *   u_i = sum_j G(x_i, y_j) sigma_j + v_j . grad_y G(x_i, y_j)
 *   g_i = grad_x u_i
 *
 * 3D kernels.  With d = x - y, r the principal root of d.d and G = g(r), the
 * chain rule (r^2 = d.d, bilinear, so grad_x r = d / r) gives
 *   grad_x G = g'(r) d / r,   grad_y G = -g'(r) d / r,
 *   grad_x (v . grad_y G) = -[ g'(r) v / r + (g''(r) - g'(r)/r) (v.d) d / r^2 ]
 * with g = 1/(4 pi r), g' = -g/r, g'' = 2 g / r^2 (Laplace) and
 * g = e^{i kappa r}/(4 pi r), g' = g (i kappa - 1/r),
 * g'' = g ((i kappa - 1/r)^2 + 1/r^2) (Helmholtz).
 *   charge : complex128[n_src] or NULL;  dipole : complex128[n_src][3] or NULL
 *   pot    : complex128[n_trg] or NULL;  grad   : complex128[n_trg][3] or NULL
 * Self pairs (self_idx) and pairs at s = 0 are skipped.  Neumaier sums.
 */
int oracle_layer3(int kernel, double kappa, int64_t n_trg, const double* trg, int64_t n_src,
                  const double* src, const double* charge, const double* dipole,
                  const int64_t* self_idx, double* pot, double* grad, int nthreads)
{
    if (kernel != OR_LAPLACE && kernel != OR_HELMHOLTZ) return -1;
    if (kernel == OR_HELMHOLTZ && !(kappa > 0.0)) return -1;
    if (n_trg < 0 || n_src < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const cplx* T = (const cplx*)trg;
    const cplx* S = (const cplx*)src;
    const cplx* Q = (const cplx*)charge;
    const cplx* V = (const cplx*)dipole;
    cplx* U = (cplx*)pot;
    cplx* G = (cplx*)grad;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n_trg; ++i) {
        neum_t acc[8];
        for (int k = 0; k < 8; ++k) acc[k].s = acc[k].c = 0.0;
        int64_t skip = self_idx ? self_idx[i] : -1;
        for (int64_t j = 0; j < n_src; ++j) {
            if (j == skip) continue;
            cplx d[3], s = 0.0;
            for (int k = 0; k < 3; ++k) {
                d[k] = T[i * 3 + k] - S[j * 3 + k];
                s += d[k] * d[k];
            }
            if (creal(s) == 0.0 && cimag(s) == 0.0) continue;
            cplx r = csqrt(s);
            cplx g, g1, g2;
            if (kernel == OR_HELMHOLTZ) {
                g = cexp(I * kappa * r) / (4.0 * OR_PI * r);
                cplx a = I * kappa - 1.0 / r;
                g1 = g * a;
                g2 = g * (a * a + 1.0 / (r * r));
            } else {
                g = 1.0 / (4.0 * OR_PI * r);
                g1 = -g / r;
                g2 = 2.0 * g / (r * r);
            }
            cplx u = 0.0, gr[3] = {0.0, 0.0, 0.0};
            if (Q) {
                u += g * Q[j];
                for (int k = 0; k < 3; ++k) gr[k] += g1 * d[k] / r * Q[j];
            }
            if (V) {
                const cplx* v = V + j * 3;
                cplx vd = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
                u += -g1 * vd / r;
                for (int k = 0; k < 3; ++k)
                    gr[k] += -(g1 * v[k] / r + (g2 - g1 / r) * vd * d[k] / (r * r));
            }
            neum_add(&acc[0], creal(u));
            neum_add(&acc[1], cimag(u));
            for (int k = 0; k < 3; ++k) {
                neum_add(&acc[2 + 2 * k], creal(gr[k]));
                neum_add(&acc[3 + 2 * k], cimag(gr[k]));
            }
        }
        if (U) U[i] = (acc[0].s + acc[0].c) + I * (acc[1].s + acc[1].c);
        if (G)
            for (int k = 0; k < 3; ++k)
                G[i * 3 + k] = (acc[2 + 2 * k].s + acc[2 + 2 * k].c) + I * (acc[3 + 2 * k].s + acc[3 + 2 * k].c);
    }
    return 0;
}
