// Cylindrical Bessel and Hankel functions of complex argument for the 2D
// Helmholtz kernel and its expansions (Sec. 3.2; the Graf addition theorem
// and the multipole / local expansions of Sec. 4.3).
//
// H0, H1 of z with Re z > 0:
//   |z| < 3, or |z| < 6 with Im z < 0:
//                  power series of J0, J1, Y0, Y1 (DLMF 10.2.2, 10.8.1); for
//                  Im z > 0 the sum J + iY cancels by e^{-2 Im z}, hence the
//                  smaller radius there
//   otherwise for |z| < 20: Hankel's Laplace-type integral
//                    H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} / Gamma(nu+1/2)
//                              * int_0^inf e^{-t} t^{nu-1/2} (1 + i t/(2z))^{nu-1/2} dt
//                  with t = x^2 and a 48-point Gauss-Hermite rule
//   |z| >= 20      Hankel's asymptotic expansion (DLMF 10.17.5)
// J_k sequences: a power series of the entire function J_k(z)/(z/2)^k plus
// backward recurrence for small |z|, Miller's algorithm normalised by
// exp(+-iz) = J0 + 2 sum (+-i)^k J_k otherwise.
#pragma once
#include "common.hpp"

namespace cfmm {

// ---------------------------------------------------------------- H0, H1
// series coefficients: 1/k^2, 1/(k(k+1)) and the harmonic numbers H_k
struct SeriesTab {
    double inv_k2[41], inv_kk1[41], harm[41];
};
constexpr SeriesTab make_series_tab()
{
    SeriesTab t{};
    double h = 0.0;
    for (int k = 1; k < 41; ++k) {
        t.inv_k2[k] = 1.0 / ((double)k * (double)k);
        t.inv_kk1[k] = 1.0 / ((double)k * (double)(k + 1));
        h += 1.0 / (double)k;
        t.harm[k] = h;
    }
    return t;
}

template <bool WANT_H1>
CFMM_HD void hankel_small(cplx z, cplx q, cplx half_log_q, cplx* h0, cplx* h1)
{
    // q = z^2/4, half_log_q = log(z/2)
    constexpr SeriesTab T = make_series_tab();
    cplx mq = -q;
    cplx t = mk(1.0, 0.0), j0 = t, s0 = mk(0.0, 0.0);
    cplx u = mk(1.0, 0.0), su = u, sh = mk(0.0, 0.0);   // J1 = (z/2) su
    double hk = 0.0;
    double aq = sqrt(cabs2(q));
    for (int k = 1; k < 40; ++k) {
        t = t * mq * T.inv_k2[k];
        double hk1 = T.harm[k];             // H_k
        j0 += t;
        s0 += hk1 * t;
        if (WANT_H1) {
            sh += (hk + hk1) * u;           // (H_{k-1} + H_k) u_{k-1}
            u = u * mq * T.inv_kk1[k];
            su += u;
        }
        hk = hk1;
        // terms shrink once k^2 > |q|; stop when they fall below the J0 sum's ulp
        if ((double)k * k > aq && cabs2(t) < 1e-36 * cabs2(j0)) break;
    }
    cplx lg = half_log_q + mk(kEuler, 0.0);
    cplx y0 = (2.0 / kPi) * (lg * j0 - s0);
    *h0 = j0 + times_i(y0);
    if (WANT_H1) {
        // the loop above stops at the J0 tolerance; finish the J1 series
        cplx zh = 0.5 * z;
        cplx j1 = zh * su;
        cplx y1 = (-2.0 / kPi) * cinv(z) + (2.0 / kPi) * (lg * j1) - (1.0 / kPi) * (zh * sh);
        *h1 = j1 + times_i(y1);
    }
}

template <bool WANT_H1>
CFMM_HD void hankel_quad(cplx z, const double* ghx, const double* ghw, cplx* h0, cplx* h1)
{
    cplx c = cdiv(mk(0.0, 0.5), z);            // i / (2z)
    cplx i0 = mk(0.0, 0.0), i1 = mk(0.0, 0.0);
    for (int k = 0; k < kGHHalf; ++k) {
        double x2 = ghx[k] * ghx[k];
        cplx a = mk(1.0 + x2 * c.re, x2 * c.im);
        cplx sq = csqrt_p(a);
        i0 += ghw[k] * cinv(sq);
        if (WANT_H1) i1 += (ghw[k] * x2) * sq;
    }
    cplx pre = csqrt_p(cdiv(mk(2.0 / kPi, 0.0), z)) * (1.0 / sqrt(kPi));
    cplx e0 = cexp_(times_i(z - mk(0.25 * kPi, 0.0)));
    *h0 = (2.0 * pre) * e0 * i0;                     // both halves of the symmetric rule
    if (WANT_H1) *h1 = (4.0 * pre) * (mk(0.0, -1.0) * e0) * i1;   // Gamma(3/2) = sqrt(pi)/2
}

template <bool WANT_H1>
CFMM_HD void hankel_asym(cplx z, cplx* h0, cplx* h1)
{
    cplx w = cdiv(mk(0.0, 0.125), z);          // i / (8z)
    cplx t0 = mk(1.0, 0.0), t1 = mk(1.0, 0.0), s0 = t0, s1 = t1;
    for (int k = 1; k < 60; ++k) {
        double m = (2.0 * k - 1.0) * (2.0 * k - 1.0);
        t0 = t0 * w * (-m / k);
        s0 += t0;
        if (WANT_H1) {
            t1 = t1 * w * ((4.0 - m) / k);
            s1 += t1;
        }
        if (cabs2(t0) < 1e-36 && (!WANT_H1 || cabs2(t1) < 1e-36)) break;
    }
    cplx pre = csqrt_p(cdiv(mk(2.0 / kPi, 0.0), z));
    cplx e0 = cexp_(times_i(z - mk(0.25 * kPi, 0.0)));
    *h0 = pre * e0 * s0;
    if (WANT_H1) *h1 = pre * (mk(0.0, -1.0) * e0) * s1;
}

// H0^(1)(z), H1^(1)(z), Re z > 0
CFMM_HD void hankel01(cplx z, const double* ghx, const double* ghw, cplx* h0, cplx* h1)
{
    double a2 = cabs2(z);
    if (a2 < 9.0 || (a2 < 36.0 && z.im < 0.0)) {
        cplx zh = 0.5 * z;
        hankel_small<true>(z, zh * zh, clog_p(zh), h0, h1);
    } else if (a2 < 400.0) {
        hankel_quad<true>(z, ghx, ghw, h0, h1);
    } else {
        hankel_asym<true>(z, h0, h1);
    }
}

// H0^(1)(kappa r) from s = r^2 (r the principal root), for the near field.
// The series branch needs only s: log(z/2) = log(kappa^2 s / 4) / 2.
CFMM_HD cplx hankel0_s(cplx s, double kappa, const double* ghx, const double* ghw)
{
    double k2 = kappa * kappa * 0.25;
    cplx q = k2 * s;
    double aq = cabs2(q);
    cplx h0, dummy;
    if (aq < 5.0625 || (aq < 81.0 && s.im < 0.0)) {   // |z| < 3, or |z| < 6 and Im z < 0
        cplx lq = clog_p(q);
        hankel_small<false>(mk(0.0, 0.0), q, 0.5 * lq, &h0, &dummy);
    } else {
        cplx z = kappa * csqrt_p(s);
        if (aq < 10000.0) hankel_quad<false>(z, ghx, ghw, &h0, &dummy);
        else hankel_asym<false>(z, &h0, &dummy);
    }
    return h0;
}

// ------------------------------------------------------------- sequences

// J_k(z), k = 0..K, by Miller's backward recurrence normalised with
// exp(+-iz) = J0 + 2 sum_k (+-i)^k J_k (the sign with |exp| >= 1, so the
// normalising sum does not cancel).
CFMM_HD void jn_miller(cplx z, int K, cplx* out, int st)
{
    cplx iz = cinv(z);
    double az = sqrt(cabs2(z));
    double mx = az > K ? az : (double)K;
    int N = (int)mx + 30 + (int)(10.0 * cbrt(mx));
    bool up = z.im > 0.0;                         // normalise by e^{-iz} (up) or e^{iz}
    cplx fnp1 = mk(0.0, 0.0), fn = mk(1e-250, 0.0);
    cplx norm = mk(0.0, 0.0);
    for (int k = N; k >= 0; --k) {
        if (k <= K) out[k * st] = fn;
        if (k == 0) {
            norm += fn;
        } else {
            int m = k & 3;
            cplx ph;  // (+-i)^k, minus sign when up
            if (m == 0) ph = mk(1.0, 0.0);
            else if (m == 2) ph = mk(-1.0, 0.0);
            else if ((m == 1) != up) ph = mk(0.0, 1.0);
            else ph = mk(0.0, -1.0);
            norm += 2.0 * (ph * fn);
            cplx fnm1 = (2.0 * k) * (iz * fn) - fnp1;
            fnp1 = fn;
            fn = fnm1;
            if (cabs2(fn) > 1e280) {          // |f| > 1e140: rescale everything kept so far
                const double sc = 1e-140;
                fn *= sc; fnp1 *= sc; norm *= sc;
                for (int j = k; j <= K; ++j) out[j * st] *= sc;
            }
        }
    }
    cplx target = up ? cexp_(mk(z.im, -z.re)) : cexp_(mk(-z.im, z.re));
    cplx scale = cdiv(target, norm);
    for (int k = 0; k <= K; ++k) out[k * st] = out[k * st] * scale;
}

// For Y = (y1, y2) in C^2 with rho^2 = y1^2 + y2^2 and e^{+-i phi} = (y1 +- i y2)/rho,
// jcore2 returns seq[k*st], k = 0..K, and bases bp, bm with
//     J_k(kappa rho) e^{+-ik phi} / r^k = seq[k] * (bp or bm)^k / (fact ? k! : 1).
// Small |z| (z = kappa rho): seq[k] = k! J_k(z)/(z/2)^k, an entire function of
// rho^2, by its power series at K and K+1 and the downward recurrence
//     s_{k-1} = s_k + qq s_{k+1} / (k (k+1)),  qq = -z^2/4   (stable downward);
// then bp,bm = kappa (y1 +- i y2) / (2r) and Y may sit on the centre.
// Large |z|: seq[k] = J_k(z) by Miller, bp,bm = e^{+-i phi} / r.
CFMM_HD void jcore2(cplx y1, cplx y2, double kappa, double r, int K, cplx* seq, int st,
                    cplx* bp, cplx* bm, bool* fact)
{
    cplx zp = mk(y1.re - y2.im, y1.im + y2.re);   // y1 + i y2
    cplx zm = mk(y1.re + y2.im, y1.im - y2.re);   // y1 - i y2
    cplx s = y1 * y1 + y2 * y2;
    cplx qq = (-0.25 * kappa * kappa) * s;
    double aq = sqrt(cabs2(qq));
    if (aq <= (double)(K + 1)) {
        cplx tk[2];
        for (int e = 0; e < 2; ++e) {
            int n = K + e;
            cplx term = mk(1.0, 0.0), sum = term;
            for (int j = 1; j < 200; ++j) {
                term = term * qq * (1.0 / ((double)j * (double)(n + j)));
                sum += term;
                if (cabs2(term) < 1e-36 * cabs2(sum)) break;
            }
            tk[e] = sum;
        }
        cplx t_hi = tk[1], t_cur = tk[0];
        seq[K * st] = t_cur;
        for (int k = K; k >= 1; --k) {
            cplx t_lo = t_cur + qq * t_hi * (1.0 / ((double)k * (double)(k + 1)));
            seq[(k - 1) * st] = t_lo;
            t_hi = t_cur;
            t_cur = t_lo;
        }
        *bp = (0.5 * kappa / r) * zp;
        *bm = (0.5 * kappa / r) * zm;
        *fact = true;
        return;
    }
    cplx rho = csqrt_p(s);
    jn_miller(kappa * rho, K, seq, st);
    *bp = cdiv(zp, rho) * (1.0 / r);
    *bm = cdiv(zm, rho) * (1.0 / r);
    *fact = false;
}

//   pos[k*st] = J_k(kappa rho) e^{+ik phi} / r^k,  neg[k*st] = J_k(kappa rho) e^{-ik phi} / r^k
CFMM_HD void jseq2(cplx y1, cplx y2, double kappa, double r, int K, cplx* pos, cplx* neg, int st)
{
    cplx bp, bm;
    bool fact;
    jcore2(y1, y2, kappa, r, K, pos, st, &bp, &bm, &fact);
    cplx pp = mk(1.0, 0.0), pm = mk(1.0, 0.0);
    for (int k = 0; k <= K; ++k) {
        cplx t = pos[k * st];
        pos[k * st] = pp * t;
        neg[k * st] = pm * t;
        double f = fact ? 1.0 / (k + 1) : 1.0;
        pp = pp * bp * f;
        pm = pm * bm * f;
    }
}

// hcore2: seq[k*st] = H_k(kappa rho) r^k, k = 0..K, and bp, bm = e^{+-i phi}, so
//     H_k(kappa rho) e^{+-ik phi} r^k = seq[k] * (bp or bm)^k.
// rho must not be small (the expansion centre is well separated from Y).
CFMM_HD void hcore2(cplx y1, cplx y2, double kappa, double r, int K, const double* ghx,
                    const double* ghw, cplx* seq, int st, cplx* bp, cplx* bm)
{
    cplx zp = mk(y1.re - y2.im, y1.im + y2.re);
    cplx zm = mk(y1.re + y2.im, y1.im - y2.re);
    cplx rho = csqrt_p(y1 * y1 + y2 * y2);
    cplx z = kappa * rho;
    cplx h0, h1;
    hankel01(z, ghx, ghw, &h0, &h1);
    *bp = cdiv(zp, rho);
    *bm = cdiv(zm, rho);
    cplx riz = r * cinv(z);
    double r2 = r * r;
    if (z.im >= -1.0) {
        // H^(1)_k grows with k for Im z >= 0: the upward recurrence is stable;
        // for -1 <= Im z < 0 the unwanted H^(2) component can gain at most
        // about e^(2 |Im z|) relative to H^(1), a few ulps
        cplx hm1 = h0, hk = r * h1;
        seq[0] = h0;
        for (int k = 1; k <= K; ++k) {
            seq[k * st] = hk;
            cplx hn = (2.0 * k) * (riz * hk) - r2 * hm1;
            hm1 = hk;
            hk = hn;
        }
        return;
    }
    // Im z < 0: H^(1)_k can decrease with k while H^(2)_k grows, so the upward
    // recurrence for H^(1) is unstable.  Use H^(1)_k = 2 J_k - H^(2)_k with J_k
    // from Miller and H^(2)_k(z) = conj(H^(1)_k(conj z)), whose upward
    // recurrence is stable (Im conj z > 0).  Neither term cancels the other:
    // H^(1) ~ 2J where H^(2) is small, and H^(1) ~ -H^(2) where J is small.
    jn_miller(z, K, seq, st);
    cplx g0, g1;
    hankel01(conj(z), ghx, ghw, &g0, &g1);
    cplx rizb = conj(riz);
    cplx gm1 = g0, gk = r * g1;
    double rk = 1.0;
    for (int k = 0; k <= K; ++k) {
        cplx gv = (k == 0) ? g0 : gk;
        seq[k * st] = (2.0 * rk) * seq[k * st] - conj(gv);
        if (k >= 1) {
            cplx gn = (2.0 * k) * (rizb * gk) - r2 * gm1;
            gm1 = gk;
            gk = gn;
        }
        rk *= r;
    }
}

//   pos[k*st] = H_k(kappa rho) e^{+ik phi} r^k,  neg[k*st] = H_k(kappa rho) e^{-ik phi} r^k
CFMM_HD void hseq2(cplx y1, cplx y2, double kappa, double r, int K, const double* ghx,
                   const double* ghw, cplx* pos, cplx* neg, int st)
{
    cplx bp, bm;
    hcore2(y1, y2, kappa, r, K, ghx, ghw, pos, st, &bp, &bm);
    cplx pp = mk(1.0, 0.0), pm = mk(1.0, 0.0);
    for (int k = 0; k <= K; ++k) {
        cplx t = pos[k * st];
        pos[k * st] = pp * t;
        neg[k * st] = pm * t;
        pp = pp * bp;
        pm = pm * bm;
    }
}

}  // namespace cfmm
