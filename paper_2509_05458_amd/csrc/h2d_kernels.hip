// 2D Helmholtz complex-coordinate FMM kernels (Sec. 4.3 and the multilevel
// steps of Sec. 6.4).  Expansions about a complexified centre c, n = -P..P:
//
//   multipole  u(x) = sum_n M_n H_n(kappa rho_X) e^{in phi_X},  M_n = sum_j sigma_j J_n(kappa rho_Y) e^{-in phi_Y}
//   local      u(x) = sum_n L_n J_n(kappa rho_X) e^{in phi_X},  L_n = sum_j sigma_j H_n(kappa rho_Y) e^{-in phi_Y}
//
// with X = x - c, Y = y - c and the complex polar coordinates of Sec. 3.1.
// Stored scaled: Mhat_n = M_n / r^|n|, Lhat_n = L_n r^|n| with r = min(1, kappa w)
// of the box's level (keeps the coefficients and the translation entries in
// range at low frequency).  Translations (Graf's addition theorem), with
// D = new centre - old centre:
//
//   M2M, L2L  out_m = sum_n J_{n-m}(kappa rho_D) e^{i(n-m) phi_D} in_n
//   M2L       out_m = sum_n H_{n-m}(kappa rho_D) e^{i(n-m) phi_D} in_n
//
// Every kernel owns its output (one workgroup per target box or leaf); there
// are no floating-point atomics, so evaluations are bitwise reproducible.
#include "bessel.hpp"
#include "kernels.hpp"
#include "quadrature.hpp"

namespace cfmm {

__constant__ double c_ghx[kGHHalf];
__constant__ double c_ghw[kGHHalf];
constexpr int kRcp = 512;
__constant__ double c_rcp[kRcp];     // 1/m, c_rcp[0] = 0

static double h_ghx[kGHHalf], h_ghw[kGHHalf];
static bool h_gh_ready = false;

static void host_gh()
{
    if (!h_gh_ready) {
        gauss_hermite_half(2 * kGHHalf, h_ghx, h_ghw);
        h_gh_ready = true;
    }
}

hipError_t h2d_init_tables(int device)
{
    (void)device;
    host_gh();
    static double rcp[kRcp];
    rcp[0] = 0.0;
    for (int m = 1; m < kRcp; ++m) rcp[m] = 1.0 / m;
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ghx), h_ghx, sizeof(h_ghx));
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rcp), rcp, sizeof(rcp))) != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_ghw), h_ghw, sizeof(h_ghw));
}

// generator entry k of a translation: pos for k >= 0, (-1)^|k| neg[|k|] otherwise
__device__ inline cplx gen_at(const cplx* gp, const cplx* gn, int k)
{
    if (k >= 0) return gp[k];
    cplx v = gn[-k];
    return (k & 1) ? -v : v;
}

__device__ inline int iabs_(int a) { return a < 0 ? -a : a; }

// ------------------------------------------------------------------ P2M
constexpr int kChunk = 16;

// Regular values at a point Y = y - c of a box with expansion length P and
// scale r (Sec. 4.2):
//   v_n = J_n(kappa rho_Y) e^{-in phi_Y} / r^|n|,  n = -P..P,
// with v_n = s_n bm^n / n! and v_{-n} = (-1)^n s_n bp^n / n! for n >= 0, where
// s_n = n! J_n(z)/(z/2)^n (z = kappa rho_Y), an entire function of
// rho_Y^2, comes from its power series at P and P+1 and the stable downward
// recurrence s_{n-1} = s_n + qq s_{n+1} / (n(n+1)), qq = -z^2/4, and
// bp, bm = kappa (y1 +- i y2) / (2r).  For |qq| > P + 1 the values come from
// Miller's recurrence for J_n (jcore2).  Reciprocals of integers come from a
// table.  P2M is M_n = sum_j sigma_j v_n(j), and L2P uses
// J_n(kappa rho_X) e^{in phi_X} / r^|n| = (-1)^n v_{-n} at the same point.
__device__ inline cplx series_s(cplx qq, int n)
{
    cplx term = mk(1.0, 0.0), sum = term;
    for (int j = 1; j < 200; ++j) {
        term = (term * qq) * (c_rcp[j] * c_rcp[n + j]);
        sum += term;
        if (cabs2(term) < 1e-36 * cabs2(sum)) break;
    }
    return sum;
}

// v[n * st], n = -P..P, for Y = (y1, y2); half = kappa / (2r)
__device__ inline void regular_values(cplx y1, cplx y2, double kappa, double half, double r, int P, cplx* v,
                                      int st)
{
    cplx zp = mk(y1.re - y2.im, y1.im + y2.re);   // y1 + i y2
    cplx zm = mk(y1.re + y2.im, y1.im - y2.re);   // y1 - i y2
    cplx qq = (-0.25 * kappa * kappa) * (y1 * y1 + y2 * y2);
    cplx bp, bm;
    bool fact;
    if (cabs2(qq) <= (double)(P + 1) * (double)(P + 1)) {
        cplx hi = series_s(qq, P + 1), cur = series_s(qq, P);
        v[P * st] = cur;
        for (int k = P; k >= 1; --k) {
            cplx lo = cur + (qq * hi) * (c_rcp[k] * c_rcp[k + 1]);
            v[(k - 1) * st] = lo;
            hi = cur;
            cur = lo;
        }
        bp = half * zp;
        bm = half * zm;
        fact = true;
    } else {
        jcore2(y1, y2, kappa, r, P, v, st, &bp, &bm, &fact);
    }
    // v[0..P] holds s_n; expand in place: v[n] = s_n bm^n/n!, v[-n] = (-1)^n s_n bp^n/n!
    cplx pp = mk(1.0, 0.0), pm = mk(1.0, 0.0);
    for (int k = 1; k <= P; ++k) {
        double f = fact ? c_rcp[k] : 1.0;
        pp = (pp * bp) * f;
        pm = (pm * bm) * f;
        cplx sk = v[k * st];
        v[k * st] = sk * pm;
        cplx w = sk * pp;
        v[-k * st] = (k & 1) ? -w : w;
    }
}

// The same values computed by two lanes, t and t ^ 32, of one wavefront:
// side = +1 writes v_n, n = 0..P, side = -1 writes v_{-n}, n = 0..P (v_0 by
// both, the same value).  Each lane sums one of the two starting series (at P
// and P+1) and takes the other from its partner; both run the downward
// recurrence, and each expands its own half.  Both lanes must be active and
// have the same point.
__device__ inline void regular_values_pair(cplx y1, cplx y2, double kappa, double half, double r, int P,
                                           cplx* v, int side)
{
    cplx zp = mk(y1.re - y2.im, y1.im + y2.re);   // y1 + i y2
    cplx zm = mk(y1.re + y2.im, y1.im - y2.re);   // y1 - i y2
    cplx qq = (-0.25 * kappa * kappa) * (y1 * y1 + y2 * y2);
    cplx bp, bm;
    bool fact;
    if (cabs2(qq) <= (double)(P + 1) * (double)(P + 1)) {
        cplx mine = series_s(qq, side > 0 ? P + 1 : P);
        cplx other = mk(__shfl_xor(mine.re, 32, 64), __shfl_xor(mine.im, 32, 64));
        cplx hi = side > 0 ? mine : other, cur = side > 0 ? other : mine;
        v[P * side] = cur;
        for (int k = P; k >= 1; --k) {
            cplx lo = cur + (qq * hi) * (c_rcp[k] * c_rcp[k + 1]);
            v[(k - 1) * side] = lo;
            hi = cur;
            cur = lo;
        }
        bp = half * zp;
        bm = half * zm;
        fact = true;
    } else {
        jcore2(y1, y2, kappa, r, P, v, side, &bp, &bm, &fact);
    }
    cplx pw = mk(1.0, 0.0), base = side > 0 ? bm : bp;
    for (int k = 1; k <= P; ++k) {
        double f = fact ? c_rcp[k] : 1.0;
        pw = (pw * base) * f;
        cplx w = v[k * side] * pw;
        v[k * side] = (side < 0 && (k & 1)) ? -w : w;
    }
}

// u = sum_n L_n (-1)^n v_{-n} = sum_k s_k (L_k bp^k + (-1)^k L_{-k} bm^k) / k!
// (k = 0 once), accumulated by Horner in bp and bm while the downward
// recurrence produces s_k.  L points at L_0.
__device__ inline cplx l2p_value(cplx y1, cplx y2, double kappa, double half, double r, int P,
                                 const cplx* __restrict__ L)
{
    cplx zp = mk(y1.re - y2.im, y1.im + y2.re);
    cplx zm = mk(y1.re + y2.im, y1.im - y2.re);
    cplx qq = (-0.25 * kappa * kappa) * (y1 * y1 + y2 * y2);
    if (cabs2(qq) <= (double)(P + 1) * (double)(P + 1)) {
        cplx bp = half * zp, bm = half * zm;
        cplx hi = series_s(qq, P + 1), cur = series_s(qq, P);
        // H+_k = a_k + bp/(k+1) H+_{k+1},  H-_k = c_k + bm/(k+1) H-_{k+1} (k >= 1)
        cplx Hp = L[P] * cur;
        cplx Hm = (P & 1) ? -(L[-P] * cur) : L[-P] * cur;
        if (P == 0) Hm = mk(0.0, 0.0);
        for (int k = P; k >= 1; --k) {
            cplx lo = cur + (qq * hi) * (c_rcp[k] * c_rcp[k + 1]);   // s_{k-1}
            double f = c_rcp[k];
            Hp = (bp * Hp) * f + L[k - 1] * lo;
            if (k >= 2) {
                cplx c = L[-(k - 1)] * lo;
                Hm = (bm * Hm) * f + (((k - 1) & 1) ? -c : c);
            }
            hi = cur;
            cur = lo;
        }
        return P >= 1 ? Hp + bm * Hm : Hp;
    }
    // large argument (rare): J_k by Miller's backward recurrence, summed by
    // Horner as it runs and normalised at the end as in jn_miller; bases
    // e^{+-i phi} / r
    cplx rho = csqrt_p(y1 * y1 + y2 * y2);
    cplx z = kappa * rho;
    cplx bp = cdiv(zp, rho) * (1.0 / r), bm = cdiv(zm, rho) * (1.0 / r);
    cplx iz = cinv(z);
    double az = sqrt(cabs2(z));
    double mx = az > P ? az : (double)P;
    int N = (int)mx + 30 + (int)(10.0 * cbrt(mx));
    bool up = z.im > 0.0;
    cplx fnp1 = mk(0.0, 0.0), fn = mk(1e-250, 0.0), norm = mk(0.0, 0.0);
    cplx Hp = mk(0.0, 0.0), Hm = mk(0.0, 0.0);
    for (int k = N; k >= 0; --k) {
        if (k <= P) {
            Hp = bp * Hp + L[k] * fn;
            if (k >= 1) {
                cplx c = L[-k] * fn;
                Hm = bm * Hm + ((k & 1) ? -c : c);
            }
        }
        if (k == 0) {
            norm += fn;
        } else {
            int m = k & 3;
            cplx ph;
            if (m == 0) ph = mk(1.0, 0.0);
            else if (m == 2) ph = mk(-1.0, 0.0);
            else if ((m == 1) != up) ph = mk(0.0, 1.0);
            else ph = mk(0.0, -1.0);
            norm += 2.0 * (ph * fn);
            cplx fnm1 = (2.0 * k) * (iz * fn) - fnp1;
            fnp1 = fn;
            fn = fnm1;
            if (cabs2(fn) > 1e280) {
                const double sc = 1e-140;
                fn *= sc; fnp1 *= sc; norm *= sc; Hp *= sc; Hm *= sc;
            }
        }
    }
    cplx target = up ? cexp_(mk(z.im, -z.re)) : cexp_(mk(-z.im, z.re));
    return cdiv(target, norm) * (Hp + bm * Hm);
}

// P2M: one workgroup of 64 per leaf; per chunk of up to 32 points, lanes q
// and q + 32 write point q's values to an LDS row (odd row length, so the
// rows of neighbouring points fall in different banks), the n >= 0 half and
// the n <= 0 half, then lane m sums sigma v_m over the chunk for its
// coefficients.
// points per staged chunk: the LDS of a chunk's values (2P+1 per point) bounds
// how many workgroups a compute unit holds
constexpr int kP2MChunk = 32;
static_assert(kP2MChunk == 32, "P2M pairs lanes q and q + 32 on point q of a chunk");

__global__ __launch_bounds__(64) void k_h2d_p2m(const int* __restrict__ leaves, int nleaf, TreeView tv,
                                                PointsView pv, double kappa, cplx* __restrict__ mpole)
{
    extern __shared__ cplx vv[];          // [kP2MChunk][2P+1] (point-major), then sigma[kP2MChunk]
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l], nc = 2 * P + 1;
    double r = tv.rs[l], half = 0.5 * kappa / r;
    int nbx = tv.nbox, t = threadIdx.x;
    int64_t n = pv.n;
    cplx* sg = vv + (size_t)nc * kP2MChunk;
    cplx c1 = mk(tv.cre[b], tv.cim[b]), c2 = mk(tv.cre[nbx + b], tv.cim[nbx + b]);
    cplx acc0 = mk(0.0, 0.0), acc1 = mk(0.0, 0.0);
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    for (int j0 = p0; j0 < p1; j0 += kP2MChunk) {
        int cnt = min(kP2MChunk, p1 - j0);
        __syncthreads();
        int q = t & 31;
        if (q < cnt) {
            int j = j0 + q;
            cplx y1 = mk(pv.xre[j] - c1.re, pv.xim[j] - c1.im);
            cplx y2 = mk(pv.xre[n + j] - c2.re, pv.xim[n + j] - c2.im);
            regular_values_pair(y1, y2, kappa, half, r, P, vv + (size_t)q * nc + P, t < 32 ? 1 : -1);
            if (t < 32) sg[q] = mk(pv.sre[j], pv.sim[j]);
        }
        __syncthreads();
        if (t < nc)
            for (int q = 0; q < cnt; ++q) cfma(acc0, vv[(size_t)q * nc + t], sg[q]);
        if (t + 64 < nc)
            for (int q = 0; q < cnt; ++q) cfma(acc1, vv[(size_t)q * nc + t + 64], sg[q]);
    }
    if (t < nc) mpole[tv.eoff[b] + t] = acc0;
    if (t + 64 < nc) mpole[tv.eoff[b] + t + 64] = acc1;
}

// ------------------------------------------------------ operator generators
// Translation generators depend only on the geometry and are built once per
// plan.  For a List-2 pair (target b, source a), D = c_b - c_a:
//   gm2l[k + 2P] = H_k(kappa rho_D) e^{ik phi_D} r^|k|,            k = -2P..2P
// with r = 1 (unscaled) on the levels below lwin, which the window M2L takes
// and for each box c with parent p (K = P_p + P_c):
//   gm2m[k + K] = J_k(kappa rho_D) e^{ik phi_D} / r_c^|k|,  D = c_p - c_c
//   gl2l[k + K] = J_k(kappa rho_D) e^{ik phi_D} / r_p^|k|,  D = c_c - c_p
// (negative k from J_{-k} = (-1)^k J_k, H_{-k} = (-1)^k H_k).
__device__ inline void fill_signed(cplx* g, int K, cplx bp, cplx bm, bool fact)
{
    // g[0..K] holds the core sequence; expand to g[-K..K] with the bases
    cplx pp = mk(1.0, 0.0), pm = mk(1.0, 0.0);
    for (int k = 1; k <= K; ++k) {
        double f = fact ? 1.0 / k : 1.0;
        pp = pp * bp * f;
        pm = pm * bm * f;
        cplx s = g[k];
        g[k] = s * pp;
        cplx v = s * pm;
        g[-k] = (k & 1) ? -v : v;
    }
}

__global__ void k_h2d_gen_m2l(int npairs, const int* __restrict__ pair_b, TreeView tv, double kappa, int lwin,
                              const int64_t* __restrict__ goff, cplx* __restrict__ gen)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npairs) return;
    int b = pair_b[e], a = tv.l2idx[e];
    int l = tv.level[b];
    int K = 2 * tv.P[l];
    double r = l < lwin ? 1.0 : tv.rs[l];
    int nbx = tv.nbox;
    cplx d1 = mk(tv.cre[b] - tv.cre[a], tv.cim[b] - tv.cim[a]);
    cplx d2 = mk(tv.cre[nbx + b] - tv.cre[nbx + a], tv.cim[nbx + b] - tv.cim[nbx + a]);
    cplx* g = gen + goff[e] + K;
    cplx bp, bm;
    hcore2(d1, d2, kappa, r, K, c_ghx, c_ghw, g, 1, &bp, &bm);
    fill_signed(g, K, bp, bm, false);
}

__global__ void k_h2d_gen_tr(const int* __restrict__ boxes, int nb, TreeView tv, double kappa,
                             const int64_t* __restrict__ toff, cplx* __restrict__ gm2m,
                             cplx* __restrict__ gl2l)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    int c = boxes[i], p = tv.parent[c];
    int lc = tv.level[c];
    int K = tv.P[lc] + tv.P[lc - 1];
    double rc = tv.rs[lc], rp = tv.rs[lc - 1];
    int nbx = tv.nbox;
    cplx d1 = mk(tv.cre[p] - tv.cre[c], tv.cim[p] - tv.cim[c]);
    cplx d2 = mk(tv.cre[nbx + p] - tv.cre[nbx + c], tv.cim[nbx + p] - tv.cim[nbx + c]);
    cplx bp, bm;
    bool fact;
    cplx* g = gm2m + toff[c] + K;
    jcore2(d1, d2, kappa, rc, K, g, 1, &bp, &bm, &fact);
    fill_signed(g, K, bp, bm, fact);
    g = gl2l + toff[c] + K;
    jcore2(-d1, -d2, kappa, rp, K, g, 1, &bp, &bm, &fact);
    fill_signed(g, K, bp, bm, fact);
}

// Launch shape shared by M2M, M2L and L2L (one launch per level): G lanes own
// the output coefficients (G >= 2P+1 when possible), S groups of G lanes split
// the input sum of a box (partial sums reduced through LDS), and 256/(G S)
// boxes share a 256-thread block.  All boxes of a launch have the same P.
// ------------------------------------------------------------------ translations
// M2M, M2L and L2L are Toeplitz matvecs with per-entry level-power factors.
// One workgroup of 64 per output box: for each source expansion the block
// stages the generator window, the source coefficients and the level's
// powers r^e in LDS; lane `lane` of slice s (G lanes x S slices, G >= 2P+1
// rounded to 16, 32 or 64) owns output coefficient lane (and lane + 64 when
// 2P+1 > 64) over the source terms n = -P + s, -P + s + S, ...; the S slice
// sums are added through LDS in a fixed order.
constexpr int kGenMax = 4 * kPMax2D + 1;
static_assert(kGenMax <= 4 * 64 && kNCoef2DMax <= 2 * 64, "M2M/M2L operand prefetch holds 4 + 2 values per lane");

// Operands of one translation held in registers between their load and their
// store to LDS: generator values i = t + nt k (k < 4, i < ng) and source
// coefficients i = t + nt k (k < 2, i < nm).
// (plain double2 registers: a struct of cplx members was kept in scratch)
using TrRegs = double2[6];
__device__ inline double2 ld2(const cplx* p)
{
    return *reinterpret_cast<const double2*>(p);
}
__device__ inline void tr_load(double2 (&r)[6], const cplx* __restrict__ G, int ng,
                               const cplx* __restrict__ M, int nm, int t, int nt)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
        r[k] = (t + k * nt < ng) ? ld2(G + t + k * nt) : double2{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k)
        r[4 + k] = (t + k * nt < nm) ? ld2(M + t + k * nt) : double2{0.0, 0.0};
}
__device__ inline void tr_store(const double2 (&r)[6], cplx* g, int ng, cplx* m, int nm, int t, int nt)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (t + k * nt < ng) g[t + k * nt] = mk(r[k].x, r[k].y);
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (t + k * nt < nm) m[t + k * nt] = mk(r[4 + k].x, r[4 + k].y);
}

// NT = threads of the block (one slice partial each); M2L runs 64-thread
// blocks and keeps its LDS small so that more of them fit on a CU
template <int NT>
struct TrShared {
    cplx g[kGenMax];            // generator window
    cplx m[kNCoef2DMax];        // source coefficients
    double pw[kPwStride];       // r^e of the level that carries the factors
    cplx part[NT];
};

// G lanes per output group (outputs beyond 64 take a second round) and S =
// blockDim / G slices of the source terms
__device__ inline void tr_shape(int ncoef, int& G, int& S)
{
    G = ncoef <= 16 ? 16 : (ncoef <= 32 ? 32 : 64);
    S = (int)blockDim.x / G;
}

template <int NT>
__device__ inline cplx slice_sum(cplx acc, TrShared<NT>& sh, int G, int S, int s)
{
    if (S == 1) return acc;
    __syncthreads();
    sh.part[threadIdx.x] = acc;
    __syncthreads();
    cplx r = acc;
    if (s == 0)
        for (int k = 1; k < S; ++k) r += sh.part[threadIdx.x + k * G];
    return r;
}

// Entry (m, n) of child c: gm2m[n - m] r_c^(|n-m| + |n| - |m|) (r_c/r_p)^|m|.
__global__ __launch_bounds__(256) void k_h2d_m2m(const int* __restrict__ boxes, int nb, TreeView tv, H2DOps ops,
                                                cplx* __restrict__ mpole)
{
    __shared__ TrShared<256> sh;
    int p = boxes[xcd_contiguous(blockIdx.x, nb)];
    int l = tv.level[p];
    int Pp = tv.P[l], Pc = tv.P[l + 1];
    int K = Pp + Pc, ncoef = 2 * Pp + 1, nsrc = 2 * Pc + 1;
    int G, S;
    tr_shape(ncoef, G, S);
    int t = threadIdx.x, lane = t % G, s = t / G;
    for (int e = t; e < kPwStride; e += blockDim.x) sh.pw[e] = ops.pw[(size_t)(l + 1) * kPwStride + e];
    cplx acc0 = mk(0.0, 0.0), acc1 = mk(0.0, 0.0);
    int c0 = tv.child0[p], nc = tv.nchild[p];
    // the next child's generator and coefficients are loaded into registers
    // while the current one is summed (2K+1 <= 4 x 64, 2P_c+1 <= 2 x 64)
    int ng = 2 * K + 1, nt = (int)blockDim.x;
    TrRegs rr;
    if (nc > 0) tr_load(rr, ops.g_m2m + ops.o_tr[c0], ng, mpole + tv.eoff[c0], nsrc, t, nt);
    for (int ci = 0; ci < nc; ++ci) {
        __syncthreads();
        tr_store(rr, sh.g, ng, sh.m, nsrc, t, nt);
        __syncthreads();
        if (ci + 1 < nc)
            tr_load(rr, ops.g_m2m + ops.o_tr[c0 + ci + 1], ng, mpole + tv.eoff[c0 + ci + 1], nsrc, t, nt);
        for (int r = 0; r < 2; ++r) {
            int mi = lane + 64 * r;
            if (mi >= ncoef) break;
            int mm = mi - Pp, am = mm < 0 ? -mm : mm;
            cplx acc = mk(0.0, 0.0);
            for (int nn = -Pc + s; nn <= Pc; nn += S) {
                int k = nn - mm;
                int e = (k < 0 ? -k : k) + (nn < 0 ? -nn : nn) - am;
                cfma(acc, sh.pw[e] * sh.g[k + K], sh.m[nn + Pc]);
            }
            if (r == 0) acc0 += acc;
            else acc1 += acc;
        }
    }
    double rat = tv.rs[l + 1] / tv.rs[l];
    for (int r = 0; r < 2; ++r) {
        cplx acc = slice_sum(r == 0 ? acc0 : acc1, sh, G, S, s);
        int mi = lane + 64 * r;
        int mm = mi - Pp, am = mm < 0 ? -mm : mm;
        if (mi < ncoef && s == 0) mpole[tv.eoff[p] + mi] = pow(rat, (double)am) * acc;
    }
}

// Entry (m, n) of source a: gm2l[n - m] r^(|m| + |n| - |n - m|), i.e.
// r^(2 min(|m|,|n|)) when m, n have the same sign and 1 otherwise.  All
// levels go in one launch (M2L has no dependence between levels).
__global__ __launch_bounds__(64) void k_h2d_m2l(const int* __restrict__ boxes, int nboxes, TreeView tv,
                                                H2DOps ops, const cplx* __restrict__ mpole,
                                                cplx* __restrict__ local)
{
    __shared__ TrShared<64> sh;
    int b = boxes[xcd_contiguous(blockIdx.x, nboxes)];
    int l = tv.level[b];
    int P = tv.P[l], ncoef = 2 * P + 1;
    int G, S;
    tr_shape(ncoef, G, S);
    int t = threadIdx.x, lane = t % G, s = t / G;
    for (int e = t; e <= 2 * P; e += 64) sh.pw[e] = ops.pw[(size_t)l * kPwStride + e];
    cplx acc0 = mk(0.0, 0.0), acc1 = mk(0.0, 0.0);
    // the next entry's generator and coefficients are loaded into registers
    // while the current one is summed (4P+1 <= 4 x 64, 2P+1 <= 2 x 64)
    int ng = 4 * P + 1, e0 = tv.l2off[b], e1 = tv.l2off[b + 1];
    TrRegs rr;
    if (e0 < e1) tr_load(rr, ops.g_m2l + ops.o_m2l[e0], ng, mpole + tv.eoff[tv.l2idx[e0]], ncoef, t, 64);
    for (int e = e0; e < e1; ++e) {
        __syncthreads();
        tr_store(rr, sh.g, ng, sh.m, ncoef, t, 64);
        __syncthreads();
        if (e + 1 < e1)
            tr_load(rr, ops.g_m2l + ops.o_m2l[e + 1], ng, mpole + tv.eoff[tv.l2idx[e + 1]], ncoef, t, 64);
        for (int r = 0; r < 2; ++r) {
            int mi = lane + 64 * r;
            if (mi >= ncoef) break;
            int mm = mi - P, am = mm < 0 ? -mm : mm;
            cplx acc = mk(0.0, 0.0);
            for (int nn = -P + s; nn <= P; nn += S) {
                int an = nn < 0 ? -nn : nn;
                bool same = (nn > 0 && mm > 0) || (nn < 0 && mm < 0);
                int ex = same ? 2 * (an < am ? an : am) : 0;
                cfma(acc, sh.pw[ex] * sh.g[nn - mm + 2 * P], sh.m[nn + P]);
            }
            if (r == 0) acc0 += acc;
            else acc1 += acc;
        }
    }
    for (int r = 0; r < 2; ++r) {
        cplx acc = slice_sum(r == 0 ? acc0 : acc1, sh, G, S, s);
        int mi = lane + 64 * r;
        if (mi < ncoef && s == 0) local[tv.eoff[b] + mi] = acc;
    }
}

// M2L by sliding windows, for levels whose operator stays in FP64 range
// unscaled.  Unscaled, the operator is Toeplitz:
//   L_m = sum_n G[n - m] M_n,  G[k] = H_k e^{ik phi} (the plan stores it so),
//   M_n = r^|n| Mhat_n,  and Lhat_m = r^|m| L_m.  A lane owns kWin consecutive outputs m0 .. m0 + 3
// of one List-2 entry and streams n: output m0 + c needs G[n - m0 - c], so
// each step loads one new G for kWin complex multiply-adds, the others
// sliding through registers.  ceil((2P+1)/4) lanes serve an entry, so one
// wavefront takes E = 64 / that many entries of the target box per round (7
// at P = 17) instead of idling the lanes beyond 2P+1; the E partial sums meet
// in LDS at the end, added in entry-slot order.  A box with more entries
// than one round holds runs in a workgroup of W wavefronts that take the
// rounds in turn, each with its own LDS (the slots of all W meet at the end,
// in wavefront-major order).  G is stored with one gap entry after every
// eight (index i at i + i/8) to spread the lanes' reads over the banks.
constexpr int kWin = 4;
// generator and coefficient values staged per lane and round: E (4P + 4) and
// E (2P + 1) are at most 64 kStageG and 64 kStageA for every P <= 63
constexpr int kStageG = 8, kStageA = 4;

__device__ inline int gskew(int i) { return i + (i >> 3); }

constexpr int kM2LWWaves = 8;    // wavefronts of a workgroup for one box with many entries

__global__ __launch_bounds__(64 * kM2LWWaves) void k_h2d_m2l_w(const int* __restrict__ boxes,
                                                              const int2* __restrict__ grp, int ngrp, TreeView tv,
                                                              H2DOps ops, const cplx* __restrict__ mpole,
                                                              cplx* __restrict__ local)
{
    extern __shared__ cplx wlds_all[];
    int2 gr = grp[xcd_contiguous(blockIdx.x, ngrp)];
    const int* gbox = boxes + gr.x;               // gr.y consecutive boxes of one level
    int nbx = gr.y;
    int b = gbox[0];
    int l = tv.level[b];
    int P = tv.P[l], nc = 2 * P + 1;
    int NG = (nc + kWin - 1) / kWin, E = 64 / NG;
    int glen = 4 * P + 1 + (kWin - 1);            // G[k], k = -2P-7 .. 2P (zero guards below -2P)
    int GS = gskew(glen - 1) + 1;
    int W = blockDim.x >> 6, wv = threadIdx.x >> 6;
    cplx* wlds = wlds_all + (size_t)wv * E * (GS + nc);
    cplx* gb = wlds;                              // [E][GS]
    cplx* ab = wlds + (size_t)E * GS;             // [E][nc]
    const double* pw = ops.pw + (size_t)l * kPwStride;
    int t = threadIdx.x & 63, slot = t / NG, j = t - slot * NG;
    bool act = slot < E;
    int m0 = -P + kWin * j;
    cplx acc[kWin];
#pragma unroll
    for (int c = 0; c < kWin; ++c) acc[c] = mk(0.0, 0.0);
    int e0 = __builtin_amdgcn_readfirstlane(tv.l2off[b]);
    int e1 = __builtin_amdgcn_readfirstlane(tv.l2off[gbox[nbx - 1] + 1]);
    // wavefront wv takes rounds wv, wv + W, ...; within a wavefront the
    // LDS writes and reads are ordered by wave barriers
    for (int eb = e0 + wv * E; eb < e1; eb += W * E) {
        int ne = min(E, e1 - eb);
        __builtin_amdgcn_wave_barrier();
        // all of the round's loads are issued before any is stored: lane sl
        // < ne fetches entry sl's offsets, shared by shuffles; element u of a
        // lane is (slot, q) = t + 64 u in slot-major order (the generator
        // stored unscaled on these levels)
        int64_t og = t < ne ? ops.o_m2l[eb + t] : 0;
        int om = t < ne ? ops.m2l_src[eb + t] : 0;
        cplx pg[kStageG], pa[kStageA];
        {
            int sl = 0, q = t;
            while (q >= glen) { q -= glen; ++sl; }
#pragma unroll
            for (int u = 0; u < kStageG; ++u) {
                int64_t o = __shfl(og, sl < 63 ? sl : 63, 64);
                int k = q - 2 * P - (kWin - 1);
                pg[u] = (sl < ne && k >= -2 * P) ? ops.g_m2l[o + k + 2 * P] : mk(0.0, 0.0);
                q += 64;
                while (q >= glen) { q -= glen; ++sl; }
            }
            sl = 0; q = t;
            while (q >= nc) { q -= nc; ++sl; }
#pragma unroll
            for (int u = 0; u < kStageA; ++u) {
                int o = __shfl(om, sl < 63 ? sl : 63, 64);
                pa[u] = sl < ne ? mpole[o + q] : mk(0.0, 0.0);
                q += 64;
                while (q >= nc) { q -= nc; ++sl; }
            }
        }
        {
            int sl = 0, q = t;
            while (q >= glen) { q -= glen; ++sl; }
#pragma unroll
            for (int u = 0; u < kStageG; ++u) {
                if (sl < ne) gb[(size_t)sl * GS + gskew(q)] = pg[u];
                q += 64;
                while (q >= glen) { q -= glen; ++sl; }
            }
            sl = 0; q = t;
            while (q >= nc) { q -= nc; ++sl; }
#pragma unroll
            for (int u = 0; u < kStageA; ++u) {
                int an = q - P < 0 ? P - q : q - P;
                if (sl < ne) ab[(size_t)sl * nc + q] = pw[an] * pa[u];
                q += 64;
                while (q >= nc) { q -= nc; ++sl; }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (act && slot < ne) {
            const cplx* G = gb + (size_t)slot * GS;
            const cplx* A = ab + (size_t)slot * nc;
            int q0 = P - m0 + (kWin - 1);          // G[n - m0] at n = -P
            cplx w[kWin];
#pragma unroll
            for (int c = 1; c < kWin; ++c) w[c] = G[gskew(q0 - c)];
#pragma unroll 4
            for (int n = 0; n < nc; ++n) {
                w[0] = G[gskew(q0 + n)];
                cplx av = A[n];
#pragma unroll
                for (int c = 0; c < kWin; ++c) cfma(acc[c], w[c], av);
#pragma unroll
                for (int c = kWin - 1; c > 0; --c) w[c] = w[c - 1];
            }
        }
    }
    __syncthreads();
    cplx* red = wlds_all;                         // [W E][NG][kWin]
    int gs = wv * E + slot;                       // slot over the workgroup
    if (act)
#pragma unroll
        for (int c = 0; c < kWin; ++c) red[((size_t)gs * NG + j) * kWin + c] = acc[c];
    __syncthreads();
    // thread u = (box, j, c) adds output m0(j) + c of a box over its slots:
    // all slots for a box alone in its group (it may take several rounds),
    // else the slots of its own entries (one round)
    for (int u = threadIdx.x; u < nbx * NG * kWin; u += blockDim.x) {
        int bi = u / (NG * kWin), r = u - bi * NG * kWin;
        int jj = r / kWin, c = r - jj * kWin, m = -P + kWin * jj + c;
        if (m > P) continue;
        int bb = gbox[bi];
        int s0 = nbx == 1 ? 0 : tv.l2off[bb] - e0, s1 = nbx == 1 ? W * E : tv.l2off[bb + 1] - e0;
        cplx v = mk(0.0, 0.0);
        for (int sl = s0; sl < s1; ++sl) v += red[((size_t)sl * NG + jj) * kWin + c];
        local[tv.eoff[bb] + m + P] = pw[m < 0 ? -m : m] * v;
    }
}

// LDS of k_h2d_m2l_w at expansion length P
static size_t m2l_w_lds(int P, int W)
{
    int nc = 2 * P + 1, NG = (nc + kWin - 1) / kWin, E = 64 / NG;
    int glen = 4 * P + 1 + (kWin - 1);
    size_t stage = (size_t)W * E * ((size_t)(glen - 1 + ((glen - 1) >> 3) + 1) + nc);
    size_t red = (size_t)W * E * NG * kWin;
    return sizeof(cplx) * (stage > red ? stage : red);
}

// ------------------------------------------------------------------ P2L
// Sources of the coarser leaves in List 4 go directly into the local
// expansion (added after M2L wrote it).  Launched per level.  Threads q and
// q + 64 of the block compute the two Hankel sequences of source q of the
// current chunk (at most 64) into LDS, H_k e^{+ik phi} r^k and
// H_k e^{-ik phi} r^k; then thread t accumulates output coefficient t % G
// over the sources q = t / G (mod S) of the chunk, and the S partial sums
// are reduced through LDS at the end.
__device__ inline void hseq2_side(cplx y1, cplx y2, double kappa, double r, int K, cplx* seq, bool pos)
{
    cplx bp, bm;
    hcore2(y1, y2, kappa, r, K, c_ghx, c_ghw, seq, 1, &bp, &bm);
    cplx b = pos ? bp : bm, pw = mk(1.0, 0.0);
    for (int k = 1; k <= K; ++k) {
        pw = pw * b;
        seq[k] = pw * seq[k];
    }
}

__global__ __launch_bounds__(128) void k_h2d_p2l(const int* __restrict__ boxes, TreeView tv,
                                                 PointsView pv, double kappa, int chunk, int pstride,
                                                 cplx* __restrict__ local)
{
    extern __shared__ cplx lds[];
    cplx* gp = lds;                              // [chunk][pstride]
    cplx* gn = gp + (size_t)chunk * pstride;     // [chunk][pstride]
    cplx* ss = gn + (size_t)chunk * pstride;     // [chunk]
    cplx* part = ss + chunk;                     // [128]
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    double r = tv.rs[l];
    int nbx = tv.nbox, ncoef = 2 * P + 1;
    int G = ncoef <= 32 ? 32 : (ncoef <= 64 ? 64 : 128), S = 128 / G;
    int64_t n = pv.n;
    int t = threadIdx.x, mi = t % G, sp = t / G, mm = mi - P;
    cplx acc = mk(0.0, 0.0);
    cplx cb1 = mk(tv.cre[b], tv.cim[b]), cb2 = mk(tv.cre[nbx + b], tv.cim[nbx + b]);
    for (int e = tv.l4off[b]; e < tv.l4off[b + 1]; ++e) {
        int c = tv.l4idx[e];
        int q0 = tv.pbeg[c], q1 = tv.pend[c];
        for (int j0 = q0; j0 < q1; j0 += chunk) {
            int cnt = min(chunk, q1 - j0);
            int qs = t & 63;
            if (qs < cnt) {
                int j = j0 + qs;
                cplx y1 = mk(pv.xre[j] - cb1.re, pv.xim[j] - cb1.im);
                cplx y2 = mk(pv.xre[n + j] - cb2.re, pv.xim[n + j] - cb2.im);
                hseq2_side(y1, y2, kappa, r, P, (t < 64 ? gp : gn) + (size_t)qs * pstride, t < 64);
                if (t < 64) ss[qs] = mk(pv.sre[j], pv.sim[j]);
            }
            __syncthreads();
            if (mi < ncoef) {
                for (int q = sp; q < cnt; q += S) {
                    const cplx* pq = gp + (size_t)q * pstride;
                    const cplx* nq = gn + (size_t)q * pstride;
                    cplx v = (mm >= 0) ? nq[mm] : ((mm & 1) ? -pq[-mm] : pq[-mm]);
                    acc += v * ss[q];
                }
            }
            __syncthreads();
        }
    }
    part[t] = acc;
    __syncthreads();
    if (sp == 0 && mi < ncoef) {
        for (int k = 1; k < S; ++k) acc += part[t + k * G];
        local[tv.eoff[b] + mi] += acc;
    }
}

// ------------------------------------------------------------------ L2L
// Entry (m, n): gl2l[n - m] r_p^(|n-m| + |m| - |n|) (r_c/r_p)^|m|; one
// workgroup per child.
__global__ __launch_bounds__(256) void k_h2d_l2l(const int* __restrict__ boxes, int nb, TreeView tv, H2DOps ops,
                                                cplx* __restrict__ local)
{
    __shared__ TrShared<256> sh;
    int c = boxes[xcd_contiguous(blockIdx.x, nb)];
    int p = tv.parent[c];
    int lc = tv.level[c];
    int Pc = tv.P[lc], Pp = tv.P[lc - 1];
    int K = Pp + Pc, ncoef = 2 * Pc + 1, nsrc = 2 * Pp + 1;
    int G, S;
    tr_shape(ncoef, G, S);
    int t = threadIdx.x, lane = t % G, s = t / G;
    for (int e = t; e < kPwStride; e += blockDim.x) sh.pw[e] = ops.pw[(size_t)(lc - 1) * kPwStride + e];
    const cplx* Gv = ops.g_l2l + ops.o_tr[c];
    const cplx* Lp = local + tv.eoff[p];
    for (int i = t; i <= 2 * K; i += blockDim.x) sh.g[i] = Gv[i];
    for (int i = t; i < nsrc; i += blockDim.x) sh.m[i] = Lp[i];
    __syncthreads();
    double rat = tv.rs[lc] / tv.rs[lc - 1];
    for (int r = 0; r < 2; ++r) {
        int mi = lane + 64 * r;
        int mm = mi - Pc, am = mm < 0 ? -mm : mm;
        cplx acc = mk(0.0, 0.0);
        if (mi < ncoef)
            for (int nn = -Pp + s; nn <= Pp; nn += S) {
                int k = nn - mm;
                int e = (k < 0 ? -k : k) + am - (nn < 0 ? -nn : nn);
                cfma(acc, sh.pw[e] * sh.g[k + K], sh.m[nn + Pp]);
            }
        acc = slice_sum(acc, sh, G, S, s);
        if (mi < ncoef && s == 0) local[tv.eoff[c] + mi] += pow(rat, (double)am) * acc;
        if (ncoef <= 64) break;
    }
}

// ------------------------------------------------------------- L2P, M2P
// L2P writes the far field of every target of a leaf with expansions (0 for
// leaves coarser than the top level).  The leaf's per-point values are
// contiguous (point-major), so a chunk of points is staged into LDS with
// coalesced loads and each thread then reads its own point's row there.
// ------------------------------------------------------------------ L2P
// One thread per target of a leaf: the leaf's local expansion by l2p_value,
// plus the leaf's List-3 parts in list order.
__global__ __launch_bounds__(64) void k_h2d_l2p(const int* __restrict__ leaves, int top, TreeView tv,
                                                PointsView pv, double kappa, const cplx* __restrict__ local,
                                                const int64_t* __restrict__ poff3, const cplx* __restrict__ part,
                                                cplx* __restrict__ ufar)
{
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    int t = threadIdx.x;
    if (l < top) {
        for (int i = p0 + t; i < p1; i += blockDim.x) ufar[i] = mk(0.0, 0.0);
        return;
    }
    int P = tv.P[l];
    double r = tv.rs[l], half = 0.5 * kappa / r;
    int nbx = tv.nbox;
    int64_t n = pv.n;
    cplx c1 = mk(tv.cre[b], tv.cim[b]), c2 = mk(tv.cre[nbx + b], tv.cim[nbx + b]);
    const cplx* L = local + tv.eoff[b] + P;
    for (int i = p0 + t; i < p1; i += blockDim.x) {
        cplx y1 = mk(pv.xre[i] - c1.re, pv.xim[i] - c1.im);
        cplx y2 = mk(pv.xre[n + i] - c2.re, pv.xim[n + i] - c2.im);
        cplx u = l2p_value(y1, y2, kappa, half, r, P, L);
        for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) u += part[poff3[e] + i - p0];
        ufar[i] = u;
    }
}

// M2P by List-3 entries: entry e = (leaf owner[e], box l3idx[e]) evaluates the
// box's multipole at the leaf's points into part[poff[e] + i - pbeg], one
// block per entry.  Each thread's Hankel sequence sits in its LDS column.
__global__ void k_h2d_m2p_part(const int* __restrict__ owner, const int64_t* __restrict__ poff, TreeView tv,
                               PointsView pv, double kappa, const cplx* __restrict__ mpole,
                               cplx* __restrict__ part)
{
    extern __shared__ cplx rows[];      // rows[k * blockDim.x + thread]
    int e = blockIdx.x;
    int b = owner[e], a = tv.l3idx[e];
    int nbx = tv.nbox, st = blockDim.x, t = threadIdx.x;
    int64_t n = pv.n;
    int la = tv.level[a];
    int Pa = tv.P[la];
    double ra = tv.rs[la];
    cplx ca1 = mk(tv.cre[a], tv.cim[a]), ca2 = mk(tv.cre[nbx + a], tv.cim[nbx + a]);
    const cplx* M = mpole + tv.eoff[a] + Pa;
    cplx* o = part + poff[e] - tv.pbeg[b];
    for (int i = tv.pbeg[b] + t; i < tv.pend[b]; i += st) {
        cplx Y1 = mk(pv.xre[i], pv.xim[i]) - ca1, Y2 = mk(pv.xre[n + i], pv.xim[n + i]) - ca2;
        cplx bp, bm;
        hcore2(Y1, Y2, kappa, ra, Pa, c_ghx, c_ghw, rows + t, st, &bp, &bm);
        cplx pp = mk(1.0, 0.0), pm = mk(1.0, 0.0), u = mk(0.0, 0.0);
        for (int k = 0; k <= Pa; ++k) {
            cplx term = pp * M[k];
            if (k > 0) {
                cplx v = pm * M[-k];
                term += (k & 1) ? -v : v;
            }
            u += rows[k * st + t] * term;
            pp = pp * bp;
            pm = pm * bm;
        }
        o[i] = u;
    }
}


// 1/b for positive normal b: the hardware estimate y0 refined by one
// third-order step of the series 1/(1 - e) = 1 + e + e^2 + O(e^3),
// e = 1 - b y0 (truncation below 2^-70 for |e| < 2^-23).
__device__ inline double rcp_nr(double b)
{
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

// Polynomial coefficients, read through scalar loads so that each Horner step
// is one FMA with a scalar addend: atan(t) = t + t^3 sum_k c_atanp[6-k] t^(2k)
// and atanh(t)/t = sum_k c_logp[7-k] t^(2k) (both below).
__constant__ double c_atanp[7] = {-0.05797887584396482, 0.07637157054800217, -0.09089056697674516,
                                  0.11111076353854933, -0.14285713928935914, 0.19999999998180903,
                                  -0.3333333333332968};
__constant__ double c_logp[8] = {0.07404856752435146, 0.07656263923854066, 0.09091815845727959,
                                 0.11111098528259822, 0.14285714380321807, 0.19999999999651163,
                                 0.33333333333333826, 1.0};

// Argument of (x, y) != (0, 0) in (-pi, pi], as atan2(y, x).  With
// num = min(|x|, |y|) and den = max(|x|, |y|), atan(num/den) lies in
// [0, pi/4]; the addition formula atan(t) = atan(c) + atan((t - c)/(1 + t c)),
// with c = 0 for t below tan(pi/16), c = tan(pi/8) up to tan(3 pi/16) and
// c = 1 above, leaves |t'| <= tan(pi/16) < 0.2.  There atan(t') = t' P(t'^2)
// with P of degree 7, the odd Chebyshev interpolant of atan on [-0.2, 0.2]
// (nodes of degree 15, computed in extended precision and rounded): relative
// error below 3e-17.  atan(c) is taken for the rounded c the code uses, so
// the identity is exact, and c = 0 keeps small angles to relative accuracy.
__device__ inline double arg2(double x, double y)
{
    double ax = fabs(x), ay = fabs(y);
    bool sw = ay > ax;
    double num = sw ? ax : ay, den = sw ? ay : ax;
    bool mid = num > 0.198912367379658 * den;             // t > tan(pi/16)
    bool hi = num > 0.6681786379192989 * den;             // t > tan(3 pi/16)
    double c = hi ? 1.0 : (mid ? 0.41421356237309503 : 0.0);
    double ac = hi ? 0.7853981633974483 : (mid ? 0.39269908169872414 : 0.0);
    double tp = fma(-c, den, num) * rcp_nr(fma(c, num, den));
    double u = tp * tp;
    double p = c_atanp[0];
#pragma unroll
    for (int k = 1; k < 7; ++k) p = fma(p, u, c_atanp[k]);
    double th = fma(tp * u, p, tp) + ac;                  // atan(num/den)
    if (sw) th = 1.5707963267948966 - th;
    if (x < 0.0) th = 3.141592653589793 - th;
    return signbit(y) ? -th : th;
}

// Natural logarithm of a positive, finite, normal x: with x = 2^e m,
// m in [sqrt(1/2), sqrt(2)), log x = e ln 2 + 2 atanh(t), t = (m - 1)/(m + 1),
// |t| < B = (sqrt2 - 1)/(sqrt2 + 1) = 0.1716.  atanh t = t P(t^2) with P of
// degree 7, the odd Chebyshev interpolant of atanh on [-B, B] (nodes of
// degree 15, computed in extended precision, coefficients rounded): relative
// error below 1e-17, against 2^-56 for the Taylor series cut after eleven
// terms.  About 1-2 ulp.
__device__ inline double log_pos(double x)
{
    int e;
    double m = frexp(x, &e);                 // m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    double t = (m - 1.0) * rcp_nr(m + 1.0);
    double t2 = t * t;
    double p = c_logp[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) p = fma(p, t2, c_logp[k]);
    // ln 2 split so that e * ln2_hi is exact for |e| < 2^11
    const double ln2_hi = 0.693147180559890330187045037746;
    const double ln2_lo = 5.4979230187083711552420206e-14;
    return (double)e * ln2_hi + ((double)e * ln2_lo + 2.0 * t * p);
}


// ------------------------------------------------- P2P by leaf pairs
// The near field as work items over List-1 entries e = (target leaf b, source
// leaf a).  Each item writes the partial potential of b's targets due to a's
// sources into C[coff[e] + (i - pbeg[b])]; a final pass adds, per target, the
// partials of its List-1 entries in list order (deterministic).
//
// Symmetric items (a < b, every pair in the small-argument regime): since
// G(x, y) = G(y, x), one evaluation serves both directions: the row sum of
// target i and the column sum of source j, which goes to the partner entry
// e' = (a, b).  Diagonal items (a == b) evaluate each unordered pair once.
//
// Pair walk.  The R x C pairs of a tile (R, C <= 64) are spread over all 64
// lanes, so that every lane but those past the end of the last step is busy
// (one target per lane would idle 64 - R of them).  With F = min(R, C) and
// O = max(R, C), pair p has fast index f = p mod F, block g = p div F and
// other index o = (g + f) mod O.  Within a block the f are distinct and so
// are the o (F <= O).  A step (64 consecutive p) spans a few blocks; lane p
// adds its terms into slot g - g0 (g0 = the step's first block) of per-slot
// row and column sums, so no two lanes of a step touch the same slot entry,
// and the slots are added in slot order at the end: the result does not
// depend on timing.  Steps that span more than kPairSlots blocks make several
// passes over the slots: with F between 32 and 63 a step spans two or three
// blocks, and two slots (a second pass now and then) beat three, whose LDS
// costs a wavefront per SIMD.
constexpr int kPairSlots = 2;

struct PairWalk {
    int F, O, dF, rF;       // 64 = dF F + rF
    int f, g;               // this lane's pair
    __device__ void init(int F_, int O_, int t)
    {
        F = F_;
        O = O_;
        dF = 64 / F;
        rF = 64 - dF * F;
        f = t % F;
        g = t / F;
    }
    __device__ int other() const
    {
        int o = g + f;
        return o >= O ? o - O : o;
    }
    __device__ void next()
    {
        f += rF;
        g += dF;
        if (f >= F) {
            f -= F;
            ++g;
        }
    }
};

// Adds (xr, xi) to row slot sums rs[slot][ri] and (yr, yi) to column slot sums
// cs[slot][ci] for this lane's block, in as many passes as the step needs.
__device__ inline void slot_add(double (*rs)[64], double (*rsi)[64], double (*cs)[64], double (*csi)[64],
                                bool act, int b, int nsl, int ri, int ci, double xr, double xi,
                                double yr, double yi)
{
    for (int ph = 0; ph < nsl; ph += kPairSlots) {
        int sl = b - ph;
        if (act && sl >= 0 && sl < kPairSlots) {
            rs[sl][ri] += xr;
            rsi[sl][ri] += xi;
            cs[sl][ci] += yr;
            csi[sl][ci] += yi;
        }
    }
}

// (ar, ai) += h (wr + i wi) as four chained FMAs
__device__ inline void cfma2(double& ar, double& ai, cplx h, double wr, double wi)
{
    ar = fma(h.re, wr, ar);
    ar = fma(-h.im, wi, ar);
    ai = fma(h.re, wi, ai);
    ai = fma(h.im, wr, ai);
}

struct P2PMap {
    const int* row_of;      // target leaf of each List-1 entry
    const int* partner;     // entry (a, b) for entry (b, a)
    const int64_t* coff;    // offset of each entry's partial sums in C
    cplx* C;
};

// Coefficients of the two power series in x = -q behind H0:
// J0 = sum_k x^k / (k!)^2 and (2/pi) S with S = sum_k H_k x^k / (k!)^2 (H_k
// harmonic), the factor 2/pi of Y0 taken into the table.
struct SerCoef {
    double j, y;
};
constexpr int kSerTerms = 40;
struct SerTab {
    SerCoef c[kSerTerms];
};
constexpr SerTab make_ser_tab()
{
    SerTab t{};
    double a = 1.0, h = 0.0;
    t.c[0] = {1.0, 0.0};
    for (int k = 1; k < kSerTerms; ++k) {
        a /= (double)k * (double)k;
        h += 1.0 / (double)k;
        t.c[k] = {a, (2.0 / kPi) * h * a};
    }
    return t;
}
__constant__ SerTab c_ser = make_ser_tab();

// a - s b with the coefficient a in scalar registers.  Written as one
// instruction so that the scheduler cannot hoist it into a two-address FMA
// whose accumulator is a copy of a.
__device__ inline double fnms_s(double s, double b, double a)
{
    double r;
    asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(r) : "v"(s), "v"(b), "s"(a));
    return r;
}

// H0(kappa r) from s = r^2 by the power series with K terms (|kappa r| < 3).
// Both series have real coefficients, so they are evaluated at the complex x
// by Knuth's scheme (division by the real quadratic w^2 - 2 Re(x) w + |x|^2,
// whose roots are x and its conjugate): b_k = a_k + 2 Re(x) b_(k+1)
// - |x|^2 b_(k+2), then p(x) = x b_1 + a_0 - |x|^2 b_2.  Two FMAs per
// coefficient instead of a complex product; on |x| <= 2.25 its rounding
// error matches that of summing the terms.
__device__ inline cplx h0_series_s(double sr, double si, double k2, double lk2, int K)
{
    double n2 = sr * sr + si * si;                        // |s|^2
    double ln2 = log_pos(n2);                             // 2 log|s|
    double ag = arg2(sr, si);                             // arg q
    double xr = -k2 * sr, xi = -k2 * si;                  // x = -q
    double rr = 2.0 * xr, ss = (k2 * k2) * n2;            // 2 Re x, |x|^2
    // two steps per pass with the roles of the two registers alternating
    // (b_(k+1) in *1, b_(k+2) in *2 at the top); an odd K takes b_K first
    double bj1 = 0.0, by1 = 0.0, bj2 = 0.0, by2 = 0.0;
    int k = K;
    if (K & 1) {
        bj1 = c_ser.c[K].j;
        by1 = c_ser.c[K].y;
        --k;
    }
    for (; k >= 2; k -= 2) {
        SerCoef a = c_ser.c[k], a1 = c_ser.c[k - 1];
        bj2 = fma(rr, bj1, fnms_s(ss, bj2, a.j));         // b_k
        by2 = fma(rr, by1, fnms_s(ss, by2, a.y));
        bj1 = fma(rr, bj2, fnms_s(ss, bj1, a1.j));        // b_(k-1)
        by1 = fma(rr, by2, fnms_s(ss, by1, a1.y));
    }
    double jr = fma(xr, bj1, fma(-ss, bj2, 1.0)), ji = xi * bj1;
    double sr0 = fma(xr, by1, -ss * by2), si0 = xi * by1;  // S has a_0 = 0
    // Y0 = (2/pi)(log(z/2) + gamma) J0 - (2/pi) S, log(z/2) = log(q)/2
    double lr = fma(0.5 / kPi, ln2, (lk2 + 2.0 * kEuler) * (1.0 / kPi)), li = ag * (1.0 / kPi);
    double yr = fma(lr, jr, fma(-li, ji, -sr0)), yi = fma(lr, ji, fma(li, jr, -si0));
    return mk(jr - yi, ji + yr);                          // J0 + i Y0
}

// The near-field kernel value of a pair from s = r^2: MODE 1, the power
// series of H0 (2D Helmholtz, |kappa r| < 3, K terms); MODE 2, Log s = 2 log r
// (2D Laplace: log |s| from |s|^2 and arg s).  The final pass applies the
// constant ((i/4) or -(1/4 pi)).
template <int MODE>
__device__ inline cplx near_value(double sr, double si, double k2, double lk2, int K)
{
    if (MODE == 2) return mk(0.5 * log_pos(sr * sr + si * si), arg2(sr, si));
    return h0_series_s(sr, si, k2, lk2, K);
}

template <int MODE>
__global__ __launch_bounds__(64) void k_h2d_p2p_sym(const int* __restrict__ items, const int* __restrict__ nterm,
                                                    P2PMap mp, TreeView tv, PointsView pv, double kappa)
{
    __shared__ double s1r[64], s1i[64], s2r[64], s2i[64], ssr[64], ssi[64];   // source tile
    __shared__ double t1r[64], t1i[64], t2r[64], t2i[64], twr[64], twi[64];   // target tile
    __shared__ double rs[kPairSlots][64], rsi[kPairSlots][64], cs[kPairSlots][64], csi[kPairSlots][64];
    int e = items[blockIdx.x], K = nterm[blockIdx.x];
    int b = mp.row_of[e], a = tv.l1idx[e], ep = mp.partner[e];
    int64_t n = pv.n;
    int t = threadIdx.x;
    double k2 = 0.25 * kappa * kappa, lk2 = log(k2);
    int pb0 = tv.pbeg[b], pb1 = tv.pend[b], pa0 = tv.pbeg[a], pa1 = tv.pend[a];
    cplx* Crow = mp.C + mp.coff[e];
    cplx* Ccol = mp.C + mp.coff[ep];
    for (int i0 = pb0; i0 < pb1; i0 += 64) {
        int R = min(64, pb1 - i0);
        __syncthreads();
        if (t < R) {
            int i = i0 + t;
            t1r[t] = pv.xre[i]; t1i[t] = pv.xim[i];
            t2r[t] = pv.xre[n + i]; t2i[t] = pv.xim[n + i];
            twr[t] = pv.sre[i]; twi[t] = pv.sim[i];
        }
        for (int k = 0; k < kPairSlots; ++k) rs[k][t] = rsi[k][t] = 0.0;
        for (int j0 = pa0; j0 < pa1; j0 += 64) {
            int C = min(64, pa1 - j0);
            __syncthreads();
            if (t < C) {
                int j = j0 + t;
                s1r[t] = pv.xre[j]; s1i[t] = pv.xim[j];
                s2r[t] = pv.xre[n + j]; s2i[t] = pv.xim[n + j];
                ssr[t] = pv.sre[j]; ssi[t] = pv.sim[j];
            }
            for (int k = 0; k < kPairSlots; ++k) cs[k][t] = csi[k][t] = 0.0;
            __syncthreads();
            bool rfast = R <= C;                      // targets on the fast index
            int P = R * C;
            PairWalk w;
            w.init(rfast ? R : C, rfast ? C : R, t);
            for (int p0 = 0; p0 < P; p0 += 64) {
                bool act = p0 + t < P;
                int o = w.other();
                int i = rfast ? w.f : o, j = rfast ? o : w.f;
                int g0 = __builtin_amdgcn_readfirstlane(w.g);
                int last = min(63, P - 1 - p0);
                int nsl = __shfl(w.g, last, 64) - g0 + 1;
                double xr = 0.0, xi = 0.0, yr = 0.0, yi = 0.0;
                if (act) {
                    double d1r = t1r[i] - s1r[j], d1i = t1i[i] - s1i[j];
                    double d2r = t2r[i] - s2r[j], d2i = t2i[i] - s2i[j];
                    double sr = d1r * d1r - d1i * d1i + d2r * d2r - d2i * d2i;
                    double si = 2.0 * (d1r * d1i + d2r * d2i);
                    if (sr != 0.0 || si != 0.0) {
                        cplx h = near_value<MODE>(sr, si, k2, lk2, K);
                        cfma2(xr, xi, h, ssr[j], ssi[j]);
                        cfma2(yr, yi, h, twr[i], twi[i]);
                    }
                }
                slot_add(rs, rsi, cs, csi, act, w.g - g0, nsl, i, j, xr, xi, yr, yi);
                w.next();
            }
            __syncthreads();
            if (t < C) {
                double cr = cs[0][t], ci = csi[0][t];
                for (int k = 1; k < kPairSlots; ++k) {
                    cr += cs[k][t];
                    ci += csi[k][t];
                }
                cplx* cc = Ccol + (j0 - pa0) + t;
                if (i0 == pb0) *cc = mk(cr, ci);
                else *cc = *cc + mk(cr, ci);
            }
        }
        __syncthreads();
        if (t < R) {
            double ar = rs[0][t], ai = rsi[0][t];
            for (int k = 1; k < kPairSlots; ++k) {
                ar += rs[k][t];
                ai += rsi[k][t];
            }
            Crow[i0 + t - pb0] = mk(ar, ai);
        }
    }
}

// Diagonal items (a == b, at most 64 points, series regime): the L(L - 1)/2
// unordered pairs in the pair walk with F = O = L, where block g pairs point
// f with point (f + g + 1) mod L: blocks g < (L - 1)/2 hold L pairs each and,
// for even L, the last block the L/2 pairs (f, f + L/2), f < L/2.  Point f
// gains the term of its partner as a row sum and the partner that of f as a
// column sum.
template <int MODE>
__global__ __launch_bounds__(64) void k_h2d_p2p_diag(const int* __restrict__ items, const int* __restrict__ nterm,
                                                     P2PMap mp, TreeView tv, PointsView pv, double kappa)
{
    __shared__ double s1r[64], s1i[64], s2r[64], s2i[64], ssr[64], ssi[64];
    __shared__ double rs[kPairSlots][64], rsi[kPairSlots][64], cs[kPairSlots][64], csi[kPairSlots][64];
    int e = items[blockIdx.x], K = nterm[blockIdx.x];
    int b = mp.row_of[e];
    int64_t n = pv.n;
    int t = threadIdx.x;
    double k2 = 0.25 * kappa * kappa, lk2 = log(k2);
    int p0b = tv.pbeg[b], L = tv.pend[b] - p0b;
    if (t < L) {
        int j = p0b + t;
        s1r[t] = pv.xre[j]; s1i[t] = pv.xim[j];
        s2r[t] = pv.xre[n + j]; s2i[t] = pv.xim[n + j];
        ssr[t] = pv.sre[j]; ssi[t] = pv.sim[j];
    }
    for (int k = 0; k < kPairSlots; ++k) rs[k][t] = rsi[k][t] = cs[k][t] = csi[k][t] = 0.0;
    __syncthreads();
    int P = L * (L - 1) / 2;
    PairWalk w;
    w.init(L > 0 ? L : 1, L > 0 ? L : 1, t);
    for (int p0 = 0; p0 < P; p0 += 64) {
        bool act = p0 + t < P;
        int i = w.f;
        int j = i + w.g + 1;
        if (j >= L) j -= L;
        int g0 = __builtin_amdgcn_readfirstlane(w.g);
        int last = min(63, P - 1 - p0);
        int nsl = __shfl(w.g, last, 64) - g0 + 1;
        double xr = 0.0, xi = 0.0, yr = 0.0, yi = 0.0;
        if (act) {
            double d1r = s1r[i] - s1r[j], d1i = s1i[i] - s1i[j];
            double d2r = s2r[i] - s2r[j], d2i = s2i[i] - s2i[j];
            double sr = d1r * d1r - d1i * d1i + d2r * d2r - d2i * d2i;
            double si = 2.0 * (d1r * d1i + d2r * d2i);
            if (sr != 0.0 || si != 0.0) {
                cplx h = near_value<MODE>(sr, si, k2, lk2, K);
                cfma2(xr, xi, h, ssr[j], ssi[j]);
                cfma2(yr, yi, h, ssr[i], ssi[i]);
            }
        }
        slot_add(rs, rsi, cs, csi, act, w.g - g0, nsl, i, j, xr, xi, yr, yi);
        w.next();
    }
    __syncthreads();
    if (t < L) {
        double ar = rs[0][t], ai = rsi[0][t];
        for (int k = 1; k < kPairSlots; ++k) {
            ar += rs[k][t];
            ai += rsi[k][t];
        }
        for (int k = 0; k < kPairSlots; ++k) {
            ar += cs[k][t];
            ai += csi[k][t];
        }
        mp.C[mp.coff[e] + t] = mk(ar, ai);
    }
}

// Row items: one direction of an entry, by the general Hankel evaluation
// (MODE 0) or near_value<MODE> (the small-argument series with K terms, or
// Log s); a == b skips the self pair.
template <int MODE>
__global__ __launch_bounds__(64) void k_h2d_p2p_row(const int* __restrict__ items, const int* __restrict__ nterm,
                                                    P2PMap mp, TreeView tv, PointsView pv, double kappa)
{
    __shared__ double s1r[64], s1i[64], s2r[64], s2i[64], ssr[64], ssi[64];
    int e = items[blockIdx.x];
    int K = MODE == 1 ? nterm[blockIdx.x] : 0;
    int b = mp.row_of[e], a = tv.l1idx[e];
    int64_t n = pv.n;
    int t = threadIdx.x;
    double k2 = 0.25 * kappa * kappa, lk2 = log(k2);
    int pb0 = tv.pbeg[b], pb1 = tv.pend[b], pa0 = tv.pbeg[a], pa1 = tv.pend[a];
    cplx* Crow = mp.C + mp.coff[e];
    for (int i0 = pb0; i0 < pb1; i0 += 64) {
        int i = i0 + t;
        bool active = i < pb1;
        double x1r = 0, x1i = 0, x2r = 0, x2i = 0;
        if (active) {
            x1r = pv.xre[i]; x1i = pv.xim[i];
            x2r = pv.xre[n + i]; x2i = pv.xim[n + i];
        }
        double ar = 0.0, ai = 0.0;
        for (int j0 = pa0; j0 < pa1; j0 += 64) {
            int cnt = min(64, pa1 - j0);
            __syncthreads();
            if (t < cnt) {
                int j = j0 + t;
                s1r[t] = pv.xre[j]; s1i[t] = pv.xim[j];
                s2r[t] = pv.xre[n + j]; s2i[t] = pv.xim[n + j];
                ssr[t] = pv.sre[j]; ssi[t] = pv.sim[j];
            }
            __syncthreads();
            if (!active) continue;
            for (int q = 0; q < cnt; ++q) {
                if (j0 + q == i) continue;
                double d1r = x1r - s1r[q], d1i = x1i - s1i[q];
                double d2r = x2r - s2r[q], d2i = x2i - s2i[q];
                double sr = d1r * d1r - d1i * d1i + d2r * d2r - d2i * d2i;
                double si = 2.0 * (d1r * d1i + d2r * d2i);
                if (sr == 0.0 && si == 0.0) continue;
                cplx h = MODE != 0 ? near_value<MODE>(sr, si, k2, lk2, K)
                                   : hankel0_s(mk(sr, si), kappa, c_ghx, c_ghw);
                cfma2(ar, ai, h, ssr[q], ssi[q]);
            }
        }
        if (active) Crow[i - pb0] = mk(ar, ai);
    }
}

// Final pass: u[perm[i] - obase] = (i/4)(near + far) (Helmholtz) or
// -(1/4 pi)(near + far) (Laplace, whose sums are of Log s = 2 log r) at the
// targets, the near field summed over the target's List-1 entries in list
// order.
template <int LAP>
__global__ __launch_bounds__(64) void k_h2d_p2p_final(const int* __restrict__ leaves, P2PMap mp, TreeView tv,
                                                      const cplx* __restrict__ ufar, IoMap io,
                                                      double* __restrict__ out)
{
    int b = leaves[blockIdx.x];
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    int e0 = tv.l1off[b], e1 = tv.l1off[b + 1];
    for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
        int64_t p = (int64_t)io.perm[i] - io.obase;
        if (p < 0) continue;            // a source that is not a target
        cplx u = ufar[i];
        for (int e = e0; e < e1; ++e) u += mp.C[mp.coff[e] + (i - p0)];
        double vr = LAP ? u.re * (-0.25 / kPi) : -0.25 * u.im;
        double vi = LAP ? u.im * (-0.25 / kPi) : 0.25 * u.re;
        out[2 * p] = vr;
        out[2 * p + 1] = vi;
        if (!isfinite(vr) || !isfinite(vi)) atomicOr(io.nonfinite, 1);
    }
}

// ---------------------------------------------------------------- launchers
hipError_t h2d_p2m(const int* leaves, int nleaf, int pmax, const TreeView& tv, const PointsView& pv,
                   double kappa, cplx* mpole, hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    size_t lds = sizeof(cplx) * (size_t)(2 * pmax + 2) * kP2MChunk;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_h2d_p2m, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    k_h2d_p2m<<<nleaf, 64, lds, st>>>(leaves, nleaf, tv, pv, kappa, mpole);
    return hipGetLastError();
}

hipError_t h2d_gen_ops(const int* pair_b, int npairs, const int* tr_boxes, int ntr,
                       const TreeView& tv, double kappa, int lwin, const int64_t* o_m2l, cplx* g_m2l,
                       const int64_t* o_tr, cplx* g_m2m, cplx* g_l2l, hipStream_t st)
{
    if (npairs > 0) k_h2d_gen_m2l<<<(npairs + 63) / 64, 64, 0, st>>>(npairs, pair_b, tv, kappa, lwin, o_m2l, g_m2l);
    if (ntr > 0) k_h2d_gen_tr<<<(ntr + 63) / 64, 64, 0, st>>>(tr_boxes, ntr, tv, kappa, o_tr, g_m2m, g_l2l);
    return hipGetLastError();
}

// G lanes cover the output coefficients; levels with few boxes split the
// input sum over S = 256 / G groups so that the level still fills the chip.
hipError_t h2d_m2m(const int* boxes, int nb, int ncoef, const TreeView& tv, const H2DOps& ops, cplx* mpole,
                   hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    // long expansions (the coarse levels, few boxes each) split their source
    // terms over four times the lanes
    k_h2d_m2m<<<nb, ncoef > 32 ? 256 : 64, 0, st>>>(boxes, nb, tv, ops, mpole);
    return hipGetLastError();
}

// Entries per round of the window kernel and its LDS at expansion length P,
// for the plan's grouping of target boxes.
int h2d_m2l_w_slots(int P) { return 64 / ((2 * P + 1 + kWin - 1) / kWin); }
int h2d_m2l_w_waves() { return kM2LWWaves; }
size_t h2d_m2l_w_lds(int P, int W) { return m2l_w_lds(P, W); }

// boxes[0 .. nwin) (the levels whose operator fits FP64 unscaled) take the
// window kernel: grp[0 .. ngrp1) one wavefront each, grp[ngrp1 .. ngrp)
// (single boxes with many entries) kM2LWWaves wavefronts each;
// boxes[nwin .. total) the scaled kernel.
hipError_t h2d_m2l(const int* boxes, const int2* grp, int ngrp1, int ngrp, size_t lds1, size_t ldsw, int nwin,
                   int total, const TreeView& tv, const H2DOps& ops, const cplx* mpole, cplx* local,
                   hipStream_t st)
{
    size_t lmax = std::max(lds1, ldsw);
    if (ngrp > 0 && lmax > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_h2d_m2l_w, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lmax);
        if (e != hipSuccess) return e;
    }
    if (ngrp1 > 0) k_h2d_m2l_w<<<ngrp1, 64, lds1, st>>>(boxes, grp, ngrp1, tv, ops, mpole, local);
    if (ngrp > ngrp1)
        k_h2d_m2l_w<<<ngrp - ngrp1, 64 * kM2LWWaves, ldsw, st>>>(boxes, grp + ngrp1, ngrp - ngrp1, tv, ops, mpole,
                                                                 local);
    if (total > nwin) k_h2d_m2l<<<total - nwin, 64, 0, st>>>(boxes + nwin, total - nwin, tv, ops, mpole, local);
    return hipGetLastError();
}

hipError_t h2d_p2l(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   double kappa, cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    int pstride = P + 1;
    int chunk = (int)(48000 / (sizeof(cplx) * (2 * (size_t)pstride + 1)));
    chunk = chunk > 64 ? 64 : (chunk < 1 ? 1 : chunk);   // threads q and q + 64 share source q
    size_t lds = sizeof(cplx) * ((size_t)chunk * (2 * (size_t)pstride + 1) + 128);
    k_h2d_p2l<<<nb, 128, lds, st>>>(boxes, tv, pv, kappa, chunk, pstride, local);
    return hipGetLastError();
}

hipError_t h2d_l2l(const int* boxes, int nb, int ncoef, const TreeView& tv, const H2DOps& ops, cplx* local,
                   hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_h2d_l2l<<<nb, ncoef > 32 ? 256 : 64, 0, st>>>(boxes, nb, tv, ops, local);
    return hipGetLastError();
}

hipError_t h2d_leaf_far(const int* leaves, int nleaf, const M2PParts& m2p, int m2p_pmax, int top,
                        const TreeView& tv, const PointsView& pv, double kappa, const cplx* mpole,
                        const cplx* local, cplx* ufar, hipStream_t st)
{
    if (m2p.n > 0) {
        int threads = 64;
        size_t lds = (size_t)threads * (m2p_pmax + 1) * sizeof(cplx);
        k_h2d_m2p_part<<<m2p.n, threads, lds, st>>>(m2p.owner, m2p.poff, tv, pv, kappa, mpole, m2p.part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nleaf > 0)
        k_h2d_l2p<<<nleaf, 64, 0, st>>>(leaves, top, tv, pv, kappa, local, m2p.poff, m2p.part, ufar);
    return hipGetLastError();
}

hipError_t h2d_p2p(const H2DNear& nr, const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv,
                   double kappa, const cplx* ufar, const IoMap& io, double* out, int laplace, hipStream_t st)
{
    P2PMap mp{nr.row_of, nr.partner, nr.coff, nr.C};
    if (laplace) {
        if (nr.nsym > 0) k_h2d_p2p_sym<2><<<nr.nsym, 64, 0, st>>>(nr.sym, nr.sym_k, mp, tv, pv, 0.0);
        if (nr.ndiag > 0) k_h2d_p2p_diag<2><<<nr.ndiag, 64, 0, st>>>(nr.diag, nr.diag_k, mp, tv, pv, 0.0);
        if (nr.nser > 0) k_h2d_p2p_row<2><<<nr.nser, 64, 0, st>>>(nr.ser, nr.ser_k, mp, tv, pv, 0.0);
        if (nleaf > 0) k_h2d_p2p_final<1><<<nleaf, 64, 0, st>>>(leaves, mp, tv, ufar, io, out);
        return hipGetLastError();
    }
    if (nr.nsym > 0) k_h2d_p2p_sym<1><<<nr.nsym, 64, 0, st>>>(nr.sym, nr.sym_k, mp, tv, pv, kappa);
    if (nr.ndiag > 0) k_h2d_p2p_diag<1><<<nr.ndiag, 64, 0, st>>>(nr.diag, nr.diag_k, mp, tv, pv, kappa);
    if (nr.nser > 0) k_h2d_p2p_row<1><<<nr.nser, 64, 0, st>>>(nr.ser, nr.ser_k, mp, tv, pv, kappa);
    if (nr.ngen > 0) k_h2d_p2p_row<0><<<nr.ngen, 64, 0, st>>>(nr.gen, nullptr, mp, tv, pv, kappa);
    if (nleaf > 0) k_h2d_p2p_final<0><<<nleaf, 64, 0, st>>>(leaves, mp, tv, ufar, io, out);
    return hipGetLastError();
}

// |H_n(kappa R) J_n(kappa r)| for the expansion-length rule, scaled so that
// neither factor overflows.
double h2d_nterms_crit(double kappa, double R, double r, int n)
{
    host_gh();
    double rs = fmin(1.0, kappa * R);
    cplx hp[2 * kPMax2D + 4], hn[2 * kPMax2D + 4], jp[2 * kPMax2D + 4], jn[2 * kPMax2D + 4];
    hseq2(mk(R, 0.0), mk(0.0, 0.0), kappa, rs, n, h_ghx, h_ghw, hp, hn, 1);
    jseq2(mk(r, 0.0), mk(0.0, 0.0), kappa, rs, n, jp, jn, 1);
    return sqrt(cabs2(hp[n] * jp[n]));
}

}  // namespace cfmm
