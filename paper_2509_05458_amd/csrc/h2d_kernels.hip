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
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ghx), h_ghx, sizeof(h_ghx));
    if (e != hipSuccess) return e;
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

__global__ __launch_bounds__(128) void k_h2d_p2m(const int* __restrict__ boxes, TreeView tv,
                                                 PointsView pv, double kappa, cplx* __restrict__ mpole)
{
    __shared__ cplx spos[kChunk][kPMax2D + 1];
    __shared__ cplx sneg[kChunk][kPMax2D + 1];
    __shared__ cplx ssig[kChunk];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    double r = tv.rs[l];
    int nbx = tv.nbox;
    int64_t n = pv.n;
    cplx c1 = mk(tv.cre[b], tv.cim[b]), c2 = mk(tv.cre[nbx + b], tv.cim[nbx + b]);
    int t = threadIdx.x, ncoef = 2 * P + 1, mm = t - P;
    cplx acc = mk(0.0, 0.0);
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    for (int j0 = p0; j0 < p1; j0 += kChunk) {
        int cnt = min(kChunk, p1 - j0);
        if (t < cnt) {
            int j = j0 + t;
            cplx y1 = mk(pv.xre[j] - c1.re, pv.xim[j] - c1.im);
            cplx y2 = mk(pv.xre[n + j] - c2.re, pv.xim[n + j] - c2.im);
            jseq2(y1, y2, kappa, r, P, &spos[t][0], &sneg[t][0], 1);
            ssig[t] = mk(pv.sre[j], pv.sim[j]);
        }
        __syncthreads();
        if (t < ncoef) {
            for (int q = 0; q < cnt; ++q) {
                cplx v = (mm >= 0) ? sneg[q][mm] : ((mm & 1) ? -spos[q][-mm] : spos[q][-mm]);
                acc += v * ssig[q];
            }
        }
        __syncthreads();
    }
    if (t < ncoef) mpole[tv.eoff[b] + t] = acc;
}

// ------------------------------------------------------------------ M2M
__global__ __launch_bounds__(128) void k_h2d_m2m(const int* __restrict__ boxes, TreeView tv,
                                                 double kappa, cplx* __restrict__ mpole)
{
    __shared__ cplx gp[4][2 * kPMax2D + 1];
    __shared__ cplx gn[4][2 * kPMax2D + 1];
    __shared__ cplx mc[4][kNCoef2DMax];
    __shared__ double pw[2 * kPMax2D + 2];
    __shared__ double rat[kPMax2D + 1];
    int p = boxes[blockIdx.x];
    int l = tv.level[p];
    int Pp = tv.P[l], Pc = tv.P[l + 1];
    double rp = tv.rs[l], rc = tv.rs[l + 1];
    int c0 = tv.child0[p], nc = tv.nchild[p];
    int K = Pp + Pc, nbx = tv.nbox, ncc = 2 * Pc + 1;
    int t = threadIdx.x;
    if (t < nc) {
        int c = c0 + t;
        cplx d1 = mk(tv.cre[p] - tv.cre[c], tv.cim[p] - tv.cim[c]);
        cplx d2 = mk(tv.cre[nbx + p] - tv.cre[nbx + c], tv.cim[nbx + p] - tv.cim[nbx + c]);
        jseq2(d1, d2, kappa, rc, K, &gp[t][0], &gn[t][0], 1);
    }
    for (int e = t; e <= 2 * Pc; e += blockDim.x) pw[e] = pow(rc, (double)e);
    for (int j = t; j <= Pp; j += blockDim.x) rat[j] = pow(rc / rp, (double)j);
    for (int q = t; q < nc * ncc; q += blockDim.x) {
        int ci = q / ncc, k = q - ci * ncc;
        mc[ci][k] = mpole[tv.eoff[c0 + ci] + k];
    }
    __syncthreads();
    if (t < 2 * Pp + 1) {
        int mm = t - Pp, am = iabs_(mm);
        cplx acc = mk(0.0, 0.0);
        for (int ci = 0; ci < nc; ++ci) {
            for (int nn = -Pc; nn <= Pc; ++nn) {
                int k = nn - mm;
                int e = iabs_(k) + iabs_(nn) - am;
                acc += (pw[e] * gen_at(gp[ci], gn[ci], k)) * mc[ci][nn + Pc];
            }
        }
        mpole[tv.eoff[p] + t] = rat[am] * acc;
    }
}

// ------------------------------------------------------------- M2L + P2L
constexpr int kM2LBatch = 8;

__global__ __launch_bounds__(128) void k_h2d_m2l(const int* __restrict__ boxes, TreeView tv,
                                                 PointsView pv, double kappa,
                                                 const cplx* __restrict__ mpole,
                                                 cplx* __restrict__ local)
{
    __shared__ cplx gp[kM2LBatch][2 * kPMax2D + 1];
    __shared__ cplx gn[kM2LBatch][2 * kPMax2D + 1];
    __shared__ cplx ms[kM2LBatch][kNCoef2DMax];
    __shared__ double pw[2 * kPMax2D + 2];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    double r = tv.rs[l];
    int nbx = tv.nbox, ncoef = 2 * P + 1;
    int64_t n = pv.n;
    int t = threadIdx.x, mm = t - P, am = iabs_(mm);
    for (int e = t; e <= 2 * P; e += blockDim.x) pw[e] = pow(r, (double)e);
    cplx acc = mk(0.0, 0.0);
    int e0 = tv.l2off[b], e1 = tv.l2off[b + 1];
    for (int eb = e0; eb < e1; eb += kM2LBatch) {
        int cnt = min(kM2LBatch, e1 - eb);
        if (t < cnt) {
            int a = tv.l2idx[eb + t];
            cplx d1 = mk(tv.cre[b] - tv.cre[a], tv.cim[b] - tv.cim[a]);
            cplx d2 = mk(tv.cre[nbx + b] - tv.cre[nbx + a], tv.cim[nbx + b] - tv.cim[nbx + a]);
            hseq2(d1, d2, kappa, r, 2 * P, c_ghx, c_ghw, &gp[t][0], &gn[t][0], 1);
        }
        for (int q = t; q < cnt * ncoef; q += blockDim.x) {
            int ai = q / ncoef, k = q - ai * ncoef;
            ms[ai][k] = mpole[tv.eoff[tv.l2idx[eb + ai]] + k];
        }
        __syncthreads();
        if (t < ncoef) {
            for (int ai = 0; ai < cnt; ++ai) {
                for (int nn = -P; nn <= P; ++nn) {
                    int k = nn - mm;
                    int e = am + iabs_(nn) - iabs_(k);
                    acc += (pw[e] * gen_at(gp[ai], gn[ai], k)) * ms[ai][nn + P];
                }
            }
        }
        __syncthreads();
    }
    // P2L: sources of the coarser leaves in List 4, directly into the local
    cplx cb1 = mk(tv.cre[b], tv.cim[b]), cb2 = mk(tv.cre[nbx + b], tv.cim[nbx + b]);
    for (int e = tv.l4off[b]; e < tv.l4off[b + 1]; ++e) {
        int c = tv.l4idx[e];
        int q0 = tv.pbeg[c], q1 = tv.pend[c];
        for (int j0 = q0; j0 < q1; j0 += kM2LBatch) {
            int cnt = min(kM2LBatch, q1 - j0);
            if (t < cnt) {
                int j = j0 + t;
                cplx y1 = mk(pv.xre[j] - cb1.re, pv.xim[j] - cb1.im);
                cplx y2 = mk(pv.xre[n + j] - cb2.re, pv.xim[n + j] - cb2.im);
                hseq2(y1, y2, kappa, r, P, c_ghx, c_ghw, &gp[t][0], &gn[t][0], 1);
                ms[t][0] = mk(pv.sre[j], pv.sim[j]);
            }
            __syncthreads();
            if (t < ncoef) {
                for (int q = 0; q < cnt; ++q) {
                    cplx v = (mm >= 0) ? gn[q][mm] : ((mm & 1) ? -gp[q][-mm] : gp[q][-mm]);
                    acc += v * ms[q][0];
                }
            }
            __syncthreads();
        }
    }
    if (t < ncoef) local[tv.eoff[b] + t] = acc;
}

// ------------------------------------------------------------------ L2L
__global__ __launch_bounds__(128) void k_h2d_l2l(const int* __restrict__ boxes, TreeView tv,
                                                 double kappa, cplx* __restrict__ local)
{
    __shared__ cplx gp[2 * kPMax2D + 1];
    __shared__ cplx gn[2 * kPMax2D + 1];
    __shared__ cplx lp[kNCoef2DMax];
    __shared__ double pw[2 * kPMax2D + 2];
    __shared__ double rat[kPMax2D + 1];
    int c = boxes[blockIdx.x];
    int p = tv.parent[c];
    int lc = tv.level[c];
    int Pc = tv.P[lc], Pp = tv.P[lc - 1];
    double rc = tv.rs[lc], rp = tv.rs[lc - 1];
    int K = Pp + Pc, nbx = tv.nbox;
    int t = threadIdx.x;
    if (t == 0) {
        cplx d1 = mk(tv.cre[c] - tv.cre[p], tv.cim[c] - tv.cim[p]);
        cplx d2 = mk(tv.cre[nbx + c] - tv.cre[nbx + p], tv.cim[nbx + c] - tv.cim[nbx + p]);
        jseq2(d1, d2, kappa, rp, K, gp, gn, 1);
    }
    for (int e = t; e <= 2 * Pc; e += blockDim.x) pw[e] = pow(rp, (double)e);
    for (int j = t; j <= Pc; j += blockDim.x) rat[j] = pow(rc / rp, (double)j);
    for (int k = t; k < 2 * Pp + 1; k += blockDim.x) lp[k] = local[tv.eoff[p] + k];
    __syncthreads();
    if (t < 2 * Pc + 1) {
        int mm = t - Pc, am = iabs_(mm);
        cplx acc = mk(0.0, 0.0);
        for (int nn = -Pp; nn <= Pp; ++nn) {
            int k = nn - mm;
            int e = iabs_(k) + am - iabs_(nn);
            acc += (pw[e] * gen_at(gp, gn, k)) * lp[nn + Pp];
        }
        local[tv.eoff[c] + t] += rat[am] * acc;
    }
}

// ------------------------------------------------------------- L2P + M2P
__global__ void k_h2d_leaf_far(const int* __restrict__ leaves, int top, TreeView tv, PointsView pv,
                               double kappa, const cplx* __restrict__ mpole,
                               const cplx* __restrict__ local, cplx* __restrict__ ufar)
{
    extern __shared__ cplx rows[];      // rows[k * blockDim.x + thread]
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    int nbx = tv.nbox, st = blockDim.x, t = threadIdx.x;
    int64_t n = pv.n;
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    for (int i0 = p0; i0 < p1; i0 += st) {
        int i = i0 + t;
        if (i >= p1) break;
        cplx u = mk(0.0, 0.0);
        if (l >= top) {
            cplx x1 = mk(pv.xre[i], pv.xim[i]), x2 = mk(pv.xre[n + i], pv.xim[n + i]);
            int P = tv.P[l];
            double r = tv.rs[l];
            cplx X1 = x1 - mk(tv.cre[b], tv.cim[b]), X2 = x2 - mk(tv.cre[nbx + b], tv.cim[nbx + b]);
            cplx bp, bm;
            bool fact;
            jcore2(X1, X2, kappa, r, P, rows + t, st, &bp, &bm, &fact);
            const cplx* L = local + tv.eoff[b] + P;
            cplx pp = mk(1.0, 0.0), pm = mk(1.0, 0.0);
            for (int k = 0; k <= P; ++k) {
                cplx term = pp * L[k];
                if (k > 0) {
                    cplx v = pm * L[-k];
                    term += (k & 1) ? -v : v;
                }
                u += rows[k * st + t] * term;
                double f = fact ? 1.0 / (k + 1) : 1.0;
                pp = pp * bp * f;
                pm = pm * bm * f;
            }
            for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) {
                int a = tv.l3idx[e];
                int la = tv.level[a];
                int Pa = tv.P[la];
                double ra = tv.rs[la];
                cplx Y1 = x1 - mk(tv.cre[a], tv.cim[a]), Y2 = x2 - mk(tv.cre[nbx + a], tv.cim[nbx + a]);
                hcore2(Y1, Y2, kappa, ra, Pa, c_ghx, c_ghw, rows + t, st, &bp, &bm);
                const cplx* M = mpole + tv.eoff[a] + Pa;
                pp = mk(1.0, 0.0);
                pm = mk(1.0, 0.0);
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
            }
        }
        ufar[i] = u;
    }
}

// ------------------------------------------------------------------ P2P
// One workgroup (one wavefront) per target leaf; each lane keeps a target in
// registers while source tiles of the leaves in List 1 are staged in LDS as
// SoA doubles (coalesced loads, broadcast reads).  Writes
// u[perm[i]] = (i/4) (near + far) in the caller's order.
__global__ __launch_bounds__(64) void k_h2d_p2p(const int* __restrict__ leaves, TreeView tv,
                                                PointsView pv, double kappa,
                                                const cplx* __restrict__ ufar,
                                                const int* __restrict__ perm, double* __restrict__ out)
{
    __shared__ double s1r[64], s1i[64], s2r[64], s2i[64], ssr[64], ssi[64];
    int b = leaves[blockIdx.x];
    int64_t n = pv.n;
    int t = threadIdx.x;
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    int e0 = tv.l1off[b], e1 = tv.l1off[b + 1];
    for (int i0 = p0; i0 < p1; i0 += 64) {
        int i = i0 + t;
        bool active = i < p1;
        double x1r = 0, x1i = 0, x2r = 0, x2i = 0;
        if (active) {
            x1r = pv.xre[i]; x1i = pv.xim[i];
            x2r = pv.xre[n + i]; x2i = pv.xim[n + i];
        }
        double ar = 0.0, ai = 0.0;
        for (int e = e0; e < e1; ++e) {
            int a = tv.l1idx[e];
            int q0 = tv.pbeg[a], q1 = tv.pend[a];
            for (int j0 = q0; j0 < q1; j0 += 64) {
                int cnt = min(64, q1 - j0);
                __syncthreads();
                if (t < cnt) {
                    int j = j0 + t;
                    s1r[t] = pv.xre[j]; s1i[t] = pv.xim[j];
                    s2r[t] = pv.xre[n + j]; s2i[t] = pv.xim[n + j];
                    ssr[t] = pv.sre[j]; ssi[t] = pv.sim[j];
                }
                __syncthreads();
                if (active) {
                    for (int q = 0; q < cnt; ++q) {
                        if (j0 + q == i) continue;
                        double d1r = x1r - s1r[q], d1i = x1i - s1i[q];
                        double d2r = x2r - s2r[q], d2i = x2i - s2i[q];
                        cplx s = mk(d1r * d1r - d1i * d1i + d2r * d2r - d2i * d2i,
                                    2.0 * (d1r * d1i + d2r * d2i));
                        if (s.re == 0.0 && s.im == 0.0) continue;
                        cplx h = hankel0_s(s, kappa, c_ghx, c_ghw);
                        ar += h.re * ssr[q] - h.im * ssi[q];
                        ai += h.re * ssi[q] + h.im * ssr[q];
                    }
                }
            }
        }
        if (active) {
            cplx f = ufar[i];
            double tr = ar + f.re, ti = ai + f.im;
            int64_t p = perm[i];
            out[2 * p] = -0.25 * ti;      // (i/4) (tr + i ti)
            out[2 * p + 1] = 0.25 * tr;
        }
    }
}

// ---------------------------------------------------------------- launchers
hipError_t h2d_p2m(const int* boxes, int nb, const TreeView& tv, const PointsView& pv,
                   double kappa, cplx* mpole, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_h2d_p2m<<<nb, 128, 0, st>>>(boxes, tv, pv, kappa, mpole);
    return hipGetLastError();
}

hipError_t h2d_m2m(const int* boxes, int nb, const TreeView& tv, double kappa, cplx* mpole,
                   hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_h2d_m2m<<<nb, 128, 0, st>>>(boxes, tv, kappa, mpole);
    return hipGetLastError();
}

hipError_t h2d_m2l(const int* boxes, int nb, const TreeView& tv, const PointsView& pv,
                   double kappa, const cplx* mpole, cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_h2d_m2l<<<nb, 128, 0, st>>>(boxes, tv, pv, kappa, mpole, local);
    return hipGetLastError();
}

hipError_t h2d_l2l(const int* boxes, int nb, const TreeView& tv, double kappa, cplx* local,
                   hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_h2d_l2l<<<nb, 128, 0, st>>>(boxes, tv, kappa, local);
    return hipGetLastError();
}

hipError_t h2d_leaf_far(const int* leaves, int nleaf, int top, int pmax, const TreeView& tv,
                        const PointsView& pv, double kappa, const cplx* mpole, const cplx* local,
                        cplx* ufar, hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    int threads = 64;
    size_t lds = (size_t)threads * (pmax + 1) * sizeof(cplx);
    while (lds > 65536 && threads > 8) {
        threads /= 2;
        lds = (size_t)threads * (pmax + 1) * sizeof(cplx);
    }
    k_h2d_leaf_far<<<nleaf, threads, lds, st>>>(leaves, top, tv, pv, kappa, mpole, local, ufar);
    return hipGetLastError();
}

hipError_t h2d_p2p(const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv,
                   double kappa, const cplx* ufar, const int* perm, double* out, int mixed,
                   hipStream_t st)
{
    (void)mixed;
    if (nleaf <= 0) return hipSuccess;
    k_h2d_p2p<<<nleaf, 64, 0, st>>>(leaves, tv, pv, kappa, ufar, perm, out);
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
