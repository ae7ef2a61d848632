// 2D Laplace complex-coordinate FMM kernels (Sec. 4.2, with the multilevel
// steps of Sec. 6.4).  G = -(1/2 pi) log r with r the principal root of
// (x - y).(x - y).
//
// A point x in C^2 relative to a centre c is carried by the two complex
// numbers z = (x1 - c1) + i (x2 - c2) and w = (x1 - c1) - i (x2 - c2): in
// complex polar coordinates z = r e^{i phi}, w = r e^{-i phi} and r^2 = z w,
// so e^{i n phi} / r^n = w^-n and e^{-i n phi} / r^n = z^-n.  The expansions
// of the paper (multipole: M_0 log r + sum M_n^+ e^{in phi}/r^n + M_n^-
// e^{-in phi}/r^n; local: L_0 + sum L_n^+ r^n e^{in phi} + L_n^- r^n
// e^{-in phi}) become two power series, one in z and one in w:
//
//   multipole  u = M0 log r + sum_n A_n z^-n + B_n w^-n,
//              A_n = -(1/2n) sum sigma z_y^n,  B_n = -(1/2n) sum sigma w_y^n
//   local      u = L0 + sum_n C_n z^n + D_n w^n,
//              L0 = sum sigma log r_y,  C_n = -(1/2n) sum sigma z_y^-n,
//              D_n = -(1/2n) sum sigma w_y^-n
//
// (log r_xy = log r_x + Log(1 - z_y/z_x)/2 + Log(1 - w_y/w_x)/2 under the
// separation of the lemma of Sec. 4.1).  The translations are the binomial
// identities of Sec. 4.2 in each variable; with d = new centre - old centre
// (z_d, w_d its two variables) and every coefficient scaled by its level's
// box width w_l (A_n / w_l^n, C_n w_l^n; z-hat = z / w_l):
//
//   M2M  A'_k = -(1/2k) zd^k M0 + sum_{n<=k} C(k-1, n-1) zd^(k-n) 2^-n A_n,   zd = (c_child - c_parent)/w_p
//   M2L  C_k += -(1/2k) t^k M0 + sum_n (-1)^n C(n+k-1, k) t^(n+k) A_n,         t = w / (z_src - z_trg)
//        L0  += M0 log r0 + sum_n (-1)^n t^n A_n   (and the same in w with B, D)
//   L2L  C'_k = sum_{n>=k} C(n, k) zd^(n-k) 2^-k C_n,  L0' = L0 + sum_n zd^n C_n,   zd = (c_child - c_parent)/w_p
//
// The M2L term of M0 in C_k is -(1/2k) t^k M0: the expansion of
// M0 log r about the target centre (the paper's formula prints -1/2).
// Storage per box: 2P+1 complex values, e[P] = M0 or L0, e[P + n] the z
// series and e[P - n] the w series, n = 1..P.  The far field is returned as
// 2 sum log r sigma, the convention of the near field (which sums Log s =
// 2 log r); the final pass applies -1/(4 pi).
#include "common.hpp"
#include "kernels.hpp"

namespace cfmm {

namespace {

constexpr int kL2DRcp = 2 * kPMax2D + 2;
__constant__ double c_l2d_rcp[kL2DRcp];        // 1/m, c_l2d_rcp[0] = 0

__device__ inline cplx zvar(cplx a1, cplx a2) { return mk(a1.re - a2.im, a1.im + a2.re); }   // a1 + i a2
__device__ inline cplx wvar(cplx a1, cplx a2) { return mk(a1.re + a2.im, a1.im - a2.re); }   // a1 - i a2

// log r with r the principal root of z w: Log(z w)/2 (Re(z w) > 0 for the
// separated pairs the expansions serve)
__device__ inline cplx log_r(cplx z, cplx w)
{
    cplx s = z * w;
    return mk(0.5 * log(hypot(s.re, s.im)), 0.5 * atan2(s.im, s.re));
}

__device__ inline void centre2(const TreeView& tv, int b, cplx& c1, cplx& c2)
{
    c1 = mk(tv.cre[b], tv.cim[b]);
    c2 = mk(tv.cre[tv.nbox + b], tv.cim[tv.nbox + b]);
}

// z and w of point i relative to (c1, c2), times s
__device__ inline void point_zw(const PointsView& pv, int i, cplx c1, cplx c2, double s, cplx& z, cplx& w)
{
    int64_t n = pv.n;
    cplx a1 = mk(pv.xre[i] - c1.re, pv.xim[i] - c1.im);
    cplx a2 = mk(pv.xre[n + i] - c2.re, pv.xim[n + i] - c2.im);
    z = zvar(a1, a2) * s;
    w = wvar(a1, a2) * s;
}

constexpr int kL2DChunk = 64;

// P2M (one block of 64 per leaf) and P2L (one block per List-4 target box):
// a chunk of source points is staged in LDS as (z-hat, w-hat, sigma), then
// thread q owns output e[q] (q < 2P+1; q + 64 as well when 2P+1 > 64) and
// sums over the chunk in point order.  P2M: powers z-hat^n; P2L: the source
// boxes of the box's List 4, powers z-hat^-n and L0 = sum sigma log r.
template <bool LOCAL>
__global__ __launch_bounds__(64) void k_l2d_p2x(const int* __restrict__ boxes, TreeView tv, PointsView pv,
                                                cplx* __restrict__ coef)
{
    __shared__ cplx zs[kL2DChunk], ws[kL2DChunk], ss[kL2DChunk], lr[kL2DChunk];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l], nc = 2 * P + 1;
    double sc = tv.rs[l];                  // 1 / w_l
    double w_l = 1.0 / sc;
    int t = threadIdx.x;
    cplx c1, c2;
    centre2(tv, b, c1, c2);
    cplx acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
    int e0 = LOCAL ? tv.l4off[b] : 0, e1 = LOCAL ? tv.l4off[b + 1] : 1;
    for (int e = e0; e < e1; ++e) {
        int a = LOCAL ? tv.l4idx[e] : b;
        int p0 = tv.pbeg[a], p1 = tv.pend[a];
        for (int j0 = p0; j0 < p1; j0 += kL2DChunk) {
            int cnt = min(kL2DChunk, p1 - j0);
            __syncthreads();
            if (t < cnt) {
                cplx z, w;
                point_zw(pv, j0 + t, c1, c2, sc, z, w);
                if (LOCAL) {
                    // log r_y of the unscaled offset: log(w_l) + log r of the scaled one
                    cplx g = log_r(z, w);
                    lr[t] = mk(g.re + log(w_l), g.im);
                    z = cinv(z);
                    w = cinv(w);
                }
                zs[t] = z;
                ws[t] = w;
                ss[t] = mk(pv.sre[j0 + t], pv.sim[j0 + t]);
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int q = t + 64 * h;
                if (q >= nc) continue;
                int k = q - P;                         // > 0: z series, < 0: w series
                int m = k < 0 ? -k : k;
                double f = -0.5 * c_l2d_rcp[m];        // -1/(2m)
                for (int j = 0; j < cnt; ++j) {
                    cplx v;
                    if (k == 0) {
                        v = LOCAL ? lr[j] : mk(1.0, 0.0);
                    } else {
                        cplx base = k > 0 ? zs[j] : ws[j];
                        // base^m by squaring
                        cplx r = mk(1.0, 0.0), p = base;
                        for (int mm = m; mm; mm >>= 1) {
                            if (mm & 1) r = r * p;
                            p = p * p;
                        }
                        v = r * f;
                    }
                    cfma(acc[h], v, ss[j]);
                }
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int q = t + 64 * h;
        if (q < nc) {
            cplx* o = coef + tv.eoff[b];
            if (LOCAL) o[q] = o[q] + acc[h];      // after M2L on the same stream
            else o[q] = acc[h];
        }
    }
}

// M2M: one block per parent box; thread q owns output e[q] and adds the
// shifted expansions of the children in child order.  Powers of the child
// offset zd, wd sit in LDS.
__global__ __launch_bounds__(128) void k_l2d_m2m(const int* __restrict__ boxes, TreeView tv,
                                                 cplx* __restrict__ mpole)
{
    __shared__ cplx pz[kPMax2D + 1], pw[kPMax2D + 1], src[kNCoef2DMax];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l], nc = 2 * P + 1;
    int Pc = tv.P[l + 1];
    double sc = tv.rs[l];
    int t = threadIdx.x;
    cplx cp1, cp2;
    centre2(tv, b, cp1, cp2);
    cplx acc = mk(0.0, 0.0);
    for (int c = tv.child0[b]; c < tv.child0[b] + tv.nchild[b]; ++c) {
        __syncthreads();
        const cplx* M = mpole + tv.eoff[c];
        for (int i = t; i < 2 * Pc + 1; i += blockDim.x) src[i] = M[i];
        if (t < 2) {
            cplx cc1, cc2;
            centre2(tv, c, cc1, cc2);
            cplx a1 = cc1 - cp1, a2 = cc2 - cp2;
            cplx d = (t == 0 ? zvar(a1, a2) : wvar(a1, a2)) * sc;
            cplx* pp = t == 0 ? pz : pw;
            cplx v = mk(1.0, 0.0);
            for (int j = 0; j <= P; ++j) {
                pp[j] = v;
                v = v * d;
            }
        }
        __syncthreads();
        if (t >= nc) continue;
        int k = t - P;
        if (k == 0) {
            acc += src[Pc];
            continue;
        }
        int m = k < 0 ? -k : k;
        const cplx* pd = k > 0 ? pz : pw;
        int sgn = k > 0 ? 1 : -1;
        cplx v = pd[m] * (src[Pc] * (-0.5 * c_l2d_rcp[m]));
        double bin = 1.0, h = 0.5;                 // C(m-1, n-1), 2^-n at n = 1
        for (int n = 1; n <= m && n <= Pc; ++n) {
            cfma(v, pd[m - n] * (bin * h), src[Pc + sgn * n]);
            bin = bin * (double)(m - n) * c_l2d_rcp[n];
            h *= 0.5;
        }
        acc += v;
    }
    if (t < nc) mpole[tv.eoff[b] + t] = acc;
}

// M2L: one block per target box; for each List-2 source box the powers
// t^j = (w / (z_a - z_b))^j (and in w) for j <= 2P sit in LDS, and thread q
// adds its output's terms.
__global__ __launch_bounds__(128) void k_l2d_m2l(const int* __restrict__ boxes, int nboxes, TreeView tv,
                                                 const cplx* __restrict__ mpole, cplx* __restrict__ local)
{
    __shared__ cplx pz[2 * kPMax2D + 2], pw[2 * kPMax2D + 2], src[kNCoef2DMax];
    __shared__ cplx lg;
    int b = boxes[xcd_contiguous(blockIdx.x, nboxes)];
    int l = tv.level[b];
    int P = tv.P[l], nc = 2 * P + 1;
    double sc = tv.rs[l];
    int t = threadIdx.x;
    cplx cb1, cb2;
    centre2(tv, b, cb1, cb2);
    cplx acc = mk(0.0, 0.0);
    for (int e = tv.l2off[b]; e < tv.l2off[b + 1]; ++e) {
        int a = tv.l2idx[e];
        __syncthreads();
        const cplx* M = mpole + tv.eoff[a];
        for (int i = t; i < nc; i += blockDim.x) src[i] = M[i];
        if (t < 2) {
            cplx ca1, ca2;
            centre2(tv, a, ca1, ca2);
            cplx a1 = ca1 - cb1, a2 = ca2 - cb2;
            cplx z0 = zvar(a1, a2), w0 = wvar(a1, a2);
            if (t == 0) lg = log_r(z0, w0);             // log r0, unscaled
            cplx tt = cinv((t == 0 ? z0 : w0) * sc);
            cplx* pp = t == 0 ? pz : pw;
            cplx v = mk(1.0, 0.0);
            for (int j = 0; j <= 2 * P; ++j) {
                pp[j] = v;
                v = v * tt;
            }
        }
        __syncthreads();
        if (t >= nc) continue;
        int k = t - P;
        cplx M0 = src[P];
        if (k == 0) {
            cplx v = M0 * lg;
            for (int n = 1; n <= P; ++n) {
                double sg = (n & 1) ? -1.0 : 1.0;
                cfma(v, pz[n] * sg, src[P + n]);
                cfma(v, pw[n] * sg, src[P - n]);
            }
            acc += v;
            continue;
        }
        int m = k < 0 ? -k : k;
        const cplx* pt = k > 0 ? pz : pw;
        int sgn = k > 0 ? 1 : -1;
        cplx v = pt[m] * (M0 * (-0.5 * c_l2d_rcp[m]));
        double bin = 1.0;                              // C(n+m-1, m) at n = 1
        for (int n = 1; n <= P; ++n) {
            double f = (n & 1) ? -bin : bin;
            cfma(v, pt[n + m] * f, src[P + sgn * n]);
            bin = bin * (double)(n + m) * c_l2d_rcp[n];
        }
        acc += v;
    }
    if (t < nc) local[tv.eoff[b] + t] = acc;
}

// L2L: one block per child box, from its parent's local expansion.
__global__ __launch_bounds__(128) void k_l2d_l2l(const int* __restrict__ boxes, TreeView tv,
                                                 cplx* __restrict__ local)
{
    __shared__ cplx pz[kPMax2D + 1], pw[kPMax2D + 1], src[kNCoef2DMax];
    int c = boxes[blockIdx.x];
    int p = tv.parent[c];
    int l = tv.level[c];
    int P = tv.P[l], nc = 2 * P + 1, Pp = tv.P[l - 1];
    double scp = tv.rs[l - 1];
    int t = threadIdx.x;
    const cplx* Lp = local + tv.eoff[p];
    for (int i = t; i < 2 * Pp + 1; i += blockDim.x) src[i] = Lp[i];
    if (t < 2) {
        cplx cc1, cc2, cp1, cp2;
        centre2(tv, c, cc1, cc2);
        centre2(tv, p, cp1, cp2);
        cplx a1 = cc1 - cp1, a2 = cc2 - cp2;
        cplx d = (t == 0 ? zvar(a1, a2) : wvar(a1, a2)) * scp;
        cplx* pp = t == 0 ? pz : pw;
        cplx v = mk(1.0, 0.0);
        for (int j = 0; j <= Pp; ++j) {
            pp[j] = v;
            v = v * d;
        }
    }
    __syncthreads();
    if (t >= nc) return;
    int k = t - P;
    cplx v;
    if (k == 0) {
        v = src[Pp];
        for (int n = 1; n <= Pp; ++n) {
            cfma(v, pz[n], src[Pp + n]);
            cfma(v, pw[n], src[Pp - n]);
        }
    } else {
        int m = k < 0 ? -k : k;
        const cplx* pd = k > 0 ? pz : pw;
        int sgn = k > 0 ? 1 : -1;
        v = mk(0.0, 0.0);
        double bin = 1.0;                              // C(n, m) at n = m
        for (int n = m; n <= Pp; ++n) {
            cfma(v, pd[n - m] * bin, src[Pp + sgn * n]);
            bin = bin * (double)(n + 1) * c_l2d_rcp[n + 1 - m];
        }
        v = v * ldexp(1.0, -m);                        // (w_c / w_p)^m
    }
    cplx* o = local + tv.eoff[c];
    o[t] = o[t] + v;
}

// Multipole of box a (level la) at a point: M0 log r + sum A_n z^-n + B_n w^-n
// (Horner in 1/z, 1/w), times 2.
__device__ inline cplx m2p_value(cplx z, cplx w, double sc, int P, const cplx* M)
{
    cplx iz = cinv(z * sc), iw = cinv(w * sc);
    cplx sz = mk(0.0, 0.0), sw = mk(0.0, 0.0);
    for (int n = P; n >= 1; --n) {
        sz = (sz + M[P + n]) * iz;
        sw = (sw + M[P - n]) * iw;
    }
    return (M[P] * log_r(z, w) + sz + sw) * 2.0;
}

// M2P by List-3 entries: entry e = (leaf owner[e], box l3idx[e]) evaluates the
// box's multipole at the leaf's points into part[poff[e] + i - pbeg].
__global__ __launch_bounds__(64) void k_l2d_m2p_part(const int* __restrict__ owner,
                                                     const int64_t* __restrict__ poff, TreeView tv,
                                                     PointsView pv, const cplx* __restrict__ mpole,
                                                     cplx* __restrict__ part)
{
    int e = blockIdx.x;
    int b = owner[e], a = tv.l3idx[e];
    int la = tv.level[a];
    int Pa = tv.P[la];
    double sc = tv.rs[la];
    cplx ca1, ca2;
    centre2(tv, a, ca1, ca2);
    const cplx* M = mpole + tv.eoff[a];
    cplx* o = part + poff[e] - tv.pbeg[b];
    for (int i = tv.pbeg[b] + threadIdx.x; i < tv.pend[b]; i += blockDim.x) {
        cplx z, w;
        point_zw(pv, i, ca1, ca2, 1.0, z, w);
        o[i] = m2p_value(z, w, sc, Pa, M);
    }
}

// L2P plus the leaf's List-3 parts in list order: ufar = 2 (L0 + sum C_n z^n
// + D_n w^n) + parts.  Leaves coarser than the top level have no expansion.
__global__ __launch_bounds__(64) void k_l2d_l2p(const int* __restrict__ leaves, int top, TreeView tv,
                                                PointsView pv, const cplx* __restrict__ local,
                                                const int64_t* __restrict__ poff3, const cplx* __restrict__ part,
                                                cplx* __restrict__ ufar)
{
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    int t = threadIdx.x;
    bool has = l >= top;
    int P = has ? tv.P[l] : 0;
    double sc = tv.rs[l];
    cplx c1, c2;
    centre2(tv, b, c1, c2);
    const cplx* L = has ? local + tv.eoff[b] : nullptr;
    for (int i = p0 + t; i < p1; i += blockDim.x) {
        cplx u = mk(0.0, 0.0);
        if (has) {
            cplx z, w;
            point_zw(pv, i, c1, c2, sc, z, w);
            cplx sz = mk(0.0, 0.0), sw = mk(0.0, 0.0);
            for (int n = P; n >= 1; --n) {
                sz = (sz + L[P + n]) * z;
                sw = (sw + L[P - n]) * w;
            }
            u = (L[P] + sz + sw) * 2.0;
        }
        for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) u += part[poff3[e] + i - p0];
        ufar[i] = u;
    }
}

}  // namespace

hipError_t l2d_init_tables(int device)
{
    (void)device;
    double rcp[kL2DRcp];
    rcp[0] = 0.0;
    for (int m = 1; m < kL2DRcp; ++m) rcp[m] = 1.0 / m;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_l2d_rcp), rcp, sizeof(rcp));
}

hipError_t l2d_p2m(const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv, cplx* mpole,
                   hipStream_t st)
{
    if (nleaf > 0) k_l2d_p2x<false><<<nleaf, 64, 0, st>>>(leaves, tv, pv, mpole);
    return hipGetLastError();
}

hipError_t l2d_m2m(const int* boxes, int nb, const TreeView& tv, cplx* mpole, hipStream_t st)
{
    if (nb > 0) k_l2d_m2m<<<nb, 128, 0, st>>>(boxes, tv, mpole);
    return hipGetLastError();
}

hipError_t l2d_m2l(const int* boxes, int nb, const TreeView& tv, const cplx* mpole, cplx* local, hipStream_t st)
{
    if (nb > 0) k_l2d_m2l<<<nb, 128, 0, st>>>(boxes, nb, tv, mpole, local);
    return hipGetLastError();
}

hipError_t l2d_p2l(const int* boxes, int nb, const TreeView& tv, const PointsView& pv, cplx* local,
                   hipStream_t st)
{
    if (nb > 0) k_l2d_p2x<true><<<nb, 64, 0, st>>>(boxes, tv, pv, local);
    return hipGetLastError();
}

hipError_t l2d_l2l(const int* boxes, int nb, const TreeView& tv, cplx* local, hipStream_t st)
{
    if (nb > 0) k_l2d_l2l<<<nb, 128, 0, st>>>(boxes, tv, local);
    return hipGetLastError();
}

hipError_t l2d_leaf_far(const int* leaves, int nleaf, const M2PParts& m2p, int top, const TreeView& tv,
                        const PointsView& pv, const cplx* mpole, const cplx* local, cplx* ufar, hipStream_t st)
{
    if (m2p.n > 0) {
        k_l2d_m2p_part<<<m2p.n, 64, 0, st>>>(m2p.owner, m2p.poff, tv, pv, mpole, m2p.part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nleaf > 0) k_l2d_l2p<<<nleaf, 64, 0, st>>>(leaves, top, tv, pv, local, m2p.poff, m2p.part, ufar);
    return hipGetLastError();
}

}  // namespace cfmm
