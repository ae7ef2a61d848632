// 3D near field (P2P, step 3 of Sec. 6.4) for the Laplace kernel 1/(4 pi r)
// and the Helmholtz kernel e^{i kappa r}/(4 pi r), by List-1 entries.
//
// G(x, y) = G(y, x) (the squared complex distance is the same either way), so
// every pair of near leaves is evaluated once for both directions.  A work
// item is an entry e = (b, a) with a < b (neighbour item) or a = b (diagonal
// item).  Each entry e owns the partial sums C[coff[e] + (i - pbeg[b])] of
// b's targets due to a's sources; a neighbour item writes C[e] (rows) and
// C[partner e] (columns), a diagonal item writes C[e].  A final pass adds, per
// target, its entries' partials in list order, so results are reproducible.
//
// Inside an item a wavefront holds targets in its lanes and a tile of up to
// 64 sources in LDS, and the source's column sum travels with the source,
// one lane down per step, while the row sums stay in the lanes.  Neighbour
// items hold two rows of 64 targets per lane and travel cyclically: at step
// s lane l pairs with source (s + l) mod C of a tile of C, so every lane is
// busy at every step (cyc_pass).  Diagonal items take the leaf's tiles of 64
// in pairs: a tile against itself by rotation with period L, steps 1..L/2
// only (at step L/2 just lanes l < L/2 when L is even), which covers each
// unordered pair once; two distinct tiles by cyclic travel.
//
// Precision: FP64, or MIXED (differences formed in FP64 and cast to FP32, the
// kernel in FP32, each tile's sums accumulated in FP32 with Kahan compensation
// and the compensated sum formed and added in FP64).  In MIXED mode a
// Helmholtz item whose near field can reach kappa r > 8 (flag from the plan)
// forms r and the phase in FP64, reduced mod 2 pi before the FP32 sincos.
#include "common.hpp"
#include "kernels.hpp"

namespace cfmm {

namespace {

struct Tile {
    double xr[3][64], xi[3][64], sr[64], si[64];
};

template <int KIND, int PREC>
struct Kernel;

// 1/sqrt(x) for positive normal x: the hardware estimate y0 (relative error
// below 2^-24 on gfx950) refined by one third-order step of the binomial
// series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3), e = 1 - x y0^2:
// y = y0 (1 + e (1/2 + 3e/8)).  The truncation is below 2^-70; rounding
// leaves about 1.2 ulp, as two Newton steps do, in five operations instead of
// eight.
__device__ inline double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-(x * y), y, 1.0);
    return fma(y, e * fma(0.375, e, 0.5), y);
}

// 1/r (principal r): (t - i Im s/(2t)) / |s|, t = sqrt((|s| + Re s)/2).
// The FP32 forms use the hardware reciprocal square root directly.
// With u = 1/|s| from rsq_nr, h = |s| + Re s = |s|^2 u + Re s and
// v = 1/sqrt(h): t = sqrt(1/2) h v and 1/(2t) = sqrt(1/2) v, so
// 1/r = sqrt(1/2) (h u v, -Im s u v); no division.  The Laplace kernels
// return 1/r without the factor sqrt(1/2), which the final pass applies once
// per target.
// s = (x - y).(x - y) from the FP64 differences dr + i di, started from the
// first product (an accumulation started from zero costs a register copy per
// evaluation: fma(a, b, +0) is not a * b when the product is -0).
__device__ inline void sdist(const double* dr, const double* di, double& sr, double& si)
{
    double a = fma(dr[0], dr[0], -(di[0] * di[0]));
    a = fma(dr[1], dr[1], a);
    a = fma(-di[1], di[1], a);
    a = fma(dr[2], dr[2], a);
    sr = fma(-di[2], di[2], a);
    double b = dr[0] * di[0];
    b = fma(dr[1], di[1], b);
    si = 2.0 * fma(dr[2], di[2], b);
}
__device__ inline void sdistf(const double* dr, const double* di, float& sr, float& si)
{
    float x0 = (float)dr[0], x1 = (float)dr[1], x2 = (float)dr[2];
    float y0 = (float)di[0], y1 = (float)di[1], y2 = (float)di[2];
    float a = fmaf(x0, x0, -(y0 * y0));
    a = fmaf(x1, x1, a);
    a = fmaf(-y1, y1, a);
    a = fmaf(x2, x2, a);
    sr = fmaf(-y2, y2, a);
    float b = x0 * y0;
    b = fmaf(x1, y1, b);
    si = 2.0f * fmaf(x2, y2, b);
}

// FP64 kernels: G = false leaves out the test for s = 0 (coincident points,
// which contribute zero); pairs of distinct leaves never have s = 0 (points
// with equal real parts share a leaf, and the plan's geometry check rejects
// s = 0 between leaves).
template <>
struct Kernel<0, 0> {
    template <bool G = true>
    __device__ static void eval(const double* dr, const double* di, double, double& gr, double& gi)
    {
        double sr, si;
        sdist(dr, di, sr, si);
        if (G && sr == 0.0 && si == 0.0) { gr = gi = 0.0; return; }
        double q = sr * sr + si * si;
        double u = rsq_nr(q);
        double h = fma(q, u, sr);
        double uv = u * rsq_nr(h);
        gr = h * uv;
        gi = -si * uv;
    }
};
template <>
struct Kernel<0, 1> {
    __device__ static void eval(const double* dr, const double* di, double, float& gr, float& gi)
    {
        float sr, si;
        sdistf(dr, di, sr, si);
        if (sr == 0.0f && si == 0.0f) { gr = gi = 0.0f; return; }
        float q = sr * sr + si * si;
        float u = __builtin_amdgcn_rsqf(q);
        float h = fmaf(q, u, sr);
        float uv = u * __builtin_amdgcn_rsqf(h);
        gr = h * uv;
        gi = -si * uv;
    }
};
// e^{i kappa r}/r = e^{-kappa Im r}(cos + i sin)(kappa Re r) conj(r)/|s|, with
// r = (t, Im s/(2t)) and 1/|s|, 1/t from rsq_nr as for 1/r.
template <>
struct Kernel<1, 0> {
    template <bool G = true>
    __device__ static void eval(const double* dr, const double* di, double kappa, double& gr, double& gi)
    {
        double sr, si;
        sdist(dr, di, sr, si);
        if (G && sr == 0.0 && si == 0.0) { gr = gi = 0.0; return; }
        double q = sr * sr + si * si;
        double u = rsq_nr(q);
        double h = 0.5 * (q * u + sr);
        double v = rsq_nr(h);
        double rr = h * v, ri = 0.5 * si * v;
        // near-field phases stay far below 2^20: the expansion-length limit
        // bounds a leaf's width in wavelengths
        double sn, cs;
        sincos_cw(kappa * rr, &sn, &cs);
        double ex = exp_cw(-kappa * ri) * u;
        gr = (cs * rr + sn * ri) * ex;
        gi = (sn * rr - cs * ri) * ex;
    }
};
template <>
struct Kernel<1, 1> {
    __device__ static void eval(const double* dr, const double* di, double kappa, float& gr, float& gi)
    {
        float sr, si;
        sdistf(dr, di, sr, si);
        if (sr == 0.0f && si == 0.0f) { gr = gi = 0.0f; return; }
        float kf = (float)kappa;
        float q = sr * sr + si * si;
        float u = __builtin_amdgcn_rsqf(q);
        float h = 0.5f * (q * u + sr);
        float v = __builtin_amdgcn_rsqf(h);
        float rr = h * v, ri = 0.5f * si * v;
        float sn, cs;
        sincosf(kf * rr, &sn, &cs);
        float ex = expf(-kf * ri) * u;
        gr = (cs * rr + sn * ri) * ex;
        gi = (sn * rr - cs * ri) * ex;
    }
};
// mixed, wide phase: r and kappa Re r in FP64, the rest in FP32
template <>
struct Kernel<1, 2> {
    __device__ static void eval(const double* dr, const double* di, double kappa, float& gr, float& gi)
    {
        double sr, si;
        sdist(dr, di, sr, si);
        if (sr == 0.0 && si == 0.0) { gr = gi = 0.0f; return; }
        double q = sr * sr + si * si;
        double u = rsq_nr(q);
        double h = 0.5 * (q * u + sr);
        double v = rsq_nr(h);
        double tt = h * v;
        double ph = kappa * tt;
        ph -= (2.0 * kPi) * rint(ph * (1.0 / (2.0 * kPi)));
        float rr = (float)tt, ri = (float)(0.5 * si * v);
        float sn, cs;
        sincosf((float)ph, &sn, &cs);
        float ex = expf(-(float)kappa * ri) * (float)u;
        gr = (cs * rr + sn * ri) * ex;
        gi = (sn * rr - cs * ri) * ex;
    }
};

template <int PREC>
struct Acc {
    typedef double T;
};
template <>
struct Acc<1> {
    typedef float T;
};
template <>
struct Acc<2> {
    typedef float T;
};

// A tile's running sum.  FP64: plain.  FP32: compensated (Kahan): c carries
// the rounding error of the last addition, which the next term corrects, so
// the error of a sum of up to 64 terms stays near one FP32 rounding of the
// total instead of growing with the term count; val() forms s - c in FP64.
template <class T>
struct Sum {
    T s = 0;
    __device__ inline void add(T x) { s += x; }
    // s + a b + c d as two fused multiply-adds
    __device__ inline void add2(T a, T b, T c, T d) { s = fma(a, b, fma(c, d, s)); }
    __device__ inline double val() const { return (double)s; }
    __device__ inline void shfl(int src) { s = __shfl(s, src, 64); }
};
template <>
struct Sum<float> {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x)
    {
        float y = x - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ inline void add2(float a, float b, float c2, float d) { add(fmaf(a, b, c2 * d)); }
    __device__ inline double val() const { return (double)s - (double)c; }
    __device__ inline void shfl(int src)
    {
        s = __shfl(s, src, 64);
        c = __shfl(c, src, 64);
    }
};

__device__ inline void load_tile(Tile& sh, const PointsView& pv, int j0, int cnt, int t)
{
    int64_t n = pv.n;
    if (t < cnt) {
        int j = j0 + t;
        for (int d = 0; d < 3; ++d) {
            sh.xr[d][t] = pv.xre[d * n + j];
            sh.xi[d][t] = pv.xim[d * n + j];
        }
        sh.sr[t] = pv.sre[j];
        sh.si[t] = pv.sim[j];
    }
}

// One tile pair by rotation with period L = max(R, C) (R targets in lanes
// 0..R-1, C sources in the tile): at step s lane l < L pairs its target with
// source (l + s) mod L and hands its travelling column sum to lane l - 1
// (mod L), so after L steps lane l holds the column sum of source l.  A tile
// against itself (R = C = L) takes steps 1..L/2, at step L/2 (L even) only
// lanes l < L/2, which covers each unordered pair once; a last shuffle
// returns each column sum to its home lane.  Row sums (ar, ai) accumulate in
// the lane.
template <int KIND, int PREC>
__device__ inline void tile_pair(const Tile& sh, int R, int C, bool self, const double* x, const double* y,
                                 double wr, double wi, double kappa, double& ar, double& ai,
                                 double& cr_out, double& ci_out)
{
    typedef typename Acc<PREC>::T T;
    int t = threadIdx.x;
    int L = max(R, C);
    int nxt = t < L ? (t + 1 == L ? 0 : t + 1) : t;
    int s0 = self ? 1 : 0, s1 = self ? L / 2 : L - 1;
    Sum<T> rr, ri, cr, ci;
    T fwr = (T)wr, fwi = (T)wi;
    int q = t + s0;
    if (q >= L) q -= L;
    for (int step = s0; step <= s1; ++step) {
        bool on = t < R && q < C && (!self || 2 * step < L || 2 * t < L);
        if (on) {
            double dr[3], di[3];
            for (int d = 0; d < 3; ++d) {
                dr[d] = x[d] - sh.xr[d][q];
                di[d] = y[d] - sh.xi[d][q];
            }
            T gr, gi;
            Kernel<KIND, PREC>::eval(dr, di, kappa, gr, gi);
            T sr = (T)sh.sr[q], si = (T)sh.si[q];
            rr.add2(gr, sr, -gi, si);
            ri.add2(gr, si, gi, sr);
            cr.add2(gr, fwr, -gi, fwi);
            ci.add2(gr, fwi, gi, fwr);
        }
        cr.shfl(nxt);
        ci.shfl(nxt);
        if (++q >= L) q -= L;
    }
    if (self) {
        // after L/2 hand-offs lane u holds the column sum of point (u + L/2 + 1) mod L
        int src = t;
        if (t < L) {
            src = t - L / 2 - 1;
            while (src < 0) src += L;
        }
        cr.shfl(src);
        ci.shfl(src);
    }
    ar += rr.val();
    ai += ri.val();
    cr_out = cr.val();
    ci_out = ci.val();
}

// Cyclic travel of a tile of C <= 64 points (Y, in LDS) past two rows of
// points held in the lanes (X: lane l holds rows 0 and 1, R0 >= R1 valid):
// at step s lane l pairs with tile point (s + l) mod C, so every lane is busy
// at every step whatever C and the rows' fill.  The lane sums (each X point
// against all of Y) stay in the lane; the sum of each Y point travels one
// lane down per step, with the point it belongs to.  The value leaving lane 0
// at step s is complete for Y point s and goes to flush[s]; lane 0 restarts
// from zero, which reaches lane 63.  After C steps lane l (< 63) holds a last
// segment of Y point l mod C, put in seg[l]; Y point j's sum is flush[j] plus
// seg[j], seg[j + C], ... in that order.  When C divides 64 the value leaving
// lane 0 reaches lane 63, which pairs with the same Y point at the next step,
// so nothing is flushed (flush[j] counts as zero).
// ZG keeps the test for s = 0 in the FP64 kernels (tiles of one leaf, which
// may hold coincident points).
template <int KIND, int PREC, bool FULL, bool ZG = false>
__device__ inline void cyc_pass(const Tile& ty, int C, int R0, int R1, const double (&x)[2][3],
                                const double (&y)[2][3], const double (&wr)[2], const double (&wi)[2],
                                double kappa, double (&ar)[2], double (&ai)[2], double2* flush, double2* seg)
{
    typedef typename Acc<PREC>::T T;
    int t = threadIdx.x;
    int nxt = (t + 1) & 63;
    Sum<T> rr[2], ri[2], cr, ci;
    T fwr[2] = {(T)wr[0], (T)wr[1]}, fwi[2] = {(T)wi[0], (T)wi[1]};
    int q = t % C;
    bool wrap = (64 % C) == 0;
    for (int step = 0; step < C; ++step) {
        double sxr[3], sxi[3];
        for (int d = 0; d < 3; ++d) {
            sxr[d] = ty.xr[d][q];
            sxi[d] = ty.xi[d][q];
        }
        T sr = (T)ty.sr[q], si = (T)ty.si[q];
        if constexpr (FULL) {
            // every lane holds two targets: the two evaluations run without
            // a branch, so their dependency chains interleave
            T gr[2], gi[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                double dr[3], di[3];
                for (int d = 0; d < 3; ++d) {
                    dr[d] = x[r][d] - sxr[d];
                    di[d] = y[r][d] - sxi[d];
                }
                if constexpr (PREC == 0) Kernel<KIND, PREC>::template eval<ZG>(dr, di, kappa, gr[r], gi[r]);
                else Kernel<KIND, PREC>::eval(dr, di, kappa, gr[r], gi[r]);
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                rr[r].add2(gr[r], sr, -gi[r], si);
                ri[r].add2(gr[r], si, gi[r], sr);
                cr.add2(gr[r], fwr[r], -gi[r], fwi[r]);
                ci.add2(gr[r], fwi[r], gi[r], fwr[r]);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (t < (r ? R1 : R0)) {
                    double dr[3], di[3];
                    for (int d = 0; d < 3; ++d) {
                        dr[d] = x[r][d] - sxr[d];
                        di[d] = y[r][d] - sxi[d];
                    }
                    T gr, gi;
                    // distinct leaves: s != 0, so FP64 skips the zero test
                    if constexpr (PREC == 0) Kernel<KIND, PREC>::template eval<ZG>(dr, di, kappa, gr, gi);
                    else Kernel<KIND, PREC>::eval(dr, di, kappa, gr, gi);
                    rr[r].add2(gr, sr, -gi, si);
                    ri[r].add2(gr, si, gi, sr);
                    cr.add2(gr, fwr[r], -gi, fwi[r]);
                    ci.add2(gr, fwi[r], gi, fwr[r]);
                }
            }
        }
        if (!wrap && t == 0) {
            flush[step] = make_double2(cr.val(), ci.val());
            cr = Sum<T>();
            ci = Sum<T>();
        }
        cr.shfl(nxt);
        ci.shfl(nxt);
        if (++q == C) q = 0;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        ar[r] += rr[r].val();
        ai[r] += ri[r].val();
    }
    seg[t] = make_double2(cr.val(), ci.val());
}

// Y point j's total after cyc_pass (the caller synchronises first).
__device__ inline cplx cyc_total(const double2* flush, const double2* seg, int C, int j)
{
    cplx v = (64 % C) == 0 ? mk(0.0, 0.0) : mk(flush[j].x, flush[j].y);
    for (int l = j; l < 64; l += C) v += mk(seg[l].x, seg[l].y);
    return v;
}

// Neighbour items (a < b): rows into C[e], columns into C[partner e].  b's
// targets go through the lanes in passes of 128 (two rows of 64) against a's
// sources in tiles of 64 and a last tile of the rest (cyclic travel).  A remainder of r <= 64
// targets after the full passes runs with the roles swapped when that takes
// fewer steps (ceil(na / 128) r < na): a's points in the lanes, 128 per pass,
// the r targets travelling; so a leaf of 132 points costs 128 + 4 steps per
// 64 lanes instead of two half-filled passes.
template <int KIND, int PREC>
__global__ __launch_bounds__(64) void k_near3_pair(const int* __restrict__ items, Near3Map mp, TreeView tv,
                                                   PointsView pv, double kappa)
{
    __shared__ Tile sh;
    __shared__ double2 flush[64], seg[64];
    int e = items[blockIdx.x];
    int b = mp.row_of[e], a = tv.l1idx[e], ep = mp.partner[e];
    int64_t n = pv.n;
    int t = threadIdx.x;
    int pb0 = tv.pbeg[b], pb1 = tv.pend[b], pa0 = tv.pbeg[a], pa1 = tv.pend[a];
    cplx* Crow = mp.C + mp.coff[e];
    cplx* Ccol = mp.C + mp.coff[ep];
    int nt = pb1 - pb0, na = pa1 - pa0;
    const int Cs = 64;                                    // source tiles of 64, the last one shorter
    int nfull = nt / 128, rem = nt - 128 * nfull;
    bool swap = rem > 0 && rem <= 64 && ((na + 127) / 128) * rem < na;
    int npass = nfull + (rem > 0 && !swap ? 1 : 0);
    // lane rows of points p0 + t and p0 + 64 + t (counts R0, R1)
    auto load_rows = [&](int p0, int R0, int R1, double (&x)[2][3], double (&y)[2][3], double (&wr)[2],
                         double (&wi)[2]) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            int i = p0 + 64 * r + t;
            bool ok = t < (r ? R1 : R0);
            for (int d = 0; d < 3; ++d) {
                x[r][d] = ok ? pv.xre[d * n + i] : 0.0;
                y[r][d] = ok ? pv.xim[d * n + i] : 0.0;
            }
            wr[r] = ok ? pv.sre[i] : 0.0;
            wi[r] = ok ? pv.sim[i] : 0.0;
        }
    };
    for (int ps = 0; ps < npass; ++ps) {
        int left = nt - 128 * ps;
        int R0 = min(64, left), R1 = max(0, min(64, left - 64));
        double x[2][3], y[2][3], wr[2], wi[2], ar[2] = {0.0, 0.0}, ai[2] = {0.0, 0.0};
        load_rows(pb0 + 128 * ps, R0, R1, x, y, wr, wi);
        for (int j0 = pa0; j0 < pa1; j0 += Cs) {
            int cnt = min(Cs, pa1 - j0);
            __syncthreads();
            load_tile(sh, pv, j0, cnt, t);
            __syncthreads();
            if (R1 == 64) cyc_pass<KIND, PREC, true>(sh, cnt, R0, R1, x, y, wr, wi, kappa, ar, ai, flush, seg);
            else cyc_pass<KIND, PREC, false>(sh, cnt, R0, R1, x, y, wr, wi, kappa, ar, ai, flush, seg);
            __syncthreads();
            if (t < cnt) {
                cplx v = cyc_total(flush, seg, cnt, t);
                cplx* cc = Ccol + (j0 - pa0) + t;
                *cc = ps == 0 ? v : *cc + v;
            }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if (t < (r ? R1 : R0)) Crow[128 * ps + 64 * r + t] = mk(ar[r], ai[r]);
    }
    if (swap) {
        int i0 = 128 * nfull;
        __syncthreads();
        load_tile(sh, pv, pb0 + i0, rem, t);
        for (int p0 = 0; p0 < na; p0 += 128) {
            int left = na - p0;
            int R0 = min(64, left), R1 = max(0, min(64, left - 64));
            double x[2][3], y[2][3], wr[2], wi[2], ar[2] = {0.0, 0.0}, ai[2] = {0.0, 0.0};
            load_rows(pa0 + p0, R0, R1, x, y, wr, wi);
            __syncthreads();
            if (R1 == 64) cyc_pass<KIND, PREC, true>(sh, rem, R0, R1, x, y, wr, wi, kappa, ar, ai, flush, seg);
            else cyc_pass<KIND, PREC, false>(sh, rem, R0, R1, x, y, wr, wi, kappa, ar, ai, flush, seg);
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (t < (r ? R1 : R0)) {
                    cplx* cc = Ccol + p0 + 64 * r + t;
                    *cc = npass == 0 ? mk(ar[r], ai[r]) : *cc + mk(ar[r], ai[r]);
                }
            }
            __syncthreads();
            if (t < rem) {
                cplx v = cyc_total(flush, seg, rem, t);
                cplx* cr = Crow + i0 + t;
                *cr = p0 == 0 ? v : *cr + v;
            }
        }
    }
}

// Diagonal items (a = b): tile pairs (T, S) with T <= S of the leaf's tiles
// of 64; both rows and columns land in C[e].  A tile against itself takes the
// half rotation, a pair of distinct tiles the cyclic travel (so a short last
// tile costs as many steps as it has points).  The block first clears its
// region.
template <int KIND, int PREC>
__global__ __launch_bounds__(64) void k_near3_diag(const int* __restrict__ items, Near3Map mp, TreeView tv,
                                                   PointsView pv, double kappa)
{
    __shared__ Tile sh;
    __shared__ double2 flush[64], seg[64];
    int e = items[blockIdx.x];
    int b = mp.row_of[e];
    int64_t n = pv.n;
    int t = threadIdx.x;
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    cplx* Cb = mp.C + mp.coff[e];
    for (int i = t; i < p1 - p0; i += 64) Cb[i] = mk(0.0, 0.0);
    for (int i0 = p0; i0 < p1; i0 += 64) {
        int i = i0 + t;
        bool tok = i < p1;
        double x[3] = {0, 0, 0}, y[3] = {0, 0, 0}, wr = 0, wi = 0;
        if (tok) {
            for (int d = 0; d < 3; ++d) { x[d] = pv.xre[d * n + i]; y[d] = pv.xim[d * n + i]; }
            wr = pv.sre[i];
            wi = pv.sim[i];
        }
        double ar = 0.0, ai = 0.0;
        for (int j0 = i0; j0 < p1; j0 += 64) {
            int cnt = min(64, p1 - j0);
            __syncthreads();
            load_tile(sh, pv, j0, cnt, t);
            __syncthreads();
            if (j0 == i0) {
                double cr, ci;
                tile_pair<KIND, PREC>(sh, min(64, p1 - i0), cnt, true, x, y, wr, wi, kappa, ar, ai, cr, ci);
                ar += cr;   // the column sums of the same tile are this lane's own point
                ai += ci;
            } else {
                double xx[2][3] = {{x[0], x[1], x[2]}, {0.0, 0.0, 0.0}};
                double yy[2][3] = {{y[0], y[1], y[2]}, {0.0, 0.0, 0.0}};
                double wwr[2] = {wr, 0.0}, wwi[2] = {wi, 0.0}, aar[2] = {ar, 0.0}, aai[2] = {ai, 0.0};
                cyc_pass<KIND, PREC, false, true>(sh, cnt, min(64, p1 - i0), 0, xx, yy, wwr, wwi, kappa, aar, aai,
                                                  flush, seg);
                ar = aar[0];
                ai = aai[0];
                __syncthreads();
                if (t < cnt) {
                    // written by this wavefront only; earlier tiles' rows never touch it
                    cplx* cc = Cb + (j0 - p0) + t;
                    *cc = *cc + cyc_total(flush, seg, cnt, t);
                }
            }
        }
        if (tok) Cb[i - p0] = Cb[i - p0] + mk(ar, ai);
    }
}

// u[perm[i] - obase] = (1/4pi)(near + far) at the targets, far = ufar
// (Laplace) or i kappa ufar (Helmholtz, whose expansions carry the factor
// i kappa / 4pi).
template <int KIND>
__global__ __launch_bounds__(64) void k_near3_final(const int* __restrict__ leaves, Near3Map mp, TreeView tv,
                                                    double kappa, const cplx* __restrict__ ufar, IoMap io,
                                                    double* __restrict__ out)
{
    int b = leaves[blockIdx.x];
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    int e0 = tv.l1off[b], e1 = tv.l1off[b + 1];
    double k = 1.0 / (4.0 * kPi);
    for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
        int64_t p = (int64_t)io.perm[i] - io.obase;
        if (p < 0) continue;            // a source that is not a target
        cplx u = mk(0.0, 0.0);
        for (int e = e0; e < e1; ++e) u += mp.C[mp.coff[e] + (i - p0)];
        if (KIND == 0) u = sqrt(0.5) * u;   // the Laplace kernels' omitted factor
        cplx f = ufar[i];
        if (KIND == 1) f = mk(-kappa * f.im, kappa * f.re);
        double vr = k * (u.re + f.re), vi = k * (u.im + f.im);
        out[2 * p] = vr;
        out[2 * p + 1] = vi;
        if (!isfinite(vr) || !isfinite(vi)) atomicOr(io.nonfinite, 1);
    }
}

template <int KIND, int PREC>
void launch_items(const Near3Work& w, int which, const Near3Map& mp, const TreeView& tv, const PointsView& pv,
                  double kappa, hipStream_t st)
{
    const int* it = w.items[which];
    int nit = w.nitems[which];
    if (nit <= 0) return;
    if (which == 0 || which == 2) k_near3_pair<KIND, PREC><<<nit, 64, 0, st>>>(it, mp, tv, pv, kappa);
    else k_near3_diag<KIND, PREC><<<nit, 64, 0, st>>>(it, mp, tv, pv, kappa);
}

}  // namespace

// items[0]: neighbour items, items[1]: diagonal items; in MIXED Helmholtz,
// items[2], items[3]: the same for wide-phase pairs.
hipError_t near3_p2p(const Near3Work& w, int kernel, int mixed, const int* leaves, int nleaf, const TreeView& tv,
                     const PointsView& pv, double kappa, const cplx* ufar, const IoMap& io, double* out,
                     hipStream_t st)
{
    Near3Map mp{w.row_of, w.partner, w.coff, w.C};
    if (kernel == 0) {
        if (mixed) { launch_items<0, 1>(w, 0, mp, tv, pv, kappa, st); launch_items<0, 1>(w, 1, mp, tv, pv, kappa, st); }
        else { launch_items<0, 0>(w, 0, mp, tv, pv, kappa, st); launch_items<0, 0>(w, 1, mp, tv, pv, kappa, st); }
        if (nleaf > 0) k_near3_final<0><<<nleaf, 64, 0, st>>>(leaves, mp, tv, kappa, ufar, io, out);
    } else {
        if (mixed) {
            launch_items<1, 1>(w, 0, mp, tv, pv, kappa, st);
            launch_items<1, 1>(w, 1, mp, tv, pv, kappa, st);
            launch_items<1, 2>(w, 2, mp, tv, pv, kappa, st);
            launch_items<1, 2>(w, 3, mp, tv, pv, kappa, st);
        } else {
            launch_items<1, 0>(w, 0, mp, tv, pv, kappa, st);
            launch_items<1, 0>(w, 1, mp, tv, pv, kappa, st);
        }
        if (nleaf > 0) k_near3_final<1><<<nleaf, 64, 0, st>>>(leaves, mp, tv, kappa, ufar, io, out);
    }
    return hipGetLastError();
}

}  // namespace cfmm
