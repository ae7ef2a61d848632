// 3D Laplace complex-coordinate FMM kernels (Sec. 5.2 and the multilevel steps
// of Sec. 6.4).  The angular functions are solid harmonics evaluated by their
// Cartesian recurrences directly at complex points, so no complex angle is ever
// formed.  With w+ = x + iy, w- = x - iy, r2 = x^2 + y^2 + z^2 and m >= 0:
//
//   R_m^m = w+^m / (2^m m!),   R_{m+1}^m = z R_m^m,
//   R_n^m = ((2n-1) z R_{n-1}^m - r2 R_{n-2}^m) / ((n+m)(n-m))         (regular)
//   I_0^0 = 1/rho,  I_m^m = (2m-1) w+ I_{m-1}^{m-1} / r2,  I_{m+1}^m = (2m+1) z I_m^m / r2,
//   I_n^m = ((2n-1) z I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m) / r2        (irregular)
//
// and R_n^{-m}, I_n^{-m} the same with w- and a factor (-1)^m; rho is the
// principal root of r2.  These are rho^n P_n^m e^{im phi}/(n+m)! and
// (n-m)! P_n^m e^{im phi}/rho^{n+1} continued analytically (Sec. 3.1, 3.2), and
//
//   1/|X - Y| = sum_{n,m} (-1)^m R_n^{-m}(Y) I_n^m(X)                 (|Y| < |X|)
//   R_n^m(X + Y) = sum_{j,k} R_j^k(X) R_{n-j}^{m-k}(Y).
//
// Expansions about a complexified centre c, coordinates scaled by the level's
// box width w (Mhat = M / w^n, Lhat = L w^(n+1)):
//   P2M  M_n^m = sum_j sigma_j (-1)^m R_n^{-m}(Y_j / w)       u = (1/w) sum M_n^m I_n^m(X / w)
//   P2L  L_n^m = sum_j sigma_j (-1)^m I_n^{-m}(Y_j / w)       u = (1/w) sum L_n^m R_n^m(X / w)
//   M2M  M'_n^m = sum_{j<=n,k} M_j^k 2^-j (-1)^q R_{n-j}^{-q}(d / w_p),   q = m - k, d = c_child - c_parent
//   M2L  L_j^k = (-1)^{j+k} sum_{n,m} M_n^m I_{j+n}^{m-k}(D / w),         D = c_target - c_source
//   L2L  L'_j^k = 2^-(j+1) sum_{n>=j,m} L_n^m R_{n-j}^{m-k}(d / w_p),     d = c_child - c_parent
// Coefficient (n, m) is stored at n^2 + n + m.  G = 1/(4 pi r) is applied at the end.
#include "common.hpp"
#include "kernels.hpp"
#include "l3d_layout.hpp"

namespace cfmm {

__device__ inline int nm(int n, int m) { return n * n + n + m; }

struct Vec3 {
    cplx x, y, z;
};

__device__ inline Vec3 point_rel(const PointsView& pv, int i, const cplx* c, double s)
{
    int64_t n = pv.n;
    Vec3 v;
    v.x = mk((pv.xre[i] - c[0].re) * s, (pv.xim[i] - c[0].im) * s);
    v.y = mk((pv.xre[n + i] - c[1].re) * s, (pv.xim[n + i] - c[1].im) * s);
    v.z = mk((pv.xre[2 * n + i] - c[2].re) * s, (pv.xim[2 * n + i] - c[2].im) * s);
    return v;
}

__device__ inline void box_centre(const TreeView& tv, int b, cplx* c)
{
    int nb = tv.nbox;
    for (int d = 0; d < 3; ++d) c[d] = mk(tv.cre[d * nb + b], tv.cim[d * nb + b]);
}

__device__ inline cplx wplus(const Vec3& v) { return mk(v.x.re - v.y.im, v.x.im + v.y.re); }
__device__ inline cplx wminus(const Vec3& v) { return mk(v.x.re + v.y.im, v.x.im - v.y.re); }
__device__ inline cplx dot3(const Vec3& v) { return v.x * v.x + v.y * v.y + v.z * v.z; }

// Regular column m (any sign), n = |m| .. P, times an extra sign when `flip`:
// calls f(n, value).  Diagonal by |m| steps of the product recurrence.
template <class F>
__device__ inline void col_R(const Vec3& v, int m, int P, bool flip, F f)
{
    int am = m < 0 ? -m : m;
    cplx w = m < 0 ? wminus(v) : wplus(v);
    cplx r2 = dot3(v);
    cplx d = mk(1.0, 0.0);
    for (int k = 1; k <= am; ++k) d = d * w * (0.5 / k);
    bool neg = (m < 0 && (am & 1)) != flip;
    if (neg) d = -d;
    f(am, d);
    if (am + 1 > P) return;
    cplx a = d, b = v.z * d;
    f(am + 1, b);
    for (int n = am + 2; n <= P; ++n) {
        cplx c = ((2.0 * n - 1.0) * (v.z * b) - r2 * a) * (1.0 / ((double)(n + am) * (double)(n - am)));
        f(n, c);
        a = b;
        b = c;
    }
}

// Irregular column m, n = |m| .. P (principal rho).
template <class F>
__device__ inline void col_I(const Vec3& v, int m, int P, bool flip, F f)
{
    int am = m < 0 ? -m : m;
    cplx w = m < 0 ? wminus(v) : wplus(v);
    cplx r2 = dot3(v);
    cplx ir2 = cinv(r2);
    cplx d = cinv(csqrt_p(r2));
    // w / r2 and z / r2 are folded once, so that a step's dependent chain is a
    // complex multiply and one fused multiply-add (the ir2 a term is off it)
    cplx wi = w * ir2, zi = v.z * ir2;
    for (int k = 1; k <= am; ++k) d = (d * wi) * (double)(2 * k - 1);
    bool neg = (m < 0 && (am & 1)) != flip;
    if (neg) d = -d;
    f(am, d);
    if (am + 1 > P) return;
    cplx a = d, b = (2.0 * am + 1.0) * (zi * d);
    f(am + 1, b);
    for (int n = am + 2; n <= P; ++n) {
        cplx x = zi * b, y = ir2 * a;
        double c1 = 2.0 * n - 1.0, c2 = (double)(n + am - 1) * (double)(n - am - 1);
        cplx c = mk(fma(c1, x.re, -c2 * y.re), fma(c1, x.im, -c2 * y.im));
        f(n, c);
        a = b;
        b = c;
    }
}

// The M2L table of one pair: I_l^q(v) for l = 0..Lt in this lane's order q
// (|q| <= Lt), passed to st(i, value) with i = base(l) + q in the table layout
// (rows packed in order of l, q = 0 of row l at a multiple of 16 entries and
// three guard entries below q = -l; the row bases are formed here in scalar
// registers, so no load sits on the chain).  The pair enters through its
// constants 1/r2, 1/rho, z/r2 and w/r2 (w = w+ for q >= 0, w- below; formed
// once per plan by k_l3d_m2l_pairs).  Every lane runs the same loop over l:
// steps l <= |q| climb the diagonal I_l^l, the steps past it the three-term
// recurrence in l, both of the form
//   next = (2l - 1) (u cur) - beta_l (prev / r2),  u = w / r2 or z / r2,
// where beta_l = max((l-1)^2 - q^2, 0) is (l+|q|-1)(l-|q|-1) past the
// diagonal and zero up to l = |q| + 1; so the wavefront never diverges, and a
// lane stores row l once l >= |q|.
template <class F>
__device__ inline void table_I(cplx ir2, cplx cur, cplx zi, cplx wi, int q, int Lt, F st)
{
    int aq = q < 0 ? -q : q;
    if (q < 0 && (aq & 1)) cur = -cur;
    cplx prev = mk(0.0, 0.0);
    int end = 3;                                 // one past the last entry of the previous row
    int rb = (end + 3 + 15) & ~15;               // base of row 0
    end = rb + 1;
    if (aq == 0) st(rb, cur);
    double c1 = 1.0, c2 = -(double)aq * (double)aq;
    for (int l = 1; l <= Lt; ++l) {
        cplx u = l <= aq ? wi : zi;
        double b2 = fmax(c2, 0.0);
        cplx x = u * cur, y = ir2 * prev;
        cplx c = mk(fma(c1, x.re, -b2 * y.re), fma(c1, x.im, -b2 * y.im));
        prev = cur;
        cur = c;
        rb = (end + l + 3 + 15) & ~15;
        end = rb + l + 1;
        if (l >= aq) st(rb + q, cur);
        c2 += c1;
        c1 += 2.0;
    }
}

// Recurrence constants, n, m <= 31: 1/((n+m)(n-m)) for m < n, 1/(2m), 2n-1 and
// (n+m-1)(n-m-1).
constexpr int kLT = 32;
__constant__ double c_lrr[kLT * kLT];
__constant__ double c_ldg[kLT];
__constant__ double c_lodd[kLT];
__constant__ double c_lka[kLT * kLT];

// sum over n <= P, |m| <= n of C[nm(n, m)] R_n^m(x): the diagonal start of
// column m is carried from column m - 1, and the columns +m and -m (same
// recurrence coefficients, starts from w+ and w-) run side by side.
__device__ inline cplx reg_sum(const Vec3& x, int P, const cplx* __restrict__ C)
{
    cplx wp = wplus(x), wm = wminus(x), r2 = dot3(x), z = x.z;
    cplx dp = mk(1.0, 0.0), dm = mk(1.0, 0.0), acc = mk(0.0, 0.0);
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            double f = c_ldg[m];
            dp = (dp * wp) * f;
            dm = (dm * wm) * f;
        }
        cplx ap = dp, am = (m & 1) ? -dm : dm;
        cfma(acc, C[nm(m, m)], ap);
        if (m > 0) cfma(acc, C[nm(m, -m)], am);
        if (m + 1 > P) continue;
        cplx bp = z * ap, bm = z * am;
        cfma(acc, C[nm(m + 1, m)], bp);
        if (m > 0) cfma(acc, C[nm(m + 1, -m)], bm);
        // the coefficients and constants of step n are loaded during step
        // n - 1 (uniform: scalar registers), so no step waits on its loads
        int n1 = min(m + 2, P);
        double o = c_lodd[n1], f = c_lrr[n1 * kLT + m];
        cplx kp = C[nm(n1, m)], km = C[nm(n1, -m)];
        for (int n = m + 2; n <= P; ++n) {
            int nx = min(n + 1, P);
            double o2 = c_lodd[nx], f2 = c_lrr[nx * kLT + m];
            cplx kp2 = C[nm(nx, m)], km2 = C[nm(nx, -m)];
            cplx cp = (o * (z * bp) - r2 * ap) * f;
            cplx cm = (o * (z * bm) - r2 * am) * f;
            cfma(acc, kp, cp);
            if (m > 0) cfma(acc, km, cm);
            ap = bp; bp = cp;
            am = bm; bm = cm;
            o = o2; f = f2; kp = kp2; km = km2;
        }
    }
    return acc;
}

// sum over n <= P, |m| <= n of C[nm(n, m)] I_n^m(y), principal rho.
__device__ inline cplx irr_sum(const Vec3& y, int P, const cplx* __restrict__ C)
{
    cplx r2 = dot3(y), ir2 = cinv(r2);
    cplx up = wplus(y) * ir2, um = wminus(y) * ir2, zi = y.z * ir2;
    cplx dp = cinv(csqrt_p(r2)), dm = dp, acc = mk(0.0, 0.0);
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            double f = c_lodd[m];
            dp = (dp * up) * f;
            dm = (dm * um) * f;
        }
        cplx ap = dp, am = (m & 1) ? -dm : dm;
        cfma(acc, C[nm(m, m)], ap);
        if (m > 0) cfma(acc, C[nm(m, -m)], am);
        if (m + 1 > P) continue;
        double o1 = c_lodd[m + 1];
        cplx bp = o1 * (zi * ap), bm = o1 * (zi * am);
        cfma(acc, C[nm(m + 1, m)], bp);
        if (m > 0) cfma(acc, C[nm(m + 1, -m)], bm);
        for (int n = m + 2; n <= P; ++n) {
            double o = c_lodd[n], k = c_lka[n * kLT + m];
            cplx cp = o * (zi * bp) - k * (ir2 * ap);
            cplx cm = o * (zi * bm) - k * (ir2 * am);
            cfma(acc, C[nm(n, m)], cp);
            if (m > 0) cfma(acc, C[nm(n, -m)], cm);
            ap = bp; bp = cp;
            am = bm; bm = cm;
        }
    }
    return acc;
}

// ------------------------------------------------------------ P2M / P2L
// One workgroup of kL3P2XThreads per box.  Thread (h, c), c < 2P+1, owns the
// output order m = c - P for the points h, h + H, ... of each staged chunk
// (H = kL3P2XThreads / (2P+1) point streams).  The coefficient of order m is (-1)^m X_n^{-m}, i.e. the
// column of |m| started from w- (m >= 0) or from w+ with the sign (-1)^|m|
// (m < 0); sigma is folded into the start, so a step of the column recurrence
// adds its value to the lane's LDS accumulator.  The diagonal start takes |m|
// steps and the column P - |m|, so every lane takes P steps per point.
constexpr int kP2XChunk = 64;
constexpr int kL3P2XThreads = 128;

template <bool IRREGULAR>
__global__ __launch_bounds__(kL3P2XThreads) void k_l3d_p2x(const int* __restrict__ boxes, TreeView tv, PointsView pv, int useL4,
                                                cplx* __restrict__ out)
{
    extern __shared__ cplx sh[];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    int ncol = 2 * P + 1, H = blockDim.x / ncol;
    double* pts = reinterpret_cast<double*>(sh);          // [8][kP2XChunk]: x,y,z re, x,y,z im, sigma re, im
    cplx* acc = sh + 4 * kP2XChunk;                      // [H][P+1][ncol]
    double s = tv.rs[l];
    int t = threadIdx.x, h = t / ncol, col = t % ncol;
    int m = col - P, am = m < 0 ? -m : m;
    bool act = h < H;
    for (int i = t; i < H * (P + 1) * ncol; i += blockDim.x) acc[i] = mk(0.0, 0.0);
    cplx c[3];
    box_centre(tv, b, c);
    double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
    int e0 = useL4 ? tv.l4off[b] : 0, e1 = useL4 ? tv.l4off[b + 1] : 1;
    int64_t n = pv.n;
    for (int e = e0; e < e1; ++e) {
        int src = useL4 ? tv.l4idx[e] : b;
        for (int j0 = tv.pbeg[src]; j0 < tv.pend[src]; j0 += kP2XChunk) {
            int cnt = min(kP2XChunk, tv.pend[src] - j0);
            __syncthreads();
            if (t < cnt) {
                int j = j0 + t;
                for (int d = 0; d < 3; ++d) {
                    pts[d * kP2XChunk + t] = (pv.xre[d * n + j] - c[d].re) * s;
                    pts[(3 + d) * kP2XChunk + t] = (pv.xim[d * n + j] - c[d].im) * s;
                }
                pts[6 * kP2XChunk + t] = pv.sre[j];
                pts[7 * kP2XChunk + t] = pv.sim[j];
            }
            __syncthreads();
            if (!act) continue;
            cplx* ac = acc + h * (P + 1) * ncol + col;
            for (int q = h; q < cnt; q += H) {
                Vec3 y;
                y.x = mk(pts[q], pts[3 * kP2XChunk + q]);
                y.y = mk(pts[kP2XChunk + q], pts[4 * kP2XChunk + q]);
                y.z = mk(pts[2 * kP2XChunk + q], pts[5 * kP2XChunk + q]);
                cplx sig = mk(pts[6 * kP2XChunk + q] * sg, pts[7 * kP2XChunk + q] * sg);
                cplx w = m >= 0 ? wminus(y) : wplus(y);
                cplx r2 = dot3(y);
                if (!IRREGULAR) {
                    cplx a = sig;
                    for (int k = 1; k <= am; ++k) a = (a * w) * c_ldg[k];
                    ac[am * ncol] += a;
                    if (am + 1 > P) continue;
                    cplx bb = y.z * a;
                    ac[(am + 1) * ncol] += bb;
                    for (int nn = am + 2; nn <= P; ++nn) {
                        cplx cc = (c_lodd[nn] * (y.z * bb) - r2 * a) * c_lrr[nn * kLT + am];
                        ac[nn * ncol] += cc;
                        a = bb;
                        bb = cc;
                    }
                } else {
                    cplx ir2 = cinv(r2), u = w * ir2, zi = y.z * ir2;
                    cplx a = sig * cinv(csqrt_p(r2));
                    for (int k = 1; k <= am; ++k) a = (a * u) * c_lodd[k];
                    ac[am * ncol] += a;
                    if (am + 1 > P) continue;
                    cplx bb = c_lodd[am + 1] * (zi * a);
                    ac[(am + 1) * ncol] += bb;
                    for (int nn = am + 2; nn <= P; ++nn) {
                        cplx cc = c_lodd[nn] * (zi * bb) - c_lka[nn * kLT + am] * (ir2 * a);
                        ac[nn * ncol] += cc;
                        a = bb;
                        bb = cc;
                    }
                }
            }
        }
    }
    __syncthreads();
    if (h == 0) {
        cplx* o = out + tv.eoff[b];
        for (int nn = am; nn <= P; ++nn) {
            cplx v = acc[nn * ncol + col];
            for (int hh = 1; hh < H; ++hh) v += acc[(hh * (P + 1) + nn) * ncol + col];
            if (useL4) o[nm(nn, m)] += v;
            else o[nm(nn, m)] = v;
        }
    }
}

// The same for P <= 15 with the columns paired for equal work.  Lane slot c
// of a point stream runs the column |m| = a and then the column
// b = P + 1 - a of the same sign (P - a + 1 and a steps, P + 1 in all); slot 0
// runs m = 0 alone, and for odd P the slot a = (P + 1)/2 its column alone, so
// NL = 2 ceil(P/2) + 1 slots cover the (P + 1)^2 coefficients once.  Step s of
// a slot is a column's diagonal start, sigma C w^|m| (P2M) or
// (sigma / rho) C (w / r2)^|m| (P2L), the power by squaring, or one step of
// the recurrence in n written as
//   next = alpha_s (A cur) - beta_s (B prev),
// A = z, B = r2 (P2M) or A = z / r2, B = 1 / r2 (P2L).  Each point's A, B,
// w+-, w-- (over r2 for P2L) and start factor are formed once, by one thread,
// into LDS; the step constants once per workgroup.  A wavefront holds
// floor(64 / NL) point streams with register sums (static step index); they
// meet by lane exchanges, then the wavefronts in LDS, in fixed orders.
constexpr int kP2XPairThreads = 256;
constexpr int kP2XPairChunk = 128;
constexpr int kP2XPairMaxP = 15;

struct P2XSlot {
    int sg, a, b, na;   // sign (+1 for m >= 0), first and second column (b < 0: none), steps in column a
};

__device__ inline P2XSlot p2x_slot(int c, int P)
{
    int hp = (P + 1) >> 1;
    P2XSlot q;
    q.sg = c <= hp ? 1 : -1;
    q.a = c <= hp ? c : c - hp;
    q.b = P + 1 - q.a;
    if (q.a == 0 || q.b == q.a) q.b = -1;
    q.na = P - q.a + 1;
    return q;
}

// column start factor: the sign (-1)^|m| for m < 0 times 1/(2^|m| |m|!) (P2M)
// or (2|m| - 1)!! (P2L)
template <bool IRREGULAR>
__device__ inline double p2x_start_const(int am, int sg)
{
    double c = 1.0;
    if (IRREGULAR) {
        for (int k = 1; k <= am; ++k) c *= 2.0 * k - 1.0;
    } else {
        for (int k = 1; k <= am; ++k) c *= (double)k;
        c = ldexp(1.0 / c, -am);
    }
    return (sg < 0 && (am & 1)) ? -c : c;
}

// x^ea and x^eb, 0 <= ea, eb <= 15, by squaring with no data-dependent branch
__device__ inline void cpow_pair15(cplx x, int ea, int eb, cplx& ra, cplx& rb)
{
    cplx one = mk(1.0, 0.0);
    cplx x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
    ra = (ea & 1) ? x : one;
    rb = (eb & 1) ? x : one;
    ra = ra * ((ea & 2) ? x2 : one);
    rb = rb * ((eb & 2) ? x2 : one);
    ra = ra * ((ea & 4) ? x4 : one);
    rb = rb * ((eb & 4) ? x4 : one);
    ra = ra * ((ea & 8) ? x8 : one);
    rb = rb * ((eb & 8) ? x8 : one);
}

template <bool IRREGULAR>
__global__ __launch_bounds__(kP2XPairThreads) void k_l3d_p2x_r(const int* __restrict__ boxes, TreeView tv,
                                                               PointsView pv, int useL4, cplx* __restrict__ out)
{
    constexpr int PM = kP2XPairMaxP, CH = kP2XPairChunk, NW = kP2XPairThreads / 64;
    extern __shared__ cplx sh[];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    int nc = (P + 1) * (P + 1);
    int NL = 2 * ((P + 1) >> 1) + 1, SW = 64 / NL;
    cplx* pt = sh;                                        // [5][CH]: A, B, W(m >= 0), W(m < 0), start
    cplx* acc = sh + 5 * CH;                              // [NW][nc]
    double2* coef = reinterpret_cast<double2*>(acc + NW * nc);   // [NL][P + 1]
    double s = tv.rs[l];
    int t = threadIdx.x, wv = t >> 6, ln = t & 63, h = ln / NL, c = ln - h * NL;
    bool act = h < SW;
    int nst = NW * SW, st = wv * SW + h;
    for (int i = t; i < NL * (P + 1); i += blockDim.x) {
        int cc = i / (P + 1), ss = i - cc * (P + 1);
        P2XSlot u = p2x_slot(cc, P);
        int n = -1, am = 0;
        if (ss < u.na) {
            n = u.a + ss;
            am = u.a;
        } else if (u.b >= 0) {
            n = u.b + ss - u.na;
            am = u.b;
        }
        double al = 0.0, be = 0.0;
        if (n > am) {
            if (IRREGULAR) {
                al = 2.0 * n - 1.0;
                be = (double)(n + am - 1) * (double)(n - am - 1);
            } else if (n == am + 1) {
                al = 1.0;
            } else {
                double d = 1.0 / ((double)(n + am) * (double)(n - am));
                al = (2.0 * n - 1.0) * d;
                be = d;
            }
        }
        coef[i] = make_double2(al, be);
    }
    P2XSlot q = p2x_slot(act ? c : 0, P);
    double ca = p2x_start_const<IRREGULAR>(q.a, q.sg);
    double cb = q.b >= 0 ? p2x_start_const<IRREGULAR>(q.b, q.sg) : 0.0;
    int eb = q.b >= 0 ? q.b : 0;
    const cplx* wsel = pt + (q.sg > 0 ? 2 : 3) * CH;
    const double2* cf = coef + (act ? c : 0) * (P + 1);
    cplx r[PM + 1];
#pragma unroll
    for (int k = 0; k <= PM; ++k) r[k] = mk(0.0, 0.0);
    cplx cen[3];
    box_centre(tv, b, cen);
    int e0 = useL4 ? tv.l4off[b] : 0, e1 = useL4 ? tv.l4off[b + 1] : 1;
    int64_t n = pv.n;
    for (int e = e0; e < e1; ++e) {
        int src = useL4 ? tv.l4idx[e] : b;
        for (int j0 = tv.pbeg[src]; j0 < tv.pend[src]; j0 += CH) {
            int cnt = min(CH, tv.pend[src] - j0);
            __syncthreads();
            if (t < cnt) {
                int j = j0 + t;
                Vec3 y;
                y.x = mk((pv.xre[j] - cen[0].re) * s, (pv.xim[j] - cen[0].im) * s);
                y.y = mk((pv.xre[n + j] - cen[1].re) * s, (pv.xim[n + j] - cen[1].im) * s);
                y.z = mk((pv.xre[2 * n + j] - cen[2].re) * s, (pv.xim[2 * n + j] - cen[2].im) * s);
                cplx sig = mk(pv.sre[j], pv.sim[j]);
                cplx r2 = dot3(y), wm = wminus(y), wp = wplus(y);
                if (IRREGULAR) {
                    cplx ir2 = cinv(r2);
                    pt[t] = y.z * ir2;
                    pt[CH + t] = ir2;
                    pt[2 * CH + t] = wm * ir2;
                    pt[3 * CH + t] = wp * ir2;
                    pt[4 * CH + t] = sig * cinv(csqrt_p(r2));
                } else {
                    pt[t] = y.z;
                    pt[CH + t] = r2;
                    pt[2 * CH + t] = wm;
                    pt[3 * CH + t] = wp;
                    pt[4 * CH + t] = sig;
                }
            }
            __syncthreads();
            if (!act) continue;
            for (int p = st; p < cnt; p += nst) {
                cplx A = pt[p], B = pt[CH + p], S = pt[4 * CH + p];
                cplx xa, xb;
                cpow_pair15(wsel[p], q.a, eb, xa, xb);
                cplx da = (S * xa) * ca, db = (S * xb) * cb;
                cplx prev = mk(0.0, 0.0), cur = mk(0.0, 0.0);
#pragma unroll
                for (int k = 0; k <= PM; ++k) {
                    if (k <= P) {
                        double2 ab = cf[k];
                        cplx x = A * cur, yv = B * prev;
                        cplx rec = mk(fma(ab.x, x.re, -ab.y * yv.re), fma(ab.x, x.im, -ab.y * yv.im));
                        cplx v = k == 0 ? da : (k == q.na ? db : rec);
                        r[k] += v;
                        prev = cur;
                        cur = v;
                    }
                }
            }
        }
    }
    // the streams of a wavefront: slot c of stream 0 adds streams 1.. in order
#pragma unroll
    for (int k = 0; k <= PM; ++k) {
        cplx v = r[k];
        for (int hh = 1; hh < SW; ++hh) {
            int from = min(ln + hh * NL, 63);
            v.re += __shfl(r[k].re, from, 64);
            v.im += __shfl(r[k].im, from, 64);
        }
        r[k] = v;
    }
    if (h == 0) {
#pragma unroll
        for (int k = 0; k <= PM; ++k) {
            if (k <= P) {
                int nn = -1, am = 0;
                if (k < q.na) {
                    nn = q.a + k;
                    am = q.a;
                } else if (q.b >= 0) {
                    nn = q.b + k - q.na;
                    am = q.b;
                }
                if (nn >= 0) acc[wv * nc + nm(nn, q.sg > 0 ? am : -am)] = r[k];
            }
        }
    }
    __syncthreads();
    cplx* o = out + tv.eoff[b];
    for (int i = t; i < nc; i += blockDim.x) {
        cplx v = acc[i];
        for (int w = 1; w < NW; ++w) v += acc[w * nc + i];
        if (useL4) o[i] += v;
        else o[i] = v;
    }
}

// ------------------------------------------------------------------ M2M
// Coefficient (n, m) of task u when the outputs are taken in falling n and,
// within a degree, in the order m = 0, 1, -1, 2, -2, ...
__device__ inline void l3_task_desc(int u, int P, int& n, int& m)
{
    int v = (P + 1) * (P + 1) - 1 - u;
    n = (int)sqrtf((float)v + 0.5f);
    int i = (n + 1) * (n + 1) - 1 - v;
    m = (i & 1) ? (i + 1) >> 1 : -(i >> 1);
}

// The same in rising degree.
__device__ inline void l3_task_asc(int u, int& n, int& m)
{
    n = (int)sqrtf((float)u + 0.5f);
    int i = u - n * n;
    m = (i & 1) ? (i + 1) >> 1 : -(i >> 1);
}

// The table of one child slot: T_l^q = (+-1)^q R_l^q(d / w_p), l <= P, by
// columns (thread i of nb (2P + 1) builds column q of slot i / (2P + 1)).
__device__ inline void l3_shift_tables(const TreeView& tv, const cplx* cp, int c0, int nb, int P, double s,
                                       bool sign, cplx* T)
{
    int ncol = 2 * P + 1, nc = (P + 1) * (P + 1);
    for (int i = threadIdx.x; i < nb * ncol; i += blockDim.x) {
        int g = i / ncol, q = i - g * ncol - P;
        cplx cc[3];
        box_centre(tv, c0 + g, cc);
        Vec3 d;
        d.x = (cc[0] - cp[0]) * s; d.y = (cc[1] - cp[1]) * s; d.z = (cc[2] - cp[2]) * s;
        cplx* Tg = T + g * nc;
        col_R(d, q, P, sign && (q & 1), [&](int n, cplx v) { Tg[nm(n, q)] = v; });
    }
}

// One workgroup of 256 threads per parent.  The children pass through LDS in
// batches of at most CB <= 4 (CB from the LDS budget): per child slot g the
// table T_l^q = (-1)^q R_l^q(d / w_p), which folds the sign of the shift into
// the table, and the child's multipole scaled by 2^-j.  Lane task (u, g) sums
// the contribution of slot g to output (n, m) = task u, over j <= n and only
// the orders k with |k - m| <= n - j, where the table entry
// T_{n-j}^{k-m} exists; the four slots of an output sit in adjacent lanes and
// meet by two lane exchanges in a fixed order.  Outputs are dealt in falling
// n and rising |m|, so that the lanes of a wavefront run sums of about the
// same length.
__global__ __launch_bounds__(256) void k_l3d_m2m(const int* __restrict__ boxes, TreeView tv, int CB,
                                                 cplx* __restrict__ mpole)
{
    extern __shared__ cplx sh[];
    int p = boxes[blockIdx.x];
    int l = tv.level[p];
    int P = tv.P[l];
    int nc = (P + 1) * (P + 1);
    cplx* sT = sh;             // [CB][nc]
    cplx* sM = sh + CB * nc;   // [CB][nc]
    double s = tv.rs[l];
    int t = threadIdx.x;
    cplx cp[3];
    box_centre(tv, p, cp);
    int c0 = tv.child0[p], nch = tv.nchild[p];
    cplx* out = mpole + tv.eoff[p];
    for (int b0 = 0; b0 < nch; b0 += CB) {
        int nb = min(CB, nch - b0);
        if (b0 > 0) __syncthreads();
        l3_shift_tables(tv, cp, c0 + b0, nb, P, s, true, sT);
        for (int i = t; i < nb * nc; i += blockDim.x) {
            int g = i / nc, e = i - g * nc;
            int j = (int)sqrtf((float)e + 0.5f);
            sM[g * nc + e] = ldexp(1.0, -j) * mpole[tv.eoff[c0 + b0 + g] + e];
        }
        __syncthreads();
        for (int base = 0; base < 4 * nc; base += blockDim.x) {
            int u = (base + t) >> 2, g = (base + t) & 3;
            int n = 0, m = 0;
            cplx a = mk(0.0, 0.0);
            if (u < nc) {
                l3_task_desc(u, P, n, m);
                if (g < nb) {
                    const cplx* Mg = sM + g * nc;
                    const cplx* Tg = sT + g * nc;
                    for (int j = 0; j <= n; ++j) {
                        int lr = n - j;
                        int k0 = max(-j, m - lr), k1 = min(j, m + lr);
                        const cplx* mr = Mg + j * j + j;
                        const cplx* tr = Tg + lr * lr + lr - m;
                        for (int k = k0; k <= k1; ++k) a += mr[k] * tr[k];
                    }
                }
            }
            a.re += __shfl_xor(a.re, 1, 64);
            a.im += __shfl_xor(a.im, 1, 64);
            a.re += __shfl_xor(a.re, 2, 64);
            a.im += __shfl_xor(a.im, 2, 64);
            if (u < nc && g == 0) {
                int o = nm(n, m);
                out[o] = b0 == 0 ? a : out[o] + a;
            }
        }
    }
}

// ------------------------------------------------------------------ M2L
// One workgroup of W wavefronts per target box.  For each List-2
// source box the table I_l^q(D / w), l <= 2P, is built by columns (one lane per
// order q) in LDS, entry (l, q) at base[l] + q with zero guards (layout in
// l3d_layout.hpp), and the source multipole is copied beside it.  The outputs
// are split into groups of four consecutive orders (j, k0..k0+3),
// k0 = -j + 4g; a lane owns up to R groups, as the layout's lane slots assign
// them.  Over the source coefficients (n, m), read at one LDS address by the
// whole wavefront, a group needs I_{j+n}^{m-k0-c}, c = 0..3: at fixed n these
// four entries slide one place along the row l = j + n per step in m, so each
// step loads one table entry for four complex multiply-adds, and the sixteen
// lanes of a quarter wave read sixteen distinct bank slots.  Orders past k = j
// in the last group of a row read guard or neighbouring entries and are
// discarded.  The W wavefronts of the workgroup share the table: the rows n
// of the pair's (Ps+1)^2 steps are dealt to them whole (a row starts with
// three loads of the window and runs in chunks of six steps), balanced by
// their padded length, and the partial sums meet in LDS at the end, added in
// wavefront order.  Sharing the table lets W times as
// many wavefronts reside per unit of LDS; the table itself is built by one
// wavefront while the others wait, which caps W (measured best: 4 with the
// FP64 table, 2 with the FP32 table of half the size).
constexpr int kM2LWaves = 4;
constexpr int kM2LWavesF32 = 2;
// steps per unrolled chunk of a contraction row, and the zeroed table entries
// after the table that the last chunk of the last row may read
constexpr int kM2LChunk = 6;
constexpr int kM2LPad = 8;

struct alignas(16) cplx16 {
    double re, im;
};

// Source expansion length of a List-2 pair from the max-norm distance of the
// box centres in box widths (the real parts; 3..5 with separation 2).
__device__ inline int pair_terms(const L3PairP& pp, const cplx* cb, const cplx* ca, double s)
{
    double dm = 0.0;
    for (int k = 0; k < 3; ++k) dm = fmax(dm, fabs(cb[k].re - ca[k].re));
    int d = (int)(dm * s + 0.5);
    return pp.p[d < 7 ? d : 7];
}

// Per List-2 pair (entry e of the target box's list), once per plan, at the
// scaled offset D / w = (c_target - c_source) / w: the offset src[e] of the
// source box's multipole and the pair's source expansion length Ps.  A pair
// the point-and-shoot kernel takes gets ps[e] = ~Ps (negative) and
// c[5e..5e+4] = e^{ia}, e^{-ia}, e^{ib}, e^{-ib}, 1/rho; any other pair
// ps[e] = Ps and the constants of its table, 1/r2, 1/rho, z/r2, w+/r2, w-/r2.
__global__ __launch_bounds__(64) void k_l3d_m2l_pairs(const int* __restrict__ boxes, TreeView tv, L3PairP pp,
                                                      cplx* __restrict__ c, int* __restrict__ ps,
                                                      int* __restrict__ src)
{
    int b = boxes[blockIdx.x];
    double s = tv.rs[tv.level[b]];
    cplx cb[3];
    box_centre(tv, b, cb);
    for (int e = tv.l2off[b] + (int)threadIdx.x; e < tv.l2off[b + 1]; e += blockDim.x) {
        int a = tv.l2idx[e];
        cplx ca[3];
        box_centre(tv, a, ca);
        Vec3 d;
        d.x = (cb[0] - ca[0]) * s; d.y = (cb[1] - ca[1]) * s; d.z = (cb[2] - ca[2]) * s;
        cplx r2 = dot3(d);
        cplx ir2 = cinv(r2);
        int Ps = pair_terms(pp, cb, ca, s);
        src[e] = tv.eoff[a];
        if (pp.pns_P > 0) {
            // point and shoot: D = rho (sin b cos a, sin b sin a, cos b) at
            // complex angles, e^{ia} = w+ / s, e^{ib} = (z + i s) / rho with
            // s^2 = x^2 + y^2; taken where the phases' powers stay bounded
            cplx rho = csqrt_p(r2), sq = csqrt_p(d.x * d.x + d.y * d.y);
            if (cabs2(sq) > 1e-24 * cabs2(r2)) {
                cplx is = cinv(sq), irho = cinv(rho);
                cplx ea = wplus(d) * is, iea = wminus(d) * is;
                cplx eb = (d.z + times_i(sq)) * irho, ieb = (d.z - times_i(sq)) * irho;
                double k2 = fmax(fmax(cabs2(ea), cabs2(iea)), fmax(cabs2(eb), cabs2(ieb)));
                if ((double)pp.pns_P * log(k2) <= pp.pns_logb) {
                    c[5 * (size_t)e + 0] = ea;
                    c[5 * (size_t)e + 1] = iea;
                    c[5 * (size_t)e + 2] = eb;
                    c[5 * (size_t)e + 3] = ieb;
                    c[5 * (size_t)e + 4] = irho;
                    ps[e] = ~Ps;
                    continue;
                }
            }
        }
        c[5 * (size_t)e + 0] = ir2;
        c[5 * (size_t)e + 1] = cinv(csqrt_p(r2));
        c[5 * (size_t)e + 2] = d.z * ir2;
        c[5 * (size_t)e + 3] = wplus(d) * ir2;
        c[5 * (size_t)e + 4] = wminus(d) * ir2;
        ps[e] = Ps;
    }
}

// C consecutive steps m0 .. m0 + C - 1 of contraction row n (see below);
// with PAD the steps past m = n take a zero coefficient and read finite table
// entries, or the zeroed pad after the table (at most C - 1 entries past the
// row's last step).
template <int R, int C, bool PAD>
__device__ inline void m2l_steps(cplx (&acc)[R][4], const cplx16* const (&row)[R], cplx16 (&w1)[R],
                                 cplx16 (&w2)[R], cplx16 (&w3)[R], const cplx16* Mn, int m0, int n)
{
#pragma unroll
    for (int u = 0; u < C; ++u) {
        int m = m0 + u;
        cplx am;
        if (PAD) {
            bool on = m <= n;
            cplx16 mv = Mn[on ? m : n];
            am = on ? mk(mv.re, mv.im) : mk(0.0, 0.0);
        } else {
            cplx16 mv = Mn[m];
            am = mk(mv.re, mv.im);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cplx16 w0 = row[r][m];
            cfma(acc[r][0], am, mk(w0.re, w0.im));
            cfma(acc[r][1], am, mk(w1[r].re, w1[r].im));
            cfma(acc[r][2], am, mk(w2[r].re, w2[r].im));
            cfma(acc[r][3], am, mk(w3[r].re, w3[r].im));
            w3[r] = w2[r];
            w2[r] = w1[r];
            w1[r] = w0;
        }
    }
}

template <int R>
__global__ __launch_bounds__(64 * kM2LWaves) void k_l3d_m2l(const int* __restrict__ boxes, int nboxes, TreeView tv,
                                                 const int* __restrict__ map, int ntab,
                                                 const cplx* __restrict__ pc, const int* __restrict__ pps,
                                                 const int* __restrict__ psrc, const unsigned* __restrict__ rows64,
                                                 const cplx* __restrict__ mpole,
                                                 cplx* __restrict__ local, int accum)
{
    extern __shared__ cplx16 tab16[];
    int b = boxes[xcd_contiguous(blockIdx.x, nboxes)];
    int l = tv.level[b];
    int P = tv.P[l];
    int nc = (P + 1) * (P + 1);
    cplx* tab = reinterpret_cast<cplx*>(tab16);
    int* base = reinterpret_cast<int*>(tab16 + ntab + kM2LPad);
    double s = tv.rs[l];
    int t = threadIdx.x, lane = t & 63;
    int W = blockDim.x >> 6;
    int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    int jg[R], kg[R];
    bool act[R];
    cplx acc[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int code = map[2 * P + 1 + lane + 64 * r];
        jg[r] = code & 255;
        kg[r] = -jg[r] + 4 * ((code >> 8) & 255);
        act[r] = (code >> 16) & 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = mk(0.0, 0.0);
    }
    for (int i = t; i < ntab + kM2LPad; i += blockDim.x) tab[i] = mk(0.0, 0.0);
    for (int i = t; i <= 2 * P; i += blockDim.x) base[i] = map[i];
    // the pair loop's bounds and per-pair data in scalar registers
    int e0 = __builtin_amdgcn_readfirstlane(tv.l2off[b]);
    int e1 = __builtin_amdgcn_readfirstlane(tv.l2off[b + 1]);
    for (int e = e0; e < e1; ++e) {
        // source orders n <= Ps of this pair: rows l = j + n <= P + Ps of the
        // table; this wavefront contracts the rows n of its mask.  Pairs of
        // the point-and-shoot kernel (Ps < 0) are left to it.
        int Ps = pps[e];
        if (Ps < 0) continue;
        const cplx* M = mpole + psrc[e];
        int Lt = P + Ps;
        unsigned rows = rows64[Ps * kM2LWaves + wv];
        __syncthreads();
        if (t <= 4 * P && abs(t - 2 * P) <= Lt) {
            int q = t - 2 * P;
            const cplx* k = pc + 5 * (size_t)e;
            table_I(k[0], k[1], k[2], q < 0 ? k[4] : k[3], q, Lt, [&](int i, cplx v) { tab[i] = v; });
        }
        __syncthreads();
        while (rows) {
            int n = __builtin_ctz(rows);
            rows &= rows - 1;
            // the source coefficients are read at one address by the whole
            // wavefront: scalar loads, which leave the LDS to the table
            const cplx16* Mn = reinterpret_cast<const cplx16*>(M) + n * n + n;
            const cplx16* row[R];
            cplx16 w1[R], w2[R], w3[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                row[r] = tab16 + base[jg[r] + n] - kg[r];
                w1[r] = row[r][-n - 1];
                w2[r] = row[r][-n - 2];
                w3[r] = row[r][-n - 3];
            }
            // the 2n + 1 steps in whole chunks of kM2LChunk, the last one
            // zero-padded, so no remainder loop waits on single LDS reads
            for (int m = -n; m <= n; m += kM2LChunk) m2l_steps<R, kM2LChunk, true>(acc, row, w1, w2, w3, Mn, m, n);
        }
    }
    // partial sums of wavefronts 1..W-1 through LDS (the table is free now)
    __syncthreads();
    if (wv > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) tab[((size_t)((wv - 1) * R + r) * 4 + c) * 64 + lane] = acc[r][c];
    }
    __syncthreads();
    if (wv > 0) return;
    for (int w = 1; w < W; ++w)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += tab[((size_t)((w - 1) * R + r) * 4 + c) * 64 + lane];
    cplx* o = local + tv.eoff[b];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!act[r]) continue;
        int j = jg[r];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int k = kg[r] + c;
            if (k > j) break;
            cplx v = acc[r][c];
            if ((j + k) & 1) v = -v;
            if (accum) v += o[nm(j, k)];
            o[nm(j, k)] = v;
        }
    }
}

// Mixed-precision M2L: the same lane layout with an FP32 table and FP32
// source coefficients (8-byte entries).  The table is built in FP64 and
// rounded; each row n of the contraction (2n+1 terms) is summed in FP32 and
// the row sums are added in FP64.  Used for P <= kM2LF32MaxP, where every
// table entry I_l^q (l <= 2P, |D/w| > 1.7) stays far inside the FP32 range.
constexpr int kM2LF32MaxP = 16;

template <int R>
__global__ __launch_bounds__(64 * kM2LWavesF32) void k_l3d_m2l_f32(const int* __restrict__ boxes, int nboxes, TreeView tv,
                                                     const int* __restrict__ map, int ntab,
                                                     const cplx* __restrict__ pc, const int* __restrict__ pps,
                                                     const int* __restrict__ psrc,
                                                     const unsigned* __restrict__ rows32,
                                                     const cplx* __restrict__ mpole,
                                                     cplx* __restrict__ local, int accum)
{
    extern __shared__ float2 tabf[];
    int b = boxes[xcd_contiguous(blockIdx.x, nboxes)];
    int l = tv.level[b];
    int P = tv.P[l];
    int nc = (P + 1) * (P + 1);
    float2* Ms = tabf + ntab + kM2LPad;
    int* base = reinterpret_cast<int*>(Ms + nc);
    double s = tv.rs[l];
    int t = threadIdx.x, lane = t & 63;
    int W = blockDim.x >> 6;
    int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    int jg[R], kg[R];
    bool act[R];
    cplx acc[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int code = map[2 * P + 1 + lane + 64 * r];
        jg[r] = code & 255;
        kg[r] = -jg[r] + 4 * ((code >> 8) & 255);
        act[r] = (code >> 16) & 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = mk(0.0, 0.0);
    }
    for (int i = t; i < ntab + kM2LPad; i += blockDim.x) tabf[i] = make_float2(0.0f, 0.0f);
    for (int i = t; i <= 2 * P; i += blockDim.x) base[i] = map[i];
    int e0 = __builtin_amdgcn_readfirstlane(tv.l2off[b]);
    int e1 = __builtin_amdgcn_readfirstlane(tv.l2off[b + 1]);
    for (int e = e0; e < e1; ++e) {
        int Ps = pps[e];
        if (Ps < 0) continue;                 // a point-and-shoot pair
        const cplx* M = mpole + psrc[e];
        int Lt = P + Ps, ncp = (Ps + 1) * (Ps + 1);
        unsigned rows = rows32[Ps * kM2LWavesF32 + wv];   // this wavefront's rows n
        __syncthreads();
        for (int i = t; i < ncp; i += blockDim.x) Ms[i] = make_float2((float)M[i].re, (float)M[i].im);
        if (t <= 4 * P && abs(t - 2 * P) <= Lt) {
            int q = t - 2 * P;
            const cplx* k = pc + 5 * (size_t)e;
            table_I(k[0], k[1], k[2], q < 0 ? k[4] : k[3], q, Lt,
                    [&](int i, cplx v) { tabf[i] = make_float2((float)v.re, (float)v.im); });
        }
        __syncthreads();
        while (rows) {
            int n = __builtin_ctz(rows);
            rows &= rows - 1;
            int mlo = -n, mhi = n;
            const float2* Mn = Ms + n * n + n;
            const float2* row[R];
            float2 w1[R], w2[R], w3[R], f[R][4];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                row[r] = tabf + base[jg[r] + n] - kg[r];
                w1[r] = row[r][mlo - 1];
                w2[r] = row[r][mlo - 2];
                w3[r] = row[r][mlo - 3];
#pragma unroll
                for (int c = 0; c < 4; ++c) f[r][c] = make_float2(0.0f, 0.0f);
            }
#pragma unroll 4
            for (int m = mlo; m <= mhi; ++m) {
                float2 am = Mn[m];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float2 w0 = row[r][m];
                    float2 wv4[4] = {w0, w1[r], w2[r], w3[r]};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        f[r][c].x = fmaf(am.x, wv4[c].x, f[r][c].x);
                        f[r][c].x = fmaf(-am.y, wv4[c].y, f[r][c].x);
                        f[r][c].y = fmaf(am.x, wv4[c].y, f[r][c].y);
                        f[r][c].y = fmaf(am.y, wv4[c].x, f[r][c].y);
                    }
                    w3[r] = w2[r];
                    w2[r] = w1[r];
                    w1[r] = w0;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] += mk((double)f[r][c].x, (double)f[r][c].y);
        }
    }
    // partial sums of wavefronts 1..W-1 through LDS (the table is free now)
    cplx* red = reinterpret_cast<cplx*>(tabf);
    __syncthreads();
    if (wv > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[((size_t)((wv - 1) * R + r) * 4 + c) * 64 + lane] = acc[r][c];
    }
    __syncthreads();
    if (wv > 0) return;
    for (int w = 1; w < W; ++w)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += red[((size_t)((w - 1) * R + r) * 4 + c) * 64 + lane];
    cplx* o = local + tv.eoff[b];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!act[r]) continue;
        int j = jg[r];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int k = kg[r] + c;
            if (k > j) break;
            cplx v = acc[r][c];
            if ((j + k) & 1) v = -v;
            if (accum) v += o[nm(j, k)];
            o[nm(j, k)] = v;
        }
    }
}

// ------------------------------------------------- M2L by point and shoot
// Sec. 5.2: rotate the multipole so that the offset D lies on the z axis,
// translate along it, rotate the local back.  In the orthonormal scaling
// Mh_n^m = c_n^m M_n^m, Lh_j^k = L_j^k / c_j^k with c_n^m = sqrt((n-m)!(n+m)!),
// a rotation about z multiplies order m by a phase, and a rotation about y by
// angle b is Y diag(e^{-imb}) Y^T with Y^n = d^n(pi/2), a fixed real orthogonal
// matrix per degree (Wigner's; Y^n_{m m'} = (-1)^{m-m'} Y^n_{m' m}).  With
// D = rho (sin b cos a, sin b sin a, cos b) at complex angles, one pair is
//   x0 = (-i)^m e^{ima} Mh,  x1 = Y^T x0,  x2 = e^{imb} x1,  x3 = Y x2,
//   y0_j^k = sum_n Zh^k_{jn} rho^-(j+n+1) x3_n^k,
//   Zh^k_{jn} = (-1)^{j+k} (j+n)! / sqrt((j-k)!(j+k)!(n-k)!(n+k)!)   (coaxial),
//   y1 = Y^T y0,  y2 = e^{-imb} y1,  y3 = Y y2,  Lh += i^k e^{-ika} y3,
// every dense step a real matrix per degree, the same for all pairs; only the
// phases and the powers of 1/rho belong to the pair.  One workgroup of 256
// threads per target box, thread t = n^2 + n + m owning coefficient (n, m)
// (P <= 15); its column of Y^n and its row of Zh stay in registers, the
// stages pass the coefficient vector through LDS.
constexpr int kPnsMaxP = 15;
constexpr int kPnsY = (kPnsMaxP + 1) * (2 * kPnsMaxP + 1) * (2 * kPnsMaxP + 3) / 3;
__device__ double g_pns_y[kPnsY];                                      // columns of Y^n, packed
__device__ double g_pns_z[(kPnsMaxP + 1) * (2 * kPnsMaxP + 1) * (kPnsMaxP + 1)];   // [j][k + 15][n - |k|]
__device__ double g_pns_c[(kPnsMaxP + 1) * (kPnsMaxP + 1)];            // c_n^m at n^2 + n + m
__device__ double g_pns_fact[2 * kPnsMaxP + 1];                         // i!

// base of degree n's columns in g_pns_y: sum_{n' < n} (2n' + 1)^2
__host__ __device__ constexpr int pns_ybase(int n) { return n * (2 * n - 1) * (2 * n + 1) / 3; }

// z^q for 0 <= q < 32 by binary powers
__device__ inline cplx cpow_small(cplx z, int q)
{
    cplx r = mk(1.0, 0.0);
    while (q) {
        if (q & 1) r = r * z;
        q >>= 1;
        if (q) z = z * z;
    }
    return r;
}

// A rotation of degree n over a folded row: with the symmetries of d^n(pi/2),
// Y_{m' -m} = (-1)^{n+m'} Y_{m' m}, Y_{m m'} = (-1)^{m-m'} Y_{m' m} and so
// Y_{-k, m} = (-1)^{n+m} Y_{k m},
// the lane of order m >= 0 needs only V_k = x_k + (-1)^{n+m} x_{-k} (k > 0,
// V_0 = x_0) and its column yc[k] = Y^n_{k m}, k = 0..n (zero past n).  With
// E and O the sums over even and odd k,
//   (Y^T x)_{+m} = E + O,          (Y^T x)_{-m} = (-1)^n (E - O),
//   (Y x)_{+m} = (-1)^m (E - O),   (Y x)_{-m} = (-1)^{n+m} (E + O),
// for n + 1 reads instead of 2n + 1.  Steps run in blocks of eight up to the
// wavefront's largest degree nw (uniform) with no per-lane branch: a lane's
// steps past n read finite entries of the next rows and multiply them by
// zero, so the block's loads issue together.
template <int PM>
__device__ inline void pns_halves_v(const double (&yc)[PM + 1], const cplx* vs, int nw, cplx& E, cplx& O)
{
    cplx a[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
#pragma unroll
    for (int k0 = 0; k0 <= PM; k0 += 4) {
        if (k0 <= nw) {
#pragma unroll
            for (int k = k0; k < k0 + 4 && k <= PM; ++k) {
                cplx x = vs[k];
                a[k & 1].re = fma(yc[k], x.re, a[k & 1].re);
                a[k & 1].im = fma(yc[k], x.im, a[k & 1].im);
            }
        }
    }
    E = a[0];
    O = a[1];
}

// Folded rows in the stage buffers: V with + (S) of degree n at
// pns_vbase(n, 0), with - (D) at pns_vbase(n, 1), n + 1 entries each.  At a
// step the lanes of a sixteen-lane quarter wave read at most twelve rows,
// whose bases are distinct modulo 16 (2n + p), so their sixteen-byte reads
// fall in distinct groups of four banks.
__host__ __device__ constexpr int pns_vbase(int n, int p) { return 34 * n + 17 * p; }
constexpr int kPnsBufV = 544;                 // pns_vbase(15, 1) + 16 <= 544

// Phase tables of one pair: tEa[q + P] = (-i)^q e^{iqa}, tEb[q + P] = e^{iqb}
// (|q| <= P), tR[i] = rho^-i (i <= P + 1), from this lane's prefetched
// constant (lanes 0..2P: e^{+-ia} and e^{+-ib} by the sign of q; lanes
// 64..64+P+1: 1/rho).
__device__ inline void pns_tables(int t, int P, cplx ka, cplx kb, cplx* tEa, cplx* tEb, cplx* tR)
{
    if (t < 2 * P + 1) {
        int q = t - P, aq = q < 0 ? -q : q;
        int r4 = q & 3;
        cplx ph = r4 == 0 ? mk(1.0, 0.0) : r4 == 1 ? mk(0.0, -1.0) : r4 == 2 ? mk(-1.0, 0.0) : mk(0.0, 1.0);
        tEa[t] = ph * cpow_small(ka, aq);
        tEb[t] = cpow_small(kb, aq);
    } else if (t >= 64 && t < 64 + P + 2) {
        tR[t - 64] = cpow_small(ka, t - 64);
    }
}

// The constants a lane of pns_tables needs for pair entry e.
__device__ inline void pns_consts(int t, int P, const cplx* __restrict__ pc, int e, cplx& ka, cplx& kb)
{
    const cplx* k = pc + 5 * (size_t)e;
    bool lo = t < 2 * P + 1, hi = t >= 64 && t < 64 + P + 2;
    int ia = hi ? 4 : (t < P ? 1 : 0), ib = t < P ? 3 : 2;
    if (lo || hi) ka = k[ia];
    if (lo) kb = k[ib];
}

// Stage buffers hold degree n's coefficients at pns_base(n) + n + m, with
// pns_base(n) = n (mod 16): at a rotation step every lane of degree n reads
// pns_base(n) + s, so the sixteen-byte reads of the degrees in a wavefront
// fall in distinct groups of four banks.
__host__ __device__ constexpr int pns_base(int n) { return 17 * n + 16 * (n > 9 ? n - 9 : 0); }
constexpr int kPnsBuf = 384;                  // pns_base(15) + 31 < 384

// The pairs of a box run as a pipeline of five barrier-separated phases:
//   A: stage 6 of the previous pair | stage 1 of this one,  B: stage 2,
//   C: stage 3,  D: coaxial shift,  E: stage 5 | the next pair's phase tables.
// Pair p writes its stages into buf[p & 1], buf[p & 1 ^ 1], ... alternately and
// reads its tables from slot p & 1, so phase A's two halves touch disjoint
// buffers; the next pair's multipole and constants are loaded into registers
// one pair ahead.  Thread u = n (n + 1) / 2 + m owns the coefficients (n, +m)
// and (n, -m), m >= 0.  ent[k] = (List-2 entry, source offset, Ps) of the
// box's point-and-shoot pairs k = off[b] .. off[b+1]-1.
template <int PM>
constexpr int pns_threads() { return 64 * (((PM + 1) * (PM + 2) / 2 + 63) / 64); }

template <int PM>
__global__ __launch_bounds__(pns_threads<PM>(), 3) void k_l3d_m2l_pns(const int* __restrict__ boxes, int nboxes,
                                                                 TreeView tv, const cplx* __restrict__ pc,
                                                                 const int* __restrict__ off,
                                                                 const int4* __restrict__ ent,
                                                                 const cplx* __restrict__ mpole,
                                                                 cplx* __restrict__ local)
{
    __shared__ cplx buf[2][kPnsBufV];
    __shared__ cplx tEa[2][2 * PM + 1], tEb[2][2 * PM + 1], tR[2][PM + 2];
    int b = boxes[xcd_contiguous(blockIdx.x, nboxes)];
    int P = tv.P[tv.level[b]];
    int t = threadIdx.x;
    int n = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
    while (n * (n + 1) / 2 > t) --n;
    while ((n + 1) * (n + 2) / 2 <= t) ++n;
    int m = t - n * (n + 1) / 2;
    bool on = n <= P;
    int gp = n * n + n + m, gm = n * n + n - m;   // coefficients (n, +m), (n, -m) in the expansions
    int bn = pns_base(n), ip = bn + n + m, im = bn + n - m;   // natural layout, for the coaxial step
    // folded rows: this lane reads row V of its parity and writes entry m of both
    int vr = pns_vbase(n, (n + m) & 1), vs0 = pns_vbase(n, 0) + m, vd0 = pns_vbase(n, 1) + m;
    bool two = on && m > 0;
    double sg = ((m + n) & 1) ? -1.0 : 1.0, sgm = (m & 1) ? -1.0 : 1.0, sgn = (n & 1) ? -1.0 : 1.0;
    // the largest degree among this wavefront's lanes (uniform)
    int tw = min((t | 63), (P + 1) * (P + 2) / 2 - 1);
    int nw = (int)((sqrtf(8.0f * tw + 1.0f) - 1.0f) * 0.5f);
    while (nw * (nw + 1) / 2 > tw) --nw;
    while ((nw + 1) * (nw + 2) / 2 <= tw) ++nw;
    nw = __builtin_amdgcn_readfirstlane(nw);
    double yc[PM + 1];   // Y^n_{k m}, k = 0..n
#pragma unroll
    for (int k = 0; k <= PM; ++k) yc[k] = (on && k <= n) ? g_pns_y[pns_ybase(n) + (m + n) * (2 * n + 1) + n + k] : 0.0;
    // a lane's two values +m, -m into the folded rows (m = 0: V_0 = x_0 in both)
    auto put = [&](cplx* B, cplx vp, cplx vm) {
        if (m == 0) {
            B[vs0] = vp;
            B[vd0] = vp;
        } else {
            B[vs0] = vp + vm;
            B[vd0] = vp - vm;
        }
    };
    double cn = on ? g_pns_c[gp] : 0.0;
    // coaxial factors Zh^m_{n n'} = (-1)^{n+m} (n+n')! / (c_n^m c_n'^m): stage
    // 3 divides by the source coefficient's own c, the coaxial step takes
    // (n + m + i)! by a running product from (n + m)!
    double icn = on ? 1.0 / cn : 0.0;
    double zsg = sg * icn;
    double f0 = on ? g_pns_fact[n + m] : 0.0;
    cplx accp = mk(0.0, 0.0), accm = mk(0.0, 0.0);
    // every entry a stage may read stays finite: zero at the start, and the
    // degrees past a pair's source length are zeroed before the coaxial step
    for (int i = t; i < kPnsBufV; i += blockDim.x) {
        buf[0][i] = mk(0.0, 0.0);
        buf[1][i] = mk(0.0, 0.0);
    }
    int k0 = __builtin_amdgcn_readfirstlane(off[b]);
    int k1 = __builtin_amdgcn_readfirstlane(off[b + 1]);
    int4 cur = k0 < k1 ? ent[k0] : make_int4(0, 0, -1, 0);
    cplx ka = mk(0.0, 0.0), kb = mk(0.0, 0.0), mvp = mk(0.0, 0.0), mvm = mk(0.0, 0.0);
    if (k0 < k1) {
        pns_consts(t, P, pc, cur.x, ka, kb);
        pns_tables(t, P, ka, kb, tEa[0], tEb[0], tR[0]);
        if (on && n <= cur.z) {
            mvp = mpole[cur.y + gp];
            mvm = mpole[cur.y + gm];
        }
    }
    __syncthreads();
    int qp = 0;                                   // slot of the previous pair
    cplx E, O;
    for (int k = k0; k < k1; ++k) {
        int q = (k - k0) & 1;
        int Ps = cur.z;
        bool src_on = on && n <= Ps;
        cplx* X = buf[q];
        cplx* Y = buf[q ^ 1];
        // next pair's entry, multipole and constants, one pair ahead
        int4 nxt = k + 1 < k1 ? ent[k + 1] : make_int4(0, 0, -1, 0);
        // A: the previous pair's last stage (reads buf[qp], slot qp), then
        // this pair's first stage (writes X)
        if (k > k0 && on) {
            pns_halves_v<PM>(yc, buf[qp] + vr, nw, E, O);
            accp += (sgm * (E - O)) * tEa[qp][P - m];
            accm += (sg * (E + O)) * tEa[qp][P + m];
        }
        if (src_on) put(X, tEa[q][m + P] * (cn * mvp), tEa[q][P - m] * (cn * mvm));
        cplx np = mk(0.0, 0.0), nm_ = mk(0.0, 0.0);
        if (k + 1 < k1) {
            if (on && n <= nxt.z) {
                np = mpole[nxt.y + gp];
                nm_ = mpole[nxt.y + gm];
            }
            pns_consts(t, P, pc, nxt.x, ka, kb);
        }
        __syncthreads();
        // B: x1 = Y^T x0, x2 = e^{imb} x1
        if (src_on) {
            pns_halves_v<PM>(yc, X + vr, min(nw, Ps), E, O);
            put(Y, (E + O) * tEb[q][P + m], (sgn * (E - O)) * tEb[q][P - m]);
        }
        __syncthreads();
        // C: x3 = Y x2, times rho^-n / c_n^m; degrees past Ps zeroed
        if (on) {
            cplx vp = mk(0.0, 0.0), vm = mk(0.0, 0.0);
            if (src_on) {
                pns_halves_v<PM>(yc, Y + vr, min(nw, Ps), E, O);
                vp = ((sgm * icn) * (E - O)) * tR[q][n];
                vm = ((sg * icn) * (E + O)) * tR[q][n];
            }
            X[ip] = vp;
            X[im] = vm;
        }
        __syncthreads();
        // D: coaxial for orders +m and -m, sums over source degrees m .. Ps
        if (on) {
            cplx vp = mk(0.0, 0.0), vm = mk(0.0, 0.0);
            // the start index made opaque per pair, so the compiler forms the
            // step addresses here instead of holding 2 (P + 1) of them live
            // source degree nn = m + i; the factor is zero from nn > Ps on,
            // so a clamped index (finite entries) never contributes
            int nn = m;
            asm volatile("" : "+v"(nn));
            double f = m <= Ps ? f0 : 0.0, d = (double)(n + m + 1);
#pragma unroll
            for (int i = 0; i <= PM; ++i) {
                if (i <= Ps) {
                    int ix = min(pns_base(nn) + nn, kPnsBuf - 1 - m);
                    cplx xp = X[ix + m], xm = X[ix - m];
                    vp.re = fma(f, xp.re, vp.re);
                    vp.im = fma(f, xp.im, vp.im);
                    vm.re = fma(f, xm.re, vm.re);
                    vm.im = fma(f, xm.im, vm.im);
                    f = nn < Ps ? f * d : 0.0;
                    d += 1.0;
                }
                ++nn;
            }
            cplx z = tR[q][n + 1] * zsg;
            put(Y, vp * z, vm * z);
        }
        __syncthreads();
        // E: y1 = Y^T y0, y2 = e^{-imb} y1; the next pair's tables
        if (on) {
            pns_halves_v<PM>(yc, Y + vr, nw, E, O);
            put(X, (E + O) * tEb[q][P - m], (sgn * (E - O)) * tEb[q][P + m]);
        }
        if (k + 1 < k1) pns_tables(t, P, ka, kb, tEa[q ^ 1], tEb[q ^ 1], tR[q ^ 1]);
        __syncthreads();
        qp = q;
        cur = nxt;
        mvp = np;
        mvm = nm_;
    }
    if (k1 > k0 && on) {
        pns_halves_v<PM>(yc, buf[qp] + vr, nw, E, O);
        accp += (sgm * (E - O)) * tEa[qp][P - m];
        accm += (sg * (E + O)) * tEa[qp][P + m];
    }
    if (on) {
        local[tv.eoff[b] + gp] = cn * accp;
        if (m > 0) local[tv.eoff[b] + gm] = cn * accm;
    }
}

// ------------------------------------------------------------------ L2L
// One workgroup of 256 threads per parent: its local expansion goes to LDS
// once, and its children pass through in batches of at most CB <= 4, each
// slot with its table T_l^q = R_l^q(d / w_p).  Lane task (u, g) forms output
// (j, k) = task u of slot g's child, over n >= j and only the orders m with
// |m - k| <= n - j; every output of degree j runs a sum of (P - j + 1)^2
// terms, and the tasks are dealt in rising j, so a wavefront's lanes run
// sums of the same or neighbouring lengths.
__global__ __launch_bounds__(256) void k_l3d_l2l(const int* __restrict__ boxes, TreeView tv, int CB,
                                                 cplx* __restrict__ local)
{
    extern __shared__ cplx sh[];
    int p = boxes[blockIdx.x];
    int lp = tv.level[p];
    int P = tv.P[lp];
    int nc = (P + 1) * (P + 1);
    cplx* Lp = sh;             // [nc]
    cplx* sT = sh + nc;        // [CB][nc]
    double s = tv.rs[lp];
    int t = threadIdx.x;
    cplx cp[3];
    box_centre(tv, p, cp);
    int c0 = tv.child0[p], nch = tv.nchild[p];
    for (int i = t; i < nc; i += blockDim.x) Lp[i] = local[tv.eoff[p] + i];
    for (int b0 = 0; b0 < nch; b0 += CB) {
        int nb = min(CB, nch - b0);
        if (b0 > 0) __syncthreads();
        l3_shift_tables(tv, cp, c0 + b0, nb, P, s, false, sT);
        __syncthreads();
        for (int v = t; v < 4 * nc; v += blockDim.x) {
            int u = v >> 2, g = v & 3;
            if (g >= nb) continue;
            int j, k;
            l3_task_asc(u, j, k);
            const cplx* Tg = sT + g * nc;
            cplx a = mk(0.0, 0.0);
            for (int n = j; n <= P; ++n) {
                int lr = n - j;
                int m0 = max(-n, k - lr), m1 = min(n, k + lr);
                const cplx* lrow = Lp + n * n + n;
                const cplx* tr = Tg + lr * lr + lr - k;
                for (int m = m0; m <= m1; ++m) a += lrow[m] * tr[m];
            }
            cplx* o = local + tv.eoff[c0 + b0 + g];
            o[nm(j, k)] += ldexp(1.0, -(j + 1)) * a;
        }
    }
}

// ------------------------------------------------------------- L2P + M2P
// M2P by List-3 entries: entry e = (leaf owner[e], box l3idx[e]) evaluates the
// box's multipole at the leaf's points into part[poff[e] + i - pbeg], one
// wavefront per entry, so a leaf with a long List 3 spreads over many
// wavefronts.
__global__ __launch_bounds__(64) void k_l3d_m2p_part(const int* __restrict__ owner,
                                                     const int64_t* __restrict__ poff, TreeView tv,
                                                     PointsView pv, const cplx* __restrict__ mpole,
                                                     cplx* __restrict__ part)
{
    int e = blockIdx.x;
    int b = owner[e], a = tv.l3idx[e];
    int la = tv.level[a];
    double sa = tv.rs[la];
    cplx c[3];
    box_centre(tv, a, c);
    cplx* o = part + poff[e] - tv.pbeg[b];
    for (int i = tv.pbeg[b] + threadIdx.x; i < tv.pend[b]; i += blockDim.x)
        o[i] = sa * irr_sum(point_rel(pv, i, c, sa), tv.P[la], mpole + tv.eoff[a]);
}

// L2P, one thread per target of a leaf, plus the leaf's List-3 parts in list
// order.
__global__ __launch_bounds__(64) void k_l3d_leaf_far(const int* __restrict__ leaves, int top,
                                                     TreeView tv, PointsView pv,
                                                     const cplx* __restrict__ local,
                                                     const int64_t* __restrict__ poff,
                                                     const cplx* __restrict__ part,
                                                     cplx* __restrict__ ufar)
{
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    for (int i = tv.pbeg[b] + threadIdx.x; i < tv.pend[b]; i += blockDim.x) {
        cplx u = mk(0.0, 0.0);
        if (l >= top) {
            int P = tv.P[l];
            double s = tv.rs[l];
            cplx c[3];
            box_centre(tv, b, c);
            u = s * reg_sum(point_rel(pv, i, c, s), P, local + tv.eoff[b]);
            for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) u += part[poff[e] + i - tv.pbeg[b]];
        }
        ufar[i] = u;
    }
}

// ------------------------------------------------- layer potentials (Sec. 2.1)
// Dipole sources v_j = tau_j nu_j (the double layer) and gradients at the
// targets (the normal derivatives S', D' follow by the target normal).  The
// derivatives of the solid harmonics (checked against central differences):
//   d_z R_n^m = R_{n-1}^m,   (d_x + i d_y) R_n^m = -R_{n-1}^{m+1},  (d_x - i d_y) R_n^m = R_{n-1}^{m-1}
//   d_z I_n^m = -I_{n+1}^m,  (d_x + i d_y) I_n^m = -I_{n+1}^{m+1},  (d_x - i d_y) I_n^m = I_{n+1}^{m-1}
// and v . grad = (v- (d_x + i d_y) + v+ (d_x - i d_y))/2 + v_z d_z with
// v+- = v_x +- i v_y (bilinear: no conjugate).  Coordinates of a level are
// scaled by 1/w, so each derivative in a physical coordinate carries 1/w.
//
// P2M / P2L with dipoles: thread (h, col) owns the column of order m of
// (-1)^m X_n^{-m} (X = R for P2M, I for P2L) at the points h, h + H, ...;
// each value c_n feeds four accumulators, all in the owner's column:
//   acc[n]     += sigma c_n                 (charge, output (n, m))
//   accZ[n']   += a_z  v_z c_n              (output (n', m))
//   accP[n']   += a_pm v- c_n / 2           (output (n', m + 1))
//   accM[n']   -= a_pm v+ c_n / 2           (output (n', m - 1))
// with n' = n + 1, a_z = 1, a_pm = 1 for R (P2M) and n' = n - 1, a_z = -1,
// a_pm = 1 for I (P2L), all over w; the output (n, m) adds acc and accZ of
// its own column, accP of column m - 1 and accM of column m + 1.
template <bool IRREGULAR>
__global__ void k_l3d_p2x_dip(const int* __restrict__ boxes, TreeView tv, PointsView pv,
                              const double* __restrict__ dre, const double* __restrict__ dim, int useL4,
                              cplx* __restrict__ out)
{
    extern __shared__ cplx sh[];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    int ncol = 2 * P + 1, H = blockDim.x / ncol;
    int NR = P + 2;                                       // rows 0 .. P+1
    double* pts = reinterpret_cast<double*>(sh);          // [14][kP2XChunk]
    cplx* acc = sh + 7 * kP2XChunk;                       // [4][H][NR][ncol]
    size_t AS = (size_t)H * NR * ncol;
    double s = tv.rs[l];
    int t = threadIdx.x, h = t / ncol, col = t % ncol;
    int m = col - P, am = m < 0 ? -m : m;
    bool act = h < H;
    for (size_t i = t; i < 4 * AS; i += blockDim.x) acc[i] = mk(0.0, 0.0);
    cplx c[3];
    box_centre(tv, b, c);
    double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
    int e0 = useL4 ? tv.l4off[b] : 0, e1 = useL4 ? tv.l4off[b + 1] : 1;
    int64_t n = pv.n;
    int top = IRREGULAR ? P + 1 : P;                      // highest degree of the column
    for (int e = e0; e < e1; ++e) {
        int src = useL4 ? tv.l4idx[e] : b;
        for (int j0 = tv.pbeg[src]; j0 < tv.pend[src]; j0 += kP2XChunk) {
            int cnt = min(kP2XChunk, tv.pend[src] - j0);
            __syncthreads();
            if (t < cnt) {
                int j = j0 + t;
                for (int d = 0; d < 3; ++d) {
                    pts[d * kP2XChunk + t] = (pv.xre[d * n + j] - c[d].re) * s;
                    pts[(3 + d) * kP2XChunk + t] = (pv.xim[d * n + j] - c[d].im) * s;
                    pts[(8 + d) * kP2XChunk + t] = dre[d * n + j] * s;       // v / w
                    pts[(11 + d) * kP2XChunk + t] = dim[d * n + j] * s;
                }
                pts[6 * kP2XChunk + t] = pv.sre[j];
                pts[7 * kP2XChunk + t] = pv.sim[j];
            }
            __syncthreads();
            if (!act) continue;
            cplx* a0 = acc + (size_t)h * NR * ncol + col;
            cplx* aZ = a0 + AS;
            cplx* aP = a0 + 2 * AS;
            cplx* aM = a0 + 3 * AS;
            for (int q = h; q < cnt; q += H) {
                Vec3 y;
                y.x = mk(pts[q], pts[3 * kP2XChunk + q]);
                y.y = mk(pts[kP2XChunk + q], pts[4 * kP2XChunk + q]);
                y.z = mk(pts[2 * kP2XChunk + q], pts[5 * kP2XChunk + q]);
                cplx sig = mk(pts[6 * kP2XChunk + q], pts[7 * kP2XChunk + q]);
                cplx vx = mk(pts[8 * kP2XChunk + q], pts[11 * kP2XChunk + q]);
                cplx vy = mk(pts[9 * kP2XChunk + q], pts[12 * kP2XChunk + q]);
                cplx vz = mk(pts[10 * kP2XChunk + q], pts[13 * kP2XChunk + q]);
                cplx vm = mk(vx.re + vy.im, vx.im - vy.re) * 0.5;     // (v_x - i v_y) / 2
                cplx vp = mk(vx.re - vy.im, vx.im + vy.re) * -0.5;    // -(v_x + i v_y) / 2
                if (IRREGULAR) vz = -vz;
                cplx w = m >= 0 ? wminus(y) : wplus(y);
                cplx r2 = dot3(y);
                auto feed = [&](int nn, cplx v) {
                    if (nn <= P) a0[nn * ncol] += sig * v;
                    int nd = IRREGULAR ? nn - 1 : nn + 1;
                    if (nd >= 0 && nd <= P) {
                        aZ[nd * ncol] += vz * v;
                        aP[nd * ncol] += vm * v;
                        aM[nd * ncol] += vp * v;
                    }
                };
                if (!IRREGULAR) {
                    cplx a = mk(sg, 0.0);
                    for (int k = 1; k <= am; ++k) a = (a * w) * c_ldg[k];
                    feed(am, a);
                    if (am + 1 > top) continue;
                    cplx bb = y.z * a;
                    feed(am + 1, bb);
                    for (int nn = am + 2; nn <= top; ++nn) {
                        cplx cc = (c_lodd[nn] * (y.z * bb) - r2 * a) * c_lrr[nn * kLT + am];
                        feed(nn, cc);
                        a = bb;
                        bb = cc;
                    }
                } else {
                    cplx ir2 = cinv(r2), u = w * ir2, zi = y.z * ir2;
                    cplx a = cinv(csqrt_p(r2)) * sg;
                    for (int k = 1; k <= am; ++k) a = (a * u) * c_lodd[k];
                    feed(am, a);
                    if (am + 1 > top) continue;
                    cplx bb = c_lodd[am + 1] * (zi * a);
                    feed(am + 1, bb);
                    for (int nn = am + 2; nn <= top; ++nn) {
                        cplx cc = c_lodd[nn] * (zi * bb) - c_lka[nn * kLT + am] * (ir2 * a);
                        feed(nn, cc);
                        a = bb;
                        bb = cc;
                    }
                }
            }
        }
    }
    __syncthreads();
    if (h == 0) {
        cplx* o = out + tv.eoff[b];
        for (int nn = am; nn <= P; ++nn) {
            cplx v = mk(0.0, 0.0);
            for (int hh = 0; hh < H; ++hh) {
                const cplx* base = acc + (size_t)hh * NR * ncol + nn * ncol;
                v += base[col] + base[AS + col];
                if (col > 0) v += base[2 * AS + col - 1];          // accP of order m - 1
                if (col + 1 < ncol) v += base[3 * AS + col + 1];   // accM of order m + 1
            }
            if (useL4) o[nm(nn, m)] += v;
            else o[nm(nn, m)] = v;
        }
    }
}

// sum_n C[nm(n, m)] R_n^m(x) and its gradient in x (scaled units): each
// value R_n^m feeds u (C_n^m), d_z u (C_{n+1}^m), (d_x + i d_y) u
// (-C_{n+1}^{m-1}) and (d_x - i d_y) u (C_{n+1}^{m+1}).
__device__ inline void reg_sum_grad(const Vec3& x, int P, const cplx* __restrict__ C, cplx& u, cplx* g)
{
    cplx wp = wplus(x), wm = wminus(x), r2 = dot3(x), z = x.z;
    cplx dp = mk(1.0, 0.0), dm = mk(1.0, 0.0);
    cplx uz = mk(0.0, 0.0), up = mk(0.0, 0.0), um = mk(0.0, 0.0);
    u = mk(0.0, 0.0);
    auto feed = [&](int n, int m, cplx v) {
        cfma(u, C[nm(n, m)], v);
        if (n + 1 <= P) {
            cfma(uz, C[nm(n + 1, m)], v);
            cfma(up, -C[nm(n + 1, m - 1)], v);
            cfma(um, C[nm(n + 1, m + 1)], v);
        }
    };
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            double f = c_ldg[m];
            dp = (dp * wp) * f;
            dm = (dm * wm) * f;
        }
        cplx ap = dp, am = (m & 1) ? -dm : dm;
        feed(m, m, ap);
        if (m > 0) feed(m, -m, am);
        if (m + 1 > P) continue;
        cplx bp = z * ap, bm = z * am;
        feed(m + 1, m, bp);
        if (m > 0) feed(m + 1, -m, bm);
        for (int n = m + 2; n <= P; ++n) {
            double o = c_lodd[n], f = c_lrr[n * kLT + m];
            cplx cp = (o * (z * bp) - r2 * ap) * f;
            cplx cm = (o * (z * bm) - r2 * am) * f;
            feed(n, m, cp);
            if (m > 0) feed(n, -m, cm);
            ap = bp; bp = cp;
            am = bm; bm = cm;
        }
    }
    g[0] = (up + um) * 0.5;
    g[1] = mk(0.5 * (up.im - um.im), -0.5 * (up.re - um.re));   // -(i/2)(up - um)
    g[2] = uz;
}

// sum_n C[nm(n, m)] I_n^m(y) and its gradient (scaled units): each value
// I_n^m, n <= P + 1, feeds u (C_n^m), d_z u (-C_{n-1}^m), (d_x + i d_y) u
// (-C_{n-1}^{m-1}) and (d_x - i d_y) u (C_{n-1}^{m+1}).
__device__ inline void irr_sum_grad(const Vec3& y, int P, const cplx* __restrict__ C, cplx& u, cplx* g)
{
    cplx r2 = dot3(y), ir2 = cinv(r2);
    cplx upw = wplus(y) * ir2, umw = wminus(y) * ir2, zi = y.z * ir2;
    cplx dp = cinv(csqrt_p(r2)), dm = dp;
    cplx uz = mk(0.0, 0.0), up = mk(0.0, 0.0), um = mk(0.0, 0.0);
    u = mk(0.0, 0.0);
    int Q = P + 1;
    auto coef = [&](int n, int m) -> cplx {
        return (n >= 0 && n <= P && m >= -n && m <= n) ? C[nm(n, m)] : mk(0.0, 0.0);
    };
    auto feed = [&](int n, int m, cplx v) {
        if (n <= P) cfma(u, C[nm(n, m)], v);
        cfma(uz, -coef(n - 1, m), v);
        cfma(up, -coef(n - 1, m - 1), v);
        cfma(um, coef(n - 1, m + 1), v);
    };
    for (int m = 0; m <= Q; ++m) {
        if (m > 0) {
            double f = c_lodd[m];
            dp = (dp * upw) * f;
            dm = (dm * umw) * f;
        }
        cplx ap = dp, am = (m & 1) ? -dm : dm;
        feed(m, m, ap);
        if (m > 0) feed(m, -m, am);
        if (m + 1 > Q) continue;
        double o1 = c_lodd[m + 1];
        cplx bp = o1 * (zi * ap), bm = o1 * (zi * am);
        feed(m + 1, m, bp);
        if (m > 0) feed(m + 1, -m, bm);
        for (int n = m + 2; n <= Q; ++n) {
            double o = c_lodd[n], k = c_lka[n * kLT + m];
            cplx cp = o * (zi * bp) - k * (ir2 * ap);
            cplx cm = o * (zi * bm) - k * (ir2 * am);
            feed(n, m, cp);
            if (m > 0) feed(n, -m, cm);
            ap = bp; bp = cp;
            am = bm; bm = cm;
        }
    }
    g[0] = (up + um) * 0.5;
    g[1] = mk(0.5 * (up.im - um.im), -0.5 * (up.re - um.re));
    g[2] = uz;
}

// M2P with gradient by List-3 entries: 4 complex per point (u, grad).
__global__ __launch_bounds__(64) void k_l3d_m2p_part_grad(const int* __restrict__ owner,
                                                          const int64_t* __restrict__ poff4, TreeView tv,
                                                          PointsView pv, const cplx* __restrict__ mpole,
                                                          cplx* __restrict__ part)
{
    int e = blockIdx.x;
    int b = owner[e], a = tv.l3idx[e];
    int la = tv.level[a];
    double sa = tv.rs[la];
    cplx c[3];
    box_centre(tv, a, c);
    cplx* o = part + poff4[e];
    int p0 = tv.pbeg[b];
    for (int i = p0 + threadIdx.x; i < tv.pend[b]; i += blockDim.x) {
        cplx u, g[3];
        irr_sum_grad(point_rel(pv, i, c, sa), tv.P[la], mpole + tv.eoff[a], u, g);
        cplx* oi = o + 4 * (i - p0);
        oi[0] = sa * u;
        for (int k = 0; k < 3; ++k) oi[1 + k] = (sa * sa) * g[k];
    }
}

// L2P with gradient plus the List-3 parts: ufar[i] and gfar[3 i + k].
__global__ __launch_bounds__(64) void k_l3d_leaf_far_grad(const int* __restrict__ leaves, int top, TreeView tv,
                                                          PointsView pv, const cplx* __restrict__ local,
                                                          const int64_t* __restrict__ poff4,
                                                          const cplx* __restrict__ part, cplx* __restrict__ ufar,
                                                          cplx* __restrict__ gfar)
{
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    int p0 = tv.pbeg[b];
    for (int i = p0 + threadIdx.x; i < tv.pend[b]; i += blockDim.x) {
        cplx u = mk(0.0, 0.0), g[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
        if (l >= top) {
            int P = tv.P[l];
            double s = tv.rs[l];
            cplx c[3];
            box_centre(tv, b, c);
            reg_sum_grad(point_rel(pv, i, c, s), P, local + tv.eoff[b], u, g);
            u = s * u;
            for (int k = 0; k < 3; ++k) g[k] = (s * s) * g[k];
            for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) {
                const cplx* pe = part + poff4[e] + 4 * (i - p0);
                u += pe[0];
                for (int k = 0; k < 3; ++k) g[k] += pe[1 + k];
            }
        }
        ufar[i] = u;
        for (int k = 0; k < 3; ++k) gfar[3 * (int64_t)i + k] = g[k];
    }
}

// Near field of the layer potentials, by target leaf (owner computes; no
// symmetric pairs: the dipole and gradient kernels are not symmetric).  Per
// pair, d = x - y, r the principal root, 1/r from the reciprocal square root:
//   u += sigma / r + (v.d) / r^3
//   grad u += -sigma d / r^3 + v / r^3 - 3 (v.d) d / r^5
// (times 1/(4 pi) in the final write, with the far field).
__global__ __launch_bounds__(64) void k_l3d_near_layer(const int* __restrict__ leaves, TreeView tv, PointsView pv,
                                                       const double* __restrict__ dre,
                                                       const double* __restrict__ dim, int has_dip,
                                                       const cplx* __restrict__ ufar,
                                                       const cplx* __restrict__ gfar, IoMap io,
                                                       double* __restrict__ pot, double* __restrict__ grad)
{
    __shared__ double sx[3][64], sxi[3][64], ssr[64], ssi[64], sv[3][64], svi[3][64];
    int b = leaves[blockIdx.x];
    int64_t n = pv.n;
    int t = threadIdx.x;
    int p0 = tv.pbeg[b], p1 = tv.pend[b];
    const double k4 = 1.0 / (4.0 * kPi);
    for (int i0 = p0; i0 < p1; i0 += 64) {
        int i = i0 + t;
        bool tok = i < p1;
        double xr[3] = {0, 0, 0}, xi[3] = {0, 0, 0};
        if (tok)
            for (int d = 0; d < 3; ++d) { xr[d] = pv.xre[d * n + i]; xi[d] = pv.xim[d * n + i]; }
        cplx u = mk(0.0, 0.0), g[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
        for (int e = tv.l1off[b]; e < tv.l1off[b + 1]; ++e) {
            int a = tv.l1idx[e];
            for (int j0 = tv.pbeg[a]; j0 < tv.pend[a]; j0 += 64) {
                int cnt = min(64, tv.pend[a] - j0);
                __syncthreads();
                if (t < cnt) {
                    int j = j0 + t;
                    for (int d = 0; d < 3; ++d) {
                        sx[d][t] = pv.xre[d * n + j];
                        sxi[d][t] = pv.xim[d * n + j];
                        sv[d][t] = has_dip ? dre[d * n + j] : 0.0;
                        svi[d][t] = has_dip ? dim[d * n + j] : 0.0;
                    }
                    ssr[t] = pv.sre[j];
                    ssi[t] = pv.sim[j];
                }
                __syncthreads();
                if (!tok) continue;
                for (int q = 0; q < cnt; ++q) {
                    if (j0 + q == i) continue;
                    cplx dd[3];
                    cplx s2 = mk(0.0, 0.0);
                    for (int d = 0; d < 3; ++d) {
                        dd[d] = mk(xr[d] - sx[d][q], xi[d] - sxi[d][q]);
                        s2 += dd[d] * dd[d];
                    }
                    if (s2.re == 0.0 && s2.im == 0.0) continue;
                    cplx ir = cinv(csqrt_p(s2));
                    cplx ir2 = ir * ir, ir3 = ir2 * ir;
                    cplx sig = mk(ssr[q], ssi[q]);
                    cplx v[3] = {mk(sv[0][q], svi[0][q]), mk(sv[1][q], svi[1][q]), mk(sv[2][q], svi[2][q])};
                    cplx vd = v[0] * dd[0] + v[1] * dd[1] + v[2] * dd[2];
                    u += sig * ir + vd * ir3;
                    cplx a = sig * ir3 + 3.0 * (vd * ir3 * ir2);
                    for (int d = 0; d < 3; ++d) g[d] += v[d] * ir3 - a * dd[d];
                }
            }
        }
        if (!tok) continue;
        int64_t pidx = (int64_t)io.perm[i] - io.obase;
        if (pidx < 0) continue;
        u = (u + ufar[i]) * k4;
        bool bad = false;
        if (pot) {
            pot[2 * pidx] = u.re;
            pot[2 * pidx + 1] = u.im;
            bad = !isfinite(u.re) || !isfinite(u.im);
        }
        if (grad)
            for (int d = 0; d < 3; ++d) {
                cplx gd = (g[d] + gfar[3 * (int64_t)i + d]) * k4;
                bad = bad || !isfinite(gd.re) || !isfinite(gd.im);
                grad[2 * (3 * pidx + d)] = gd.re;
                grad[2 * (3 * pidx + d) + 1] = gd.im;
            }
        if (bad) atomicOr(io.nonfinite, 1);
    }
}

// dipole vectors into sorted order, SoA [3][n] (zero at target-only points)
__global__ void k_gather_dipole(const double* __restrict__ dip, IoMap io, int64_t n, double* __restrict__ dre,
                                double* __restrict__ dim)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t p = io.perm[i];
    bool src = dip && p < io.nsrc;
    for (int d = 0; d < 3; ++d) {
        dre[d * n + i] = src ? dip[2 * (3 * p + d)] : 0.0;
        dim[d * n + i] = src ? dip[2 * (3 * p + d) + 1] : 0.0;
    }
}

// ---------------------------------------------------------------- launchers
static size_t lds_bytes(int nelem) { return (size_t)nelem * sizeof(cplx); }

static size_t p2x_pair_lds(int P)
{
    int NL = 2 * ((P + 1) / 2) + 1;
    return lds_bytes(5 * kP2XPairChunk + (kP2XPairThreads / 64) * (P + 1) * (P + 1)) +
           (size_t)NL * (P + 1) * 2 * sizeof(double);
}

static size_t p2x_lds(int P)
{
    int ncol = 2 * P + 1;
    return lds_bytes(4 * kP2XChunk + (kL3P2XThreads / ncol) * (P + 1) * ncol);
}

hipError_t l3d_p2m(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   cplx* mpole, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    if (P <= kP2XPairMaxP) k_l3d_p2x_r<false><<<nb, kP2XPairThreads, p2x_pair_lds(P), st>>>(boxes, tv, pv, 0, mpole);
    else k_l3d_p2x<false><<<nb, kL3P2XThreads, p2x_lds(P), st>>>(boxes, tv, pv, 0, mpole);
    return hipGetLastError();
}

hipError_t l3d_p2l(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    if (P <= kP2XPairMaxP) k_l3d_p2x_r<true><<<nb, kP2XPairThreads, p2x_pair_lds(P), st>>>(boxes, tv, pv, 1, local);
    else k_l3d_p2x<true><<<nb, kL3P2XThreads, p2x_lds(P), st>>>(boxes, tv, pv, 1, local);
    return hipGetLastError();
}

hipError_t l3d_init_tables(int device)
{
    (void)device;
    static double rr[kLT * kLT], dg[kLT], odd[kLT], ka[kLT * kLT];
    for (int n = 0; n < kLT; ++n) {
        odd[n] = 2.0 * n - 1.0;
        dg[n] = n > 0 ? 0.5 / n : 0.0;
        for (int m = 0; m < kLT; ++m) {
            rr[n * kLT + m] = m < n ? 1.0 / ((double)(n + m) * (double)(n - m)) : 0.0;
            ka[n * kLT + m] = (double)(n + m - 1) * (double)(n - m - 1);
        }
    }
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_lrr), rr, sizeof(rr))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_ldg), dg, sizeof(dg))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_lodd), odd, sizeof(odd))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_lka), ka, sizeof(ka))) != hipSuccess) return e;
    // point-and-shoot tables, in extended precision: Wigner's
    //   d^n_{m m'}(pi/2) = 2^-n sqrt((n+m)!(n-m)!(n+m')!(n-m')!)
    //                      sum_k (-1)^(k-m'+m) / ((n+m'-k)! k! (n-k-m)! (k-m'+m)!)
    // (its cancellation costs about three digits at n = 15, which the 64-bit
    // mantissa absorbs), the coaxial factors and the scaling c_n^m
    static double ty[kPnsY], tz[(kPnsMaxP + 1) * (2 * kPnsMaxP + 1) * (kPnsMaxP + 1)],
        tc[(kPnsMaxP + 1) * (kPnsMaxP + 1)];
    long double fac[2 * kPnsMaxP + 2];
    fac[0] = 1.0L;
    for (int i = 1; i < 2 * kPnsMaxP + 2; ++i) fac[i] = fac[i - 1] * i;
    for (int n = 0; n <= kPnsMaxP; ++n)
        for (int m = -n; m <= n; ++m) {
            tc[n * n + n + m] = (double)sqrtl(fac[n - m] * fac[n + m]);
            for (int r = -n; r <= n; ++r) {
                // column m, row r: d^n_{r m}
                long double sum = 0.0L;
                for (int k = 0; k <= 2 * n; ++k) {
                    int a = n + m - k, c = n - k - r, d = k - m + r;
                    if (a < 0 || c < 0 || d < 0) continue;
                    long double term = 1.0L / (fac[a] * fac[k] * fac[c] * fac[d]);
                    sum += ((k - m + r) & 1) ? -term : term;
                }
                long double v = sum * sqrtl(fac[n + r] * fac[n - r] * fac[n + m] * fac[n - m]) / powl(2.0L, n);
                ty[pns_ybase(n) + (m + n) * (2 * n + 1) + (r + n)] = (double)v;
            }
        }
    for (int j = 0; j <= kPnsMaxP; ++j)
        for (int k = -kPnsMaxP; k <= kPnsMaxP; ++k)
            for (int i = 0; i <= kPnsMaxP; ++i) {
                int nn = (k < 0 ? -k : k) + i;
                double v = 0.0;
                if ((k < 0 ? -k : k) <= j && nn <= kPnsMaxP) {
                    long double z = fac[j + nn] / sqrtl(fac[j - k] * fac[j + k] * fac[nn - k] * fac[nn + k]);
                    v = (double)(((j + k) & 1) ? -z : z);
                }
                tz[(j * (2 * kPnsMaxP + 1) + k + kPnsMaxP) * (kPnsMaxP + 1) + i] = v;
            }
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_pns_y), ty, sizeof(ty))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_pns_z), tz, sizeof(tz))) != hipSuccess) return e;
    double tf[2 * kPnsMaxP + 1];
    for (int i = 0; i <= 2 * kPnsMaxP; ++i) tf[i] = (double)fac[i];
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_pns_fact), tf, sizeof(tf))) != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(g_pns_c), tc, sizeof(tc));
}

// children per LDS batch of the M2M and L2L: at most four, within 64 KiB
static int l3_shift_batch(int P)
{
    int nc = (P + 1) * (P + 1);
    return std::max(1, std::min(4, (int)(65536 / (2 * lds_bytes(nc)))));
}

hipError_t l3d_m2m(const int* boxes, int nb, int P, const TreeView& tv, cplx* mpole, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    int CB = l3_shift_batch(P);
    k_l3d_m2m<<<nb, 256, lds_bytes(2 * CB * (P + 1) * (P + 1)), st>>>(boxes, tv, CB, mpole);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_m2l(const int* boxes, int nb, size_t lds, const TreeView& tv, const int* map, int ntab,
                             const L3Pairs& pr, const cplx* mpole, cplx* local, int accum, hipStream_t st)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_l3d_m2l<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    k_l3d_m2l<R><<<nb, 64 * kM2LWaves, lds, st>>>(boxes, nb, tv, map, ntab, pr.c, pr.ps, pr.src, pr.rows64, mpole,
                                                  local, accum);
    return hipGetLastError();
}

// LDS of the M2L workgroup: the table, the source multipole and the row
// bases, or the partial sums of wavefronts 1..W-1 if those need more.
static size_t m2l_red_bytes(int R, int W)
{
    return (size_t)(W - 1) * R * 4 * 64 * sizeof(cplx);
}

static int m2l_groups_per_lane(int P)
{
    int G = 0;
    for (int j = 0; j <= P; ++j) G += j / 2 + 1;
    return (G + 63) / 64;
}

size_t l3d_m2l_lds(int P, int ntab)
{
    size_t tab = (size_t)(ntab + kM2LPad) * sizeof(cplx) + (size_t)(2 * P + 1) * sizeof(int);
    return std::max(tab, m2l_red_bytes(m2l_groups_per_lane(P), kM2LWaves));
}

template <int R>
static hipError_t launch_m2l_f32(const int* boxes, int nb, size_t lds, const TreeView& tv, const int* map,
                                 int ntab, const L3Pairs& pr, const cplx* mpole, cplx* local, int accum,
                                 hipStream_t st)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_l3d_m2l_f32<R>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_l3d_m2l_f32<R><<<nb, 64 * kM2LWavesF32, lds, st>>>(boxes, nb, tv, map, ntab, pr.c, pr.ps, pr.src,
                                                         pr.rows32, mpole, local, accum);
    return hipGetLastError();
}

hipError_t l3d_m2l_pairs(const int* boxes, int nb, const TreeView& tv, const L3PairP& pp, cplx* c, int* ps,
                         int* src, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_l3d_m2l_pairs<<<nb, 64, 0, st>>>(boxes, tv, pp, c, ps, src);
    return hipGetLastError();
}

hipError_t l3d_m2l(const int* boxes, int nb, int P, const TreeView& tv, const int* map, int ntab, int R,
                   const L3Pairs& pr, int mixed, int accum, const cplx* mpole, cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    if (mixed && P <= kM2LF32MaxP) {
        size_t lds = std::max((size_t)(ntab + kM2LPad + (P + 1) * (P + 1)) * sizeof(float2) +
                                  (size_t)(2 * P + 1) * sizeof(int),
                              m2l_red_bytes(R, kM2LWavesF32));
        switch (R) {
        case 1: return launch_m2l_f32<1>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
        case 2: return launch_m2l_f32<2>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
        default: return hipErrorInvalidValue;
        }
    }
    size_t lds = l3d_m2l_lds(P, ntab);
    switch (R) {
    case 1: return launch_m2l<1>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
    case 2: return launch_m2l<2>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
    case 3: return launch_m2l<3>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
    case 4: return launch_m2l<4>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
    case 5: return launch_m2l<5>(boxes, nb, lds, tv, map, ntab, pr, mpole, local, accum, st);
    default: return hipErrorInvalidValue;
    }
}

int l3d_pns_max_p() { return kPnsMaxP; }

hipError_t l3d_m2l_pns(const int* boxes, int nb, int P, const TreeView& tv, const cplx* pc, const int* off,
                       const int4* ent, const cplx* mpole, cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    if (P > kPnsMaxP) return hipErrorInvalidValue;
    if (P <= 10) k_l3d_m2l_pns<10><<<nb, pns_threads<10>(), 0, st>>>(boxes, nb, tv, pc, off, ent, mpole, local);
    else if (P <= 12) k_l3d_m2l_pns<12><<<nb, pns_threads<12>(), 0, st>>>(boxes, nb, tv, pc, off, ent, mpole, local);
    else if (P <= 14) k_l3d_m2l_pns<14><<<nb, pns_threads<14>(), 0, st>>>(boxes, nb, tv, pc, off, ent, mpole, local);
    else k_l3d_m2l_pns<15><<<nb, pns_threads<15>(), 0, st>>>(boxes, nb, tv, pc, off, ent, mpole, local);
    return hipGetLastError();
}

hipError_t l3d_l2l(const int* parents, int nb, int P, const TreeView& tv, cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    int CB = l3_shift_batch(P);
    k_l3d_l2l<<<nb, 256, lds_bytes((1 + CB) * (P + 1) * (P + 1)), st>>>(parents, tv, CB, local);
    return hipGetLastError();
}

hipError_t l3d_leaf_far(const int* leaves, int nleaf, int top, const TreeView& tv,
                        const PointsView& pv, const cplx* mpole, const cplx* local, const M2PParts& m2p,
                        cplx* ufar, hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    if (m2p.n > 0) {
        k_l3d_m2p_part<<<m2p.n, 64, 0, st>>>(m2p.owner, m2p.poff, tv, pv, mpole, m2p.part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_l3d_leaf_far<<<nleaf, 64, 0, st>>>(leaves, top, tv, pv, local, m2p.poff, m2p.part, ufar);
    return hipGetLastError();
}


// Largest P the kernels take: at most 5 output groups per M2L lane (P <= 31),
// 4 outputs per thread of the 256-thread M2M/L2L workgroups ((P+1)^2 <= 1024),
// and the M2L table within one workgroup's share of the CU's LDS.
int l3d_m2l_waves(int fp32) { return fp32 ? kM2LWavesF32 : kM2LWaves; }

int l3d_pmax_supported()
{
    int dev = 0, lds = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
            v > lds)
            lds = v;
    }
    int P = 31;
    while (P > 1 && (l3d_m2l_layout(P).R > 5 || l3d_m2l_lds(P, l3d_m2l_layout(P).entries) > (size_t)lds)) --P;
    return P;
}

static size_t p2x_dip_lds(int P, int threads)
{
    int ncol = 2 * P + 1, H = threads / ncol;
    return lds_bytes(7 * kP2XChunk + 4 * (size_t)H * (P + 2) * ncol);
}

static int p2x_dip_threads(int P)
{
    int ncol = 2 * P + 1;
    return ((ncol + 63) / 64) * 64;      // one point stream per 64-lane multiple
}

hipError_t l3d_p2x_dip(const int* boxes, int nb, int P, int irregular, const TreeView& tv, const PointsView& pv,
                       const double* dre, const double* dim, cplx* out, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    int th = p2x_dip_threads(P);
    size_t lds = p2x_dip_lds(P, th);
    const void* f = irregular ? (const void*)k_l3d_p2x_dip<true> : (const void*)k_l3d_p2x_dip<false>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (irregular) k_l3d_p2x_dip<true><<<nb, th, lds, st>>>(boxes, tv, pv, dre, dim, 1, out);
    else k_l3d_p2x_dip<false><<<nb, th, lds, st>>>(boxes, tv, pv, dre, dim, 0, out);
    return hipGetLastError();
}

hipError_t l3d_leaf_far_grad(const int* leaves, int nleaf, int top, const TreeView& tv, const PointsView& pv,
                             const cplx* mpole, const cplx* local, const M2PParts& m2p4, cplx* ufar, cplx* gfar,
                             hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    if (m2p4.n > 0) {
        k_l3d_m2p_part_grad<<<m2p4.n, 64, 0, st>>>(m2p4.owner, m2p4.poff, tv, pv, mpole, m2p4.part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_l3d_leaf_far_grad<<<nleaf, 64, 0, st>>>(leaves, top, tv, pv, local, m2p4.poff, m2p4.part, ufar, gfar);
    return hipGetLastError();
}

hipError_t l3d_near_layer(const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv, const double* dre,
                          const double* dim, int has_dip, const cplx* ufar, const cplx* gfar, const IoMap& io,
                          double* pot, double* grad, hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    k_l3d_near_layer<<<nleaf, 64, 0, st>>>(leaves, tv, pv, dre, dim, has_dip, ufar, gfar, io, pot, grad);
    return hipGetLastError();
}

hipError_t launch_gather_dipole(const double* dip, const IoMap& io, int64_t n, double* dre, double* dim,
                                hipStream_t st)
{
    k_gather_dipole<<<(int)((n + 255) / 256), 256, 0, st>>>(dip, io, n, dre, dim);
    return hipGetLastError();
}

}  // namespace cfmm
