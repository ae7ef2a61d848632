// 3D Helmholtz complex-coordinate FMM kernels (Sec. 5.3 and the multilevel
// steps of Sec. 6.4).
//
// Expansions use Schmidt-normalised solid harmonics S_n^m(x) = rho^n Y_n^m,
// evaluated by their Cartesian column recurrences at complex points
// (w = x + iy for m >= 0, x - iy for m < 0, c_m = prod_k sqrt((2k-1)/(2k))):
//   S_|m|^m = c_|m| w^|m|,
//   S_n^m = ((2n-1) z S_{n-1}^m - sqrt((n+|m|-1)(n-|m|-1)) r2 S_{n-2}^m) / sqrt((n-|m|)(n+|m|)),
// so that P_n(cos g) = sum_m Y_n^m(x) Y_n^-m(y) and
//   h_0(k|X - Y|) = sum_n (2n+1) j_n(k rho_Y) h_n(k rho_X) sum_m Y_n^-m(Y) Y_n^m(X).
// With box width w, kw = kappa w and the level scale sc = min(1, kw), in
// coordinates scaled by 1/w:
//   A_n(x) = j_n(kw rho) / (sc rho)^n     (entire in rho^2 = x.x)
//   B_n(x) = h_n(kw rho) sc^n / rho^n     (principal rho)
//   P2M  Mhat_n^m = (2n+1) sum sigma A_n(y) S_n^-m(y),   u = (i kappa / 4pi) sum Mhat B_n(x) S_n^m(x)
//   P2L  Lhat_n^m = (2n+1) sum sigma B_n(y) S_n^-m(y),   u = (i kappa / 4pi) sum Lhat A_n(x) S_n^m(x).
//
// Translations (M2M, M2L, L2L) follow the point-and-shoot scheme of Sec. 5.2
// and Sec. 5.3: rotate the source expansion so that the offset D lies on the
// z axis, translate coaxially, rotate back.  Both steps are done by sampling
// and projection:
//  * rotation: a complex orthogonal Q (Q Q^T = I) with Q e_z = D / rho_D; the
//    degree-n part f_n = sum_m a_n^m S_n^m is sampled at Q y_j on the equator
//    y_j = (cos phi_j, sin phi_j, 0), phi_j = 2 pi j / (2P+1), together with its
//    derivative along -Q e_z (the polar derivative), and a DFT over j returns the
//    rotated coefficients (divided by S_n^m(e_x) when n+m is even, by its polar
//    derivative when n+m is odd);
//  * coaxial translation: the rotated source field is sampled, per azimuthal
//    order m, at Gauss-Legendre nodes of a sphere of radius rs about the new
//    centre, together with its radial derivative, and projected on the
//    associated Legendre functions; T_n and T'_n (the target radial function and
//    its derivative at rs) combine the two by least squares, so no zero of
//    j_n ends the translation.
// Every pair of a level runs the same seven batched kernels (geometry, rotate
// sample, DFT, radial, coaxial sample, projection, rotate back, accumulate)
// over a scratch region, and each target box sums its pairs in a fixed order.
#include "common.hpp"
#include "kernels.hpp"

namespace cfmm {

namespace {

constexpr int kT = kPMaxH3 + 3;       // recurrence tables cover n <= kPMaxH3 + 2
// Column recurrence constants by column, entry [m * kT + n] for n > m:
// s = (2n-1) b and a = sqrt((n+m-1)(n-m-1)) b with b = 1/sqrt((n-m)(n+m)),
// so that Q_n = s z Q_{n-1} - a r2 Q_{n-2}.  A column's entries are
// contiguous, so a few steps' constants come in one scalar load.
struct alignas(16) RecAB {
    double s, a;
};
struct alignas(8) RecABf {
    float s, a;
};
__constant__ RecAB c_rab[kT * kT];
__constant__ RecABf c_rabf[kT * kT];  // the same table rounded to FP32
template <class T>
struct RecOf {
    typedef RecAB type;
};
template <>
struct RecOf<float> {
    typedef RecABf type;
};
// Device addresses of the two tables per device, taken once at set-up and
// passed to the kernels as arguments (an argument pointer stays in scalar
// registers; the symbol's address would be reloaded through the GOT).
constexpr int kMaxDev = 64;
const void* g_rab[kMaxDev];
const void* g_rabf[kMaxDev];
__constant__ double c_cs[kT];         // c_m = prod_{k<=m} sqrt((2k-1)/(2k))
__constant__ double c_ck[kT];         // sqrt((2m-1)/(2m))

__device__ inline int hnm(int n, int m) { return n * n + n + m; }
__device__ inline int tri(int n, int m) { return n * (n + 1) / 2 + m; }

struct V3 {
    cplx x, y, z;
};

__device__ inline cplx dot(const V3& a, const V3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// One column step: (q0, q1) = (Q_{n-2}, Q_{n-1}) -> Q_n, with its derivative
// along a direction where z' = dz and (r2)' = dr2.
__device__ inline void col_step(const RecAB* col, int n, cplx z, cplx dz, cplx r2, cplx dr2, cplx& q0, cplx& q1,
                                cplx& dq0, cplx& dq1)
{
    RecAB c = col[n];
    cplx q2 = c.s * (z * q1) - c.a * (r2 * q0);
    cplx dq2 = c.s * (dz * q1 + z * dq1) - c.a * (dr2 * q0 + r2 * dq0);
    q0 = q1; q1 = q2; dq0 = dq1; dq1 = dq2;
}

__device__ inline void col_step_nd(const RecAB* col, int n, cplx z, cplx r2, cplx& q0, cplx& q1)
{
    RecAB c = col[n];
    cplx q2 = c.s * (z * q1) - c.a * (r2 * q0);
    q0 = q1; q1 = q2;
}

// Radial functions, written to out[n * stride] for n = 0..N.
// A_n = j_n(kw rho) / (sc rho)^n: power series at the two top orders and
// downward recurrence A_{n-1} = (2n+1)(sc/kw) A_n - sc^2 rho^2 A_{n+1} while
// |z|^2 < 2(2N + 5); otherwise Miller's backward recurrence for j_n(z),
// normalised on j_0 and j_1 by least squares, then divided by (sc rho)^n.
__device__ void radial_j(cplx rho2, double kw, double sc, int N, cplx* out, int stride)
{
    cplx z2 = (kw * kw) * rho2;
    if (cabs1(z2) < 2.0 * (2.0 * N + 5.0)) {
        auto series = [&](int n) {
            double pref = 1.0, g = kw / sc;
            for (int i = 1; i <= n; ++i) pref *= g / (2.0 * i + 1.0);
            cplx term = mk(1.0, 0.0), sum = mk(1.0, 0.0), q = -0.5 * z2;
            for (int k = 1; k < 400; ++k) {
                term = term * q * (1.0 / ((double)k * (2.0 * n + 2.0 * k + 1.0)));
                sum += term;
                if (cabs2(term) < 1e-36 * cabs2(sum)) break;
            }
            return pref * sum;
        };
        cplx aN = series(N);
        out[N * stride] = aN;
        if (N == 0) return;
        cplx aN1 = series(N - 1);
        out[(N - 1) * stride] = aN1;
        cplx s2r2 = (sc * sc) * rho2;
        double g = sc / kw;
        cplx hi = aN, mid = aN1;
        for (int n = N - 1; n >= 1; --n) {
            cplx lo = ((2.0 * n + 1.0) * g) * mid - s2r2 * hi;
            out[(n - 1) * stride] = lo;
            hi = mid;
            mid = lo;
        }
        return;
    }
    cplx rho = csqrt_p(rho2);
    cplx z = kw * rho;
    cplx iz = cinv(z);
    int start = N + 24 + (int)cabs1(z);
    cplx t1 = mk(0.0, 0.0), t0 = mk(1e-30, 0.0);   // t_{n+1}, t_n at n = start
    for (int n = start; n >= 1; --n) {
        cplx tm = ((2.0 * n + 1.0) * iz) * t0 - t1;   // t_{n-1}
        t1 = t0;
        t0 = tm;
        if (n - 1 <= N) out[(n - 1) * stride] = tm;
        if (cabs2(tm) > 1e200) {
            t0 *= 1e-150; t1 *= 1e-150;
            for (int k = n - 1; k <= N; ++k) out[k * stride] *= 1e-150;
        }
    }
    cplx sz, cz;
    {
        // sin z, cos z for complex z
        double s, c;
        sincos_cw(z.re, &s, &c);
        double eh = exp_cw(z.im), ehm = exp_cw(-z.im);
        double ch = 0.5 * (eh + ehm), sh = 0.5 * (eh - ehm);
        sz = mk(s * ch, c * sh);
        cz = mk(c * ch, -s * sh);
    }
    cplx j0 = sz * iz, j1 = (sz * iz - cz) * iz;
    cplx m0 = out[0], m1 = (N >= 1) ? out[stride] : t1;
    double nrm = fmax(cabs1(m0), cabs1(m1));
    cplx a0 = m0 * (1.0 / nrm), a1 = m1 * (1.0 / nrm);
    cplx s = cdiv(j0 * conj(a0) + j1 * conj(a1), mk(cabs2(a0) + cabs2(a1), 0.0)) * (1.0 / nrm);
    cplx f = s, step = cinv(sc * rho);
    for (int n = 0; n <= N; ++n) {
        out[n * stride] = out[n * stride] * f;
        f = f * step;
    }
}

// B_n = h_n(kw rho) sc^n / rho^n for n = 0..N.  Forward recurrence
// B_{n+1} = (2n+1)(sc/kw) B_n / rho^2 - sc^2 B_{n-1} / rho^2 from
// h_0 = -i e^{iz}/z, h_1 = -e^{iz}(z + i)/z^2 when Im z >= -1; below, the
// reflection h_n(z) = 2 j_n(z) - conj(h_n(conj z)), whose second term recurs
// forward stably.
__device__ void radial_h_fwd(cplx rho, double kw, double sc, int N, cplx* out, int stride, bool accumulate_conj)
{
    cplx z = kw * rho;
    cplx iz = cinv(z);
    cplx e = cexp_cw(times_i(z));
    cplx h0 = times_i(e * iz) * -1.0;                   // -i e^{iz} / z
    cplx h1 = -(e * (z + mk(0.0, 1.0)) * iz * iz);      // -e^{iz}(z+i)/z^2
    cplx ir2 = cinv(rho * rho);
    cplx b0 = h0, b1 = h1 * sc * cinv(rho);
    auto put = [&](int n, cplx v) {
        if (accumulate_conj) out[n * stride] = out[n * stride] - conj(v);
        else out[n * stride] = v;
    };
    put(0, b0);
    if (N == 0) return;
    put(1, b1);
    double g = sc / kw;
    for (int n = 1; n < N; ++n) {
        cplx b2 = ((2.0 * n + 1.0) * g) * (b1 * ir2) - (sc * sc) * (b0 * ir2);
        put(n + 1, b2);
        b0 = b1;
        b1 = b2;
    }
}

__device__ void radial_h(cplx rho2, double kw, double sc, int N, cplx* out, int stride)
{
    cplx rho = csqrt_p(rho2);
    cplx z = kw * rho;
    if (z.im >= -1.0) {
        radial_h_fwd(rho, kw, sc, N, out, stride, false);
        return;
    }
    // B_n(rho) = 2 sc^{2n} A_n(rho) - conj(B_n(conj rho))
    radial_j(rho2, kw, sc, N, out, stride);
    double f = 2.0;
    for (int n = 0; n <= N; ++n) {
        out[n * stride] = out[n * stride] * f;
        f *= sc * sc;
    }
    radial_h_fwd(conj(rho), kw, sc, N, out, stride, true);
}

// ------------------------------------------------------------------ P2M / P2L
// One workgroup per box; the 2P+1 output orders are repeated over S slices of
// the threads (S = blockDim / (2P+1), so that small P still fills the lanes):
// thread (slice s, order m) sweeps the points q = s, s + S, ... of each chunk
// of kPC points of the box (or of its List-4 boxes), whose radial values the
// first kPC threads compute into LDS, into its slice's accumulators; the
// slices are added in order at the end.
constexpr int kPC = 32;

template <bool IRREG>
__global__ __launch_bounds__(128) void k_h3d_p2x(const int* __restrict__ boxes, TreeView tv, PointsView pv,
                                                 H3DLevels hl, int useL4, cplx* __restrict__ out)
{
    extern __shared__ cplx lds[];
    const RecAB* rec = static_cast<const RecAB*>(hl.rec);
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    double iw = tv.rs[l], kw = hl.kw[l], sc = hl.sc[l];
    int W2 = 2 * P + 1, S = blockDim.x / W2;
    int st = S * W2;                               // accumulator row: [slice][order]
    cplx* acc = lds;                               // [(P+1)][st]
    cplx* rad = acc + (size_t)(P + 1) * st;        // [(P+2)][kPC]
    cplx* py = rad + (size_t)(P + 2) * kPC;        // [kPC][3]
    cplx* ps = py + 3 * kPC;                       // [kPC]
    int t = threadIdx.x, sl = t / W2, mm = t - sl * W2 - P;
    bool act = sl < S;
    int am = mm < 0 ? -mm : mm;
    if (act)
        for (int n = am; n <= P; ++n) acc[n * st + t] = mk(0.0, 0.0);
    cplx c[3];
    int nb = tv.nbox;
    for (int d = 0; d < 3; ++d) c[d] = mk(tv.cre[d * nb + b], tv.cim[d * nb + b]);
    int64_t n = pv.n;
    int e0 = useL4 ? tv.l4off[b] : 0, e1 = useL4 ? tv.l4off[b + 1] : 1;
    for (int e = e0; e < e1; ++e) {
        int src = useL4 ? tv.l4idx[e] : b;
        for (int j0 = tv.pbeg[src]; j0 < tv.pend[src]; j0 += kPC) {
            int cnt = min(kPC, tv.pend[src] - j0);
            __syncthreads();
            if (t < cnt) {
                int j = j0 + t;
                cplx y[3];
                for (int d = 0; d < 3; ++d)
                    y[d] = mk((pv.xre[d * n + j] - c[d].re) * iw, (pv.xim[d * n + j] - c[d].im) * iw);
                for (int d = 0; d < 3; ++d) py[3 * t + d] = y[d];
                ps[t] = mk(pv.sre[j], pv.sim[j]);
                cplx r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
                if (IRREG) radial_h(r2, kw, sc, P, rad + t, kPC);
                else radial_j(r2, kw, sc, P, rad + t, kPC);
            }
            __syncthreads();
            if (!act) continue;
            // order o = -mm of the source side
            int o = -mm;
            for (int q = sl; q < cnt; q += S) {
                cplx x = py[3 * q], yv = py[3 * q + 1], z = py[3 * q + 2];
                cplx w = o >= 0 ? mk(x.re - yv.im, x.im + yv.re) : mk(x.re + yv.im, x.im - yv.re);
                cplx r2 = x * x + yv * yv + z * z;
                cplx D = mk(c_cs[am], 0.0);
                for (int k = 0; k < am; ++k) D = D * w;
                D = D * ps[q];
                cplx q0 = mk(0.0, 0.0), q1 = mk(1.0, 0.0);
                acc[am * st + t] += D * rad[am * kPC + q];
                for (int nn = am + 1; nn <= P; ++nn) {
                    col_step_nd(rec + am * kT, nn, z, r2, q0, q1);
                    acc[nn * st + t] += (D * q1) * rad[nn * kPC + q];
                }
            }
        }
    }
    __syncthreads();
    if (act && sl == 0) {
        cplx* o = out + tv.eoff[b];
        for (int nn = am; nn <= P; ++nn) {
            cplx a = acc[nn * st + t];
            for (int k = 1; k < S; ++k) a += acc[nn * st + k * W2 + t];
            cplx v = (2.0 * nn + 1.0) * a;
            if (useL4) o[hnm(nn, mm)] += v;
            else o[hnm(nn, mm)] = v;
        }
    }
}

// ------------------------------------------------------------------ L2P + M2P
// Expansion of box a (its local expansion when loc, else its multipole) at
// point i; `my` is the calling thread's LDS column (stride 64) for the radial
// values.
__device__ inline cplx h3d_eval_point(int i, int a, bool loc, const TreeView& tv, const PointsView& pv,
                                      const H3DLevels& hl, const cplx* __restrict__ coef, cplx* my)
{
    const RecAB* rec = static_cast<const RecAB*>(hl.rec);
    int64_t n = pv.n;
    int nb = tv.nbox;
    int la = tv.level[a];
    int P = tv.P[la];
    double iw = tv.rs[la];
    cplx x[3];
    for (int d = 0; d < 3; ++d)
        x[d] = mk((pv.xre[d * n + i] - tv.cre[d * nb + a]) * iw, (pv.xim[d * n + i] - tv.cim[d * nb + a]) * iw);
    cplx r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    if (loc) radial_j(r2, hl.kw[la], hl.sc[la], P, my, 64);
    else radial_h(r2, hl.kw[la], hl.sc[la], P, my, 64);
    const cplx* C = coef + tv.eoff[a];
    cplx wp = mk(x[0].re - x[1].im, x[0].im + x[1].re);
    cplx wm = mk(x[0].re + x[1].im, x[0].im - x[1].re);
    cplx Dp = mk(1.0, 0.0), Dm = mk(1.0, 0.0), u = mk(0.0, 0.0);
    for (int am = 0; am <= P; ++am) {
        if (am > 0) {
            Dp = Dp * wp * c_ck[am];
            Dm = Dm * wm * c_ck[am];
        }
        for (int sgn = 0; sgn < (am ? 2 : 1); ++sgn) {
            int m = sgn ? -am : am;
            cplx D = sgn ? Dm : Dp;
            cplx q0 = mk(0.0, 0.0), q1 = mk(1.0, 0.0);
            cplx s = C[hnm(am, m)] * my[am * 64];
            for (int nn = am + 1; nn <= P; ++nn) {
                col_step_nd(rec + am * kT, nn, x[2], r2, q0, q1);
                s += (C[hnm(nn, m)] * q1) * my[nn * 64];
            }
            u += D * s;
        }
    }
    return u;
}

// M2P by List-3 entries: entry e = (leaf owner[e], box l3idx[e]), one
// wavefront per entry, into part[poff[e] + i - pbeg].
__global__ __launch_bounds__(64) void k_h3d_m2p_part(const int* __restrict__ owner,
                                                     const int64_t* __restrict__ poff, TreeView tv,
                                                     PointsView pv, H3DLevels hl,
                                                     const cplx* __restrict__ mpole, cplx* __restrict__ part)
{
    extern __shared__ cplx rad[];   // [(pmax+2)][64]
    int e = blockIdx.x;
    int b = owner[e], a = tv.l3idx[e];
    cplx* o = part + poff[e] - tv.pbeg[b];
    for (int i = tv.pbeg[b] + threadIdx.x; i < tv.pend[b]; i += 64)
        o[i] = h3d_eval_point(i, a, false, tv, pv, hl, mpole, rad + threadIdx.x);
}

// L2P, one wavefront per leaf and one target per thread, plus the leaf's
// List-3 parts in list order.
__global__ __launch_bounds__(64) void k_h3d_leaf_far(const int* __restrict__ leaves, int top, TreeView tv,
                                                     PointsView pv, H3DLevels hl,
                                                     const cplx* __restrict__ local,
                                                     const int64_t* __restrict__ poff,
                                                     const cplx* __restrict__ part, cplx* __restrict__ ufar)
{
    extern __shared__ cplx rad[];   // [(pmax+2)][64]
    int b = leaves[blockIdx.x];
    int l = tv.level[b];
    for (int i = tv.pbeg[b] + threadIdx.x; i < tv.pend[b]; i += 64) {
        cplx u = mk(0.0, 0.0);
        if (l >= top) {
            u = h3d_eval_point(i, b, true, tv, pv, hl, local, rad + threadIdx.x);
            for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) u += part[poff[e] + i - tv.pbeg[b]];
        }
        ufar[i] = u;
    }
}

// ------------------------------------------------------------------ translations
// K0: per pair, D = (c_dst - c_src) / w_src, rho_D = sqrt(D.D) and a complex
// orthogonal Q with third column u = D / rho_D, built by Gram-Schmidt in the
// bilinear form from the coordinate axis e_k with the smallest |u_k|:
// q1 = (e_k - u_k u) / sqrt(1 - u_k^2), q2 = u x q1, Q = [q1 q2 u].
__global__ void k_h3d_geo(H3DTr tr, TreeView tv)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tr.np) return;
    int s = tr.src[i], d = tr.dst[i], nb = tv.nbox;
    cplx D[3];
    for (int k = 0; k < 3; ++k)
        D[k] = mk((tv.cre[k * nb + d] - tv.cre[k * nb + s]) * tr.inv_w,
                  (tv.cim[k * nb + d] - tv.cim[k * nb + s]) * tr.inv_w);
    cplx rho = csqrt_p(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    cplx ir = cinv(rho);
    cplx u[3] = {D[0] * ir, D[1] * ir, D[2] * ir};
    // the axis k with the smallest |u_k|, selected without a run-time index
    // into the arrays (which would put them on the stack)
    double m0 = cabs2(u[0]), m1 = cabs2(u[1]), m2 = cabs2(u[2]);
    int k = m1 < m0 ? 1 : 0;
    if (m2 < (k ? m1 : m0)) k = 2;
    cplx uk = k == 0 ? u[0] : (k == 1 ? u[1] : u[2]);
    cplx q1[3];
    for (int q = 0; q < 3; ++q) q1[q] = -(uk * u[q]) + mk(q == k ? 1.0 : 0.0, 0.0);
    cplx nrm = cinv(csqrt_p(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2]));
    for (int q = 0; q < 3; ++q) q1[q] = q1[q] * nrm;
    cplx q2[3] = {u[1] * q1[2] - u[2] * q1[1], u[2] * q1[0] - u[0] * q1[2], u[0] * q1[1] - u[1] * q1[0]};
    cplx* g = tr.geo + (size_t)i * 10;
    for (int r = 0; r < 3; ++r) {
        g[3 * r + 0] = q1[r];
        g[3 * r + 1] = q2[r];
        g[3 * r + 2] = u[r];
    }
    g[9] = rho;
}

// K1a: coefficients of the polar derivative.  With v = -Q e_z (forward) or
// -Q^T e_z (back), the derivative of a degree-n field along v is a degree-(n-1)
// field: for the Schmidt harmonics
//   d_z S_n^m = sqrt((n-m)(n+m)) S_{n-1}^m,
//   (d_x + i d_y) S_n^m = -/+ sqrt((n-m)(n-m-1)) S_{n-1}^{m+1}   (- for m >= 0),
//   (d_x - i d_y) S_n^m = +/- sqrt((n+m)(n+m-1)) S_{n-1}^{m-1}   (+ for m > 0),
// and v.grad = v_z d_z + (v_x - i v_y)/2 (d_x + i d_y) + (v_x + i v_y)/2 (d_x - i d_y), so
// G_n = sum_m a_n^m v.grad S_n^m = sum_m' t_{n-1}^m' S_{n-1}^m' with
//   t_{n-1}^m' = v_z al(n,m') a_n^m' + (v_x - i v_y)/2 be(n,m'-1) a_n^{m'-1}
//              + (v_x + i v_y)/2 ga(n,m'+1) a_n^{m'+1}.
// Thread (pair, coefficient (n-1, m')), n = 1..P; written to A, which is free
// until the DFT that follows the sampling.
__global__ void k_h3d_rot_prep(H3DTr tr, int back, const int* __restrict__ eoff, const cplx* __restrict__ coef)
{
    int P = back ? tr.Pt : tr.Ps;
    int nc = P * P;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)tr.np * nc) return;
    int c = (int)(gid % nc);
    int i = (int)(gid / nc);
    int np1 = (int)sqrt((double)c);
    while (np1 * np1 > c) --np1;
    while ((np1 + 1) * (np1 + 1) <= c) ++np1;
    int mp = c - np1 * np1 - np1, n = np1 + 1;
    const cplx* g = tr.geo + (size_t)i * 10;
    const cplx* a = back ? tr.B + (size_t)i * tr.sB : coef + eoff[tr.src[i]];
    cplx vx, vy, vz;
    if (!back) { vx = -g[2]; vy = -g[5]; vz = -g[8]; }
    else { vx = -g[6]; vy = -g[7]; vz = -g[8]; }
    cplx hm = 0.5 * mk(vx.re + vy.im, vx.im - vy.re);   // (v_x - i v_y) / 2
    cplx hp = 0.5 * mk(vx.re - vy.im, vx.im + vy.re);   // (v_x + i v_y) / 2
    double al = sqrt((double)(n - mp) * (double)(n + mp));
    int m1 = mp - 1, m2 = mp + 1;
    double be = (m1 < 0 ? 1.0 : -1.0) * sqrt((double)(n - m1) * (double)(n - m1 - 1));
    double ga = (m2 > 0 ? 1.0 : -1.0) * sqrt((double)(n + m2) * (double)(n + m2 - 1));
    cplx t = (vz * a[hnm(n, mp)]) * al + (hm * a[hnm(n, m1)]) * be + (hp * a[hnm(n, m2)]) * ga;
    tr.A[(size_t)i * tr.sA + c] = t;
}

// Complex arithmetic in the sampling type T (double, or float for the
// mixed-precision M2L stages).
template <class T>
struct cz {
    T re, im;
};
template <class T>
__device__ inline cz<T> czmul(cz<T> a, cz<T> b)
{
    return cz<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ inline void czfma(cz<T>& acc, cz<T> a, cz<T> b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
template <class T>
__device__ inline cz<T> tocz(cplx a)
{
    return cz<T>{(T)a.re, (T)a.im};
}

// K1: rotation samples.  Workgroup (n-block, group of U pairs), thread =
// (pair u of the group, node j): x = Q y_j (forward) or Q^T y_j (back);
// accumulates F_n(j) = sum_m a_n^m S_n^m(x) and, from the derivative
// coefficients t of K1a, G_n(j) = sum_m t_{n-1}^m S_{n-1}^m(x) for the n of
// its block, sweeping the columns m with the diagonal start kept
// incrementally and folded into the column.  Each pair's coefficients of the
// block (a_n^m for n = nlo-1..nhi, t_n^m for n < P, in the packed n^2 + n + m
// order) are staged in LDS first, so the sweep reads them at one LDS address
// per pair.  With J = 2P + 1 nodes a pair fills only part of a wavefront at
// small P; U pairs per workgroup keep the lanes busy.  On the unit sphere
// r2 = 1, and the column step is
//   q_n = ((2n-1) z q_{n-1} - sqrt((n+m-1)(n-m-1)) q_{n-2}) / sqrt((n-m)(n+m)).
// T is the arithmetic type of the sweep (the samples are stored in FP64).
// smax: LDS entries per pair and array (the largest block's count).
template <int NB, class T>
__global__ __launch_bounds__(256) void k_h3d_rot_sample(H3DTr tr, int back, const int* __restrict__ eoff,
                                                        const cplx* __restrict__ coef, int U, int smax)
{
    extern __shared__ double csraw[];
    cz<T>* cs = reinterpret_cast<cz<T>*>(csraw);
    typedef typename RecOf<T>::type RecT;
    const RecT* rec = static_cast<const RecT*>(sizeof(T) == 4 ? tr.recf : tr.rec);
    int P = back ? tr.Pt : tr.Ps;
    int J = 2 * P + 1;
    int wpb = (tr.np + U - 1) / U;            // workgroups per n-block
    int blk = blockIdx.x / wpb;
    int i0 = (blockIdx.x - blk * wpb) * U;
    int nlo = blk * NB, nhi = min(P, nlo + NB - 1);
    int n0 = nlo > 0 ? nlo - 1 : 0;
    int na = (nhi + 1) * (nhi + 1) - n0 * n0;            // a_n^m, n = n0..nhi
    int nt1 = min(nhi, P - 1) + 1;
    int nt = nt1 > n0 ? nt1 * nt1 - n0 * n0 : 0;         // t_n^m, n = n0..min(nhi, P-1)
    for (int e = threadIdx.x; e < U * na; e += blockDim.x) {
        int u = e / na, k = e - u * na;
        int iu = min(i0 + u, tr.np - 1);
        const cplx* a = back ? tr.B + (size_t)iu * tr.sB : coef + eoff[tr.src[iu]];
        cz<T>* cu = cs + (size_t)u * 2 * smax;
        cu[k] = tocz<T>(a[n0 * n0 + k]);
        if (k < nt) cu[smax + k] = tocz<T>(tr.A[(size_t)iu * tr.sA + n0 * n0 + k]);
    }
    __syncthreads();
    int u = threadIdx.x / J;
    if (u >= U) return;
    int j = threadIdx.x - u * J;
    int i = i0 + u;
    bool own = i < tr.np;                     // the group's tail repeats the last pair
    if (!own) i = tr.np - 1;
    const cplx* g = tr.geo + (size_t)i * 10;
    // ca[hnm(n, m) - n0^2] = a_n^m and ct[hnm(n, m) - n0^2] = t_n^m for the block's rows
    const cz<T>* ca = cs + (size_t)u * 2 * smax;
    const cz<T>* ct = ca + smax;
    int h0 = n0 * n0;
    cz<T> zero = {(T)0, (T)0};
    double sp, cp;
    sincospi(2.0 * j / J, &sp, &cp);
    // x = M y with y = (cp, sp, 0); M = Q or Q^T
    V3 x;
    if (!back) {
        x.x = cp * g[0] + sp * g[1]; x.y = cp * g[3] + sp * g[4]; x.z = cp * g[6] + sp * g[7];
    } else {
        x.x = cp * g[0] + sp * g[3]; x.y = cp * g[1] + sp * g[4]; x.z = cp * g[2] + sp * g[5];
    }
    cz<T> z = tocz<T>(x.z);
    cz<T> F[NB], G[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) { F[k] = zero; G[k] = zero; }
    for (int sgn = 0; sgn < 2; ++sgn) {
        cz<T> w = tocz<T>(sgn ? mk(x.x.re + x.y.im, x.x.im - x.y.re) : mk(x.x.re - x.y.im, x.x.im + x.y.re));
        cz<T> D = {(T)1, (T)0};
        for (int am = 0; am <= nhi; ++am) {
            if (am > 0) {
                D = czmul(D, w);
                D.re *= (T)c_ck[am];
                D.im *= (T)c_ck[am];
            }
            if (sgn && am == 0) continue;
            int m = sgn ? -am : am;
            cz<T> q0 = zero, q1 = D;
            int n = am;
            // (s, a) of column am at degree nn (r2 = 1 on the unit sphere)
            auto coef = [&](int nn, T& cs_, T& ca_) {
                RecT c = rec[am * kT + nn];
                cs_ = (T)c.s;
                ca_ = (T)c.a;
            };
            auto step = [&](T cs_, T ca_) {
                cz<T> zq = czmul(z, q1);
                cz<T> q2 = {cs_ * zq.re - ca_ * q0.re, cs_ * zq.im - ca_ * q0.im};
                q0 = q1;
                q1 = q2;
            };
            // advance to n = nlo - 1 when the column starts below the block,
            // four steps per batch of constants
            while (n + 4 <= nlo - 1) {
                T s0, a0, s1, a1, s2, a2, s3, a3;
                coef(n + 1, s0, a0);
                coef(n + 2, s1, a1);
                coef(n + 3, s2, a2);
                coef(n + 4, s3, a3);
                step(s0, a0);
                step(s1, a1);
                step(s2, a2);
                step(s3, a3);
                n += 4;
            }
            while (n < nlo - 1) {
                ++n;
                T s0, a0;
                coef(n, s0, a0);
                step(s0, a0);
            }
            // G of degree nlo takes the column at nlo - 1
            if (nlo >= 1 && n == nlo - 1) czfma(G[0], ct[hnm(n, m) - h0], q1);
            // the block's constants, loaded before the sweep
            T bs[NB], ba[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) coef(min(nlo + k, kT - 1), bs[k], ba[k]);
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                int nn = nlo + k;
                if (nn > nhi || nn < am) continue;
                if (nn > n) {
                    step(bs[k], ba[k]);
                    n = nn;
                }
                czfma(F[k], ca[hnm(nn, m) - h0], q1);
                if (k + 1 < NB && nn + 1 <= nhi) czfma(G[k + 1], ct[hnm(nn, m) - h0], q1);
            }
        }
    }
    if (!own) return;
    cplx* FG = tr.FG + (size_t)i * tr.sFG;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        int nn = nlo + k;
        if (nn > nhi) break;
        FG[(size_t)nn * J + j] = mk((double)F[k].re, (double)F[k].im);
        FG[(size_t)(P + 1) * J + (size_t)nn * J + j] = mk((double)G[k].re, (double)G[k].im);
    }
}

// K2: DFT over the samples.  Thread (pair, degree n, order |m|):
// b_n^m = (1/J) sum_j e^{-i m phi_j} F_n(j) / S_n^m(e_x)  (n+m even)
//       = (1/J) sum_j e^{-i m phi_j} G_n(j) / d_n^m        (n+m odd).
// Orders +m and -m read the same samples (n+m and n-m have one parity) and
// conjugate twiddles, so one pass over j gives both from four sums:
// with X = F or G and e^{i m phi_j} = c + i s,
//   sum X e^{-i m phi} = (Sa + Sb, Sd - Se),  sum X e^{+i m phi} = (Sa - Sb, Sd + Se),
//   Sa = sum Re X c, Sb = sum Im X s, Sd = sum Im X c, Se = sum Re X s.
__global__ void k_h3d_rot_dft(H3DTr tr, int back, const double* __restrict__ eq_p0,
                              const double* __restrict__ eq_d0)
{
    extern __shared__ double tw[];   // cos, sin of 2 pi k / J
    int P = back ? tr.Pt : tr.Ps;
    int J = 2 * P + 1;
    for (int k = threadIdx.x; k < J; k += blockDim.x) {
        double s, c;
        sincospi(2.0 * k / J, &s, &c);
        tw[2 * k] = c;
        tw[2 * k + 1] = s;
    }
    __syncthreads();
    int nt = (P + 1) * (P + 2) / 2;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)tr.np * nt) return;
    int c = (int)(gid % nt);
    int i = (int)(gid / nt);
    int n = (int)((sqrt(8.0 * c + 1.0) - 1.0) * 0.5);
    while (n * (n + 1) / 2 > c) --n;
    while ((n + 1) * (n + 2) / 2 <= c) ++n;
    int am = c - n * (n + 1) / 2;
    bool even = ((n + am) & 1) == 0;
    const cplx* FG = tr.FG + (size_t)i * tr.sFG + (even ? 0 : (size_t)(P + 1) * J) + (size_t)n * J;
    double sa = 0.0, sb = 0.0, sd = 0.0, se = 0.0;
    int k = 0;
#pragma unroll 4
    for (int j = 0; j < J; ++j) {
        double cr = tw[2 * k], ci = tw[2 * k + 1];   // e^{i am phi_j}
        cplx f = FG[j];
        sa = fma(f.re, cr, sa);
        sb = fma(f.im, ci, sb);
        sd = fma(f.im, cr, sd);
        se = fma(f.re, ci, se);
        k += am;
        if (k >= J) k -= J;
    }
    double inv = 1.0 / ((even ? eq_p0[tri(n, am)] : eq_d0[tri(n, am)]) * J);
    cplx* o = tr.A + (size_t)i * tr.sA;
    o[hnm(n, am)] = mk((sa + sb) * inv, (sd - se) * inv);
    if (am > 0) o[hnm(n, -am)] = mk((sa - sb) * inv, (sd + se) * inv);
}

// The same DFT with the samples of U pairs staged in LDS first (coalesced
// loads), for stages where (P+1)(P+2)/2 <= 256 and the samples fit: thread
// (pair u of the workgroup, degree n, order |m|).
__global__ __launch_bounds__(256) void k_h3d_rot_dft_lds(H3DTr tr, int back, const double* __restrict__ eq_p0,
                                                         const double* __restrict__ eq_d0, int U)
{
    extern __shared__ double sh[];
    int P = back ? tr.Pt : tr.Ps;
    int J = 2 * P + 1;
    double* tw = sh;                                      // cos, sin of 2 pi k / J
    cplx* fg = reinterpret_cast<cplx*>(sh + 2 * J + (J & 1 ? 2 : 0));
    int rowlen = 2 * (P + 1) * J;                         // F rows, then G rows
    int i0 = blockIdx.x * U;
    for (int k = threadIdx.x; k < J; k += blockDim.x) {
        double s, c;
        sincospi(2.0 * k / J, &s, &c);
        tw[2 * k] = c;
        tw[2 * k + 1] = s;
    }
    for (int e = threadIdx.x; e < U * rowlen; e += blockDim.x) {
        int u = e / rowlen, k = e - u * rowlen;
        fg[e] = tr.FG[(size_t)min(i0 + u, tr.np - 1) * tr.sFG + k];
    }
    __syncthreads();
    int nt = (P + 1) * (P + 2) / 2;
    int u = threadIdx.x / nt;
    int i = i0 + u;
    if (u >= U || i >= tr.np) return;
    int c = threadIdx.x - u * nt;
    int n = (int)((sqrt(8.0 * c + 1.0) - 1.0) * 0.5);
    while (n * (n + 1) / 2 > c) --n;
    while ((n + 1) * (n + 2) / 2 <= c) ++n;
    int am = c - n * (n + 1) / 2;
    bool even = ((n + am) & 1) == 0;
    const cplx* X = fg + (size_t)u * rowlen + (even ? 0 : (size_t)(P + 1) * J) + (size_t)n * J;
    double sa = 0.0, sb = 0.0, sd = 0.0, se = 0.0;
    int k = 0;
#pragma unroll 4
    for (int j = 0; j < J; ++j) {
        double cr = tw[2 * k], ci = tw[2 * k + 1];   // e^{i am phi_j}
        cplx f = X[j];
        sa = fma(f.re, cr, sa);
        sb = fma(f.im, ci, sb);
        sd = fma(f.im, cr, sd);
        se = fma(f.re, ci, se);
        k += am;
        if (k >= J) k -= J;
    }
    double inv = 1.0 / ((even ? eq_p0[tri(n, am)] : eq_d0[tri(n, am)]) * J);
    cplx* o = tr.A + (size_t)i * tr.sA;
    o[hnm(n, am)] = mk((sa + sb) * inv, (sd - se) * inv);
    if (am > 0) o[hnm(n, -am)] = mk((sa - sb) * inv, (sd + se) * inv);
}

// K3a: radial functions of the source expansion at the coaxial nodes
// x_j = (rs sin t_j, 0, rho_D + rs cos t_j) (source-scaled coordinates).
__global__ void k_h3d_coax_radial(H3DTr tr)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)tr.np * tr.nq) return;
    int j = (int)(gid % tr.nq);
    int i = (int)(gid / tr.nq);
    cplx t = tr.geo[(size_t)i * 10 + 9];
    cplx x1 = mk(tr.rs * tr.sth[j], 0.0);
    cplx x3 = t + mk(tr.rs * tr.cth[j], 0.0);
    cplx r2 = x1 * x1 + x3 * x3;
    cplx* R = tr.R + (size_t)i * tr.sR + j;
    if (tr.src_h) radial_h(r2, tr.ks, tr.sc, tr.Ps + 1, R, tr.nq);
    else radial_j(r2, tr.ks, tr.sc, tr.Ps + 1, R, tr.nq);
}

// K3: coaxial samples and their projection.  Workgroup (group of U pairs,
// order m >= 0), thread = (pair u of the group, node j): the column of order m
// at x_j (y = 0, so S_n^-m = S_n^m there) with its derivative along
// s_j = (sin t_j, 0, cos t_j); with F = R_n(rho) S_n^m(x),
//   dF/drs = fac R_{n+1} (s.x) S_n^m + R_n s.grad S_n^m,
// fac = -kw sc for the regular A_n and -kw / sc for the singular B_n.  Each
// pair's column coefficients of orders +m and -m are staged in LDS first; U
// pairs share a workgroup so that small node counts still fill the lanes.
//
// The samples then stay in LDS for the Legendre projection, a real GEMM per
// order whose matrix W^m (rows n = |m|..Pt, columns the nodes j) is the same
// for every pair of the stage:
//     Out[n][(u, c)] = sum_j W^m[n][j] S[j][(u, c)],   c in {f.re, f.im, g.re, g.im},
// and b_n^m = Tc_n (f) + Tdc_n (g).  The workgroup's wavefronts take its
// 16 x 16 tiles (16 degrees x 4 pairs) on the FP64 matrix cores with
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// holds D[4v + l/16][l%16], v = 0..3.  The workgroup of order Ps also writes
// the zero coefficients of orders Ps < |m| <= Pt, which have no samples.
typedef double v4d __attribute__((ext_vector_type(4)));

// LDS of the coaxial workgroup: staged coefficients [U][2][Ps + 1] (complex),
// samples [2 signs][nq][ncp] (double) and one 16 x 17 transposition tile per
// wavefront.
struct CoaxLds {
    int ncp;                 // sample columns per node: 4 U rounded up to 16
    size_t cpm, smp, tile;   // offsets in doubles
    size_t bytes;
};
__host__ __device__ inline CoaxLds coax_lds(int U, int Ps, int nq, int waves)
{
    CoaxLds L;
    L.ncp = (4 * U + 15) / 16 * 16;
    L.cpm = 0;
    L.smp = L.cpm + (size_t)U * 2 * (Ps + 1) * 2;
    L.tile = L.smp + (size_t)2 * nq * L.ncp;
    L.bytes = (L.tile + (size_t)waves * 16 * 17) * sizeof(double);
    return L;
}

__global__ __launch_bounds__(256) void k_h3d_coax(H3DTr tr, int U)
{
    extern __shared__ double cl[];
    int Ps = tr.Ps, Pt = tr.Pt, nq = tr.nq;
    int nw = blockDim.x >> 6;
    CoaxLds L = coax_lds(U, Ps, nq, nw);
    cplx* cpm = reinterpret_cast<cplx*>(cl + L.cpm);
    double* smp = cl + L.smp;
    // the Ps + 1 orders of one pair group run on one XCD, so that the group's
    // radial values and coefficients are read from that XCD's L2
    int wg = xcd_contiguous(blockIdx.x, gridDim.x);
    int am = wg % (Ps + 1);
    int i0 = (wg / (Ps + 1)) * U;
    int cnt = Ps + 1 - am;
    for (int e = threadIdx.x; e < U * cnt; e += blockDim.x) {
        int u = e / cnt, n = am + (e - u * cnt);
        const cplx* a = tr.A + (size_t)min(i0 + u, tr.np - 1) * tr.sA;
        cpm[(2 * u) * (Ps + 1) + n] = a[hnm(n, am)];
        cpm[(2 * u + 1) * (Ps + 1) + n] = a[hnm(n, -am)];
    }
    __syncthreads();
    int u = threadIdx.x / nq;
    if (u < U) {
        int j = threadIdx.x - u * nq;
        int i = min(i0 + u, tr.np - 1);       // the group's tail repeats the last pair
        const cplx* cpp = cpm + (2 * u) * (Ps + 1);
        const cplx* cpn = cpp + (Ps + 1);
        const RecAB* rec = static_cast<const RecAB*>(tr.rec) + am * kT;   // column am
        cplx t = tr.geo[(size_t)i * 10 + 9];
        double s1 = tr.sth[j], s3 = tr.cth[j];
        cplx x1 = mk(tr.rs * s1, 0.0);
        cplx x3 = t + mk(tr.rs * s3, 0.0);
        cplx r2 = x1 * x1 + x3 * x3;
        cplx sx = s1 * x1 + s3 * x3;
        cplx dr2 = 2.0 * sx;
        const cplx* R = tr.R + (size_t)i * tr.sR + j;
        double fac = tr.src_h ? -tr.ks / tr.sc : -tr.ks * tr.sc;
        // diagonal start c_m x1^m and its derivative c_m m x1^{m-1} s1
        cplx D = mk(c_cs[am], 0.0), dD = mk(0.0, 0.0);
        {
            cplx pw = mk(1.0, 0.0);
            for (int k = 0; k < am; ++k) {
                if (k == am - 1) dD = (double)am * c_cs[am] * s1 * pw;
                pw = pw * x1;
            }
            D = c_cs[am] * pw;
        }
        cplx fp = mk(0.0, 0.0), fm = fp, gp = fp, gm = fp;
        // the diagonal start is folded into the column: Q = D q obeys the same
        // recurrence as q, and its derivative dQ = dD q + D dq the
        // differentiated one, so S_n^m = Q_n and its derivative is dQ_n
        cplx q0 = mk(0.0, 0.0), q1 = D, dq0 = q0, dq1 = dD;
        cplx z = x3, dz = mk(s3, 0.0);
        // radial values one degree ahead: the load for n + 2 is in flight
        // while degree n is summed
        cplx Rn = R[(size_t)am * nq], Rn1 = R[(size_t)(am + 1) * nq];
        auto accum = [&](int n) {
            cplx f = Rn * q1;
            cplx gg = (fac * Rn1) * (sx * q1) + Rn * dq1;
            cplx cp = cpp[n];
            fp += cp * f;
            gp += cp * gg;
            if (am) {
                cplx cm = cpn[n];
                fm += cm * f;
                gm += cm * gg;
            }
        };
        {
            cplx Rn2 = am + 2 <= Ps + 1 ? R[(size_t)(am + 2) * nq] : mk(0.0, 0.0);
            accum(am);
            Rn = Rn1;
            Rn1 = Rn2;
        }
#pragma unroll 2
        for (int n = am + 1; n <= Ps; ++n) {
            cplx Rn2 = n + 2 <= Ps + 1 ? R[(size_t)(n + 2) * nq] : mk(0.0, 0.0);
            col_step(rec, n, z, dz, r2, dr2, q0, q1, dq0, dq1);
            accum(n);
            Rn = Rn1;
            Rn1 = Rn2;
        }
        double* sp = smp + (size_t)j * L.ncp + 4 * u;               // order +m
        double* sm = smp + (size_t)(nq + j) * L.ncp + 4 * u;        // order -m
        sp[0] = fp.re; sp[1] = fp.im; sp[2] = gp.re; sp[3] = gp.im;
        sm[0] = fm.re; sm[1] = fm.im; sm[2] = gm.re; sm[3] = gm.im;
    }
    __syncthreads();
    // projection tiles: (sign, 16-degree row tile, 4-pair column tile)
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    int r = l & 15, kq = l >> 4;
    double* tile = cl + L.tile + (size_t)wave * 16 * 17;
    int nsg = am ? 2 : 1, nrt = (Pt - am + 16) / 16, nct = (U + 3) / 4;
    for (int tix = wave; tix < nsg * nrt * nct; tix += nw) {
        int sg = tix / (nrt * nct), rt = (tix / nct) % nrt, ct = tix % nct;
        int n0 = am + 16 * rt;
        const double* S = smp + (size_t)sg * nq * L.ncp + 16 * ct;
        int na = n0 + r;                      // A row this lane supplies
        bool arow = na <= Pt;
        const double* wrow = tr.W + (size_t)tri(arow ? na : n0, am) * nq;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < nq; k0 += 4) {
            int jj = k0 + kq;
            double av = (arow && jj < nq) ? wrow[jj] : 0.0;
            double bv = jj < nq ? S[(size_t)jj * L.ncp + r] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        // gather the four components of each pair through the wave's tile
        for (int v = 0; v < 4; ++v) tile[(4 * v + kq) * 17 + r] = acc[v];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        int dr = l >> 2, pq = l & 3;
        int n = n0 + dr, uo = 4 * ct + pq, io = i0 + uo;
        if (n <= Pt && uo < U && io < tr.np) {
            const double* tv = tile + dr * 17 + 4 * pq;
            cplx pf = mk(tv[0], tv[1]), pg = mk(tv[2], tv[3]);
            int m = sg ? -am : am;
            tr.B[(size_t)io * tr.sB + hnm(n, m)] = tr.Tc[n] * pf + tr.Tdc[n] * pg;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    // orders beyond the source expansion have no samples: zero coefficients
    if (am == Ps && Pt > Ps) {
        int per = (Pt + 1) * (Pt + 1);
        for (int e = threadIdx.x; e < U * per; e += blockDim.x) {
            int uo = e / per, c = e - uo * per, io = i0 + uo;
            int n = (int)sqrt((double)c);
            while (n * n > c) --n;
            while ((n + 1) * (n + 1) <= c) ++n;
            int m = c - n * n - n;
            if (io < tr.np && (m > Ps || m < -Ps)) tr.B[(size_t)io * tr.sB + c] = mk(0.0, 0.0);
        }
    }
}

// K7: each target box adds its pairs' translated expansions, in pair order.
__global__ void k_h3d_accum(H3DTr tr, const int* __restrict__ gdst, const int* __restrict__ goff, int ng,
                            const int* __restrict__ eoff, cplx* __restrict__ out)
{
    int nc = (tr.Pt + 1) * (tr.Pt + 1);
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)ng * nc) return;
    int c = (int)(gid % nc);
    int k = (int)(gid / nc);
    cplx s = mk(0.0, 0.0);
    // unrolled so that several pairs' loads are in flight; the sum stays in
    // pair order
#pragma unroll 8
    for (int i = goff[k]; i < goff[k + 1]; ++i) s += tr.A[(size_t)i * tr.sA + c];
    out[eoff[gdst[k]] + c] += s;
}

inline unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t h3d_init_tables(int device)
{
    static RecAB rab[kT * kT];
    static RecABf rabf[kT * kT];
    static double cs[kT], ck[kT];
    for (int m = 0; m < kT; ++m)
        for (int n = 0; n < kT; ++n) {
            double a = (double)(n + m - 1) * (double)(n - m - 1);
            double b = (double)(n - m) * (double)(n + m);
            double ib = n > m && b > 0.0 ? 1.0 / sqrt(b) : 0.0;
            RecAB& r = rab[m * kT + n];
            r.s = (2.0 * n - 1.0) * ib;
            r.a = (a > 0.0 ? sqrt(a) : 0.0) * ib;
            rabf[m * kT + n] = RecABf{(float)r.s, (float)r.a};
        }
    cs[0] = 1.0;
    ck[0] = 1.0;
    for (int m = 1; m < kT; ++m) {
        ck[m] = sqrt((2.0 * m - 1.0) / (2.0 * m));
        cs[m] = cs[m - 1] * ck[m];
    }
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rab), rab, sizeof(rab))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rabf), rabf, sizeof(rabf))) != hipSuccess) return e;
    if (device < 0 || device >= kMaxDev) return hipErrorInvalidDevice;
    void* a = nullptr;
    if ((e = hipGetSymbolAddress(&a, HIP_SYMBOL(c_rab))) != hipSuccess) return e;
    g_rab[device] = a;
    if ((e = hipGetSymbolAddress(&a, HIP_SYMBOL(c_rabf))) != hipSuccess) return e;
    g_rabf[device] = a;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_cs), cs, sizeof(cs))) != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_ck), ck, sizeof(ck));
}

// the recurrence tables of the current device (h3d_init_tables ran for it)
static hipError_t rec_tables(const void** rec, const void** recf)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev || !g_rab[dev]) return hipErrorNotInitialized;
    *rec = g_rab[dev];
    if (recf) *recf = g_rabf[dev];
    return hipSuccess;
}

static size_t p2x_lds(int P, int threads)
{
    size_t st = (size_t)(threads / (2 * P + 1)) * (2 * P + 1);
    return sizeof(cplx) * ((size_t)(P + 1) * st + (size_t)(P + 2) * kPC + 4 * kPC);
}

template <bool IRREG>
static hipError_t launch_p2x(const int* boxes, int nb, int pmax, const TreeView& tv, const PointsView& pv,
                             const H3DLevels& hl, int useL4, cplx* out, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    // up to 128 threads: as many slices of the 2P+1 orders as fit
    int threads = 128;
    size_t lds = p2x_lds(pmax, threads);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_h3d_p2x<IRREG>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    H3DLevels h = hl;
    hipError_t e = rec_tables(&h.rec, nullptr);
    if (e != hipSuccess) return e;
    k_h3d_p2x<IRREG><<<nb, threads, lds, st>>>(boxes, tv, pv, h, useL4, out);
    return hipGetLastError();
}

hipError_t h3d_p2m(const int* boxes, int nb, int pmax, const TreeView& tv, const PointsView& pv,
                   const H3DLevels& hl, cplx* mpole, hipStream_t st)
{
    return launch_p2x<false>(boxes, nb, pmax, tv, pv, hl, 0, mpole, st);
}

hipError_t h3d_p2l(const int* boxes, int nb, int pmax, const TreeView& tv, const PointsView& pv,
                   const H3DLevels& hl, cplx* local, hipStream_t st)
{
    return launch_p2x<true>(boxes, nb, pmax, tv, pv, hl, 1, local, st);
}

hipError_t h3d_leaf_far(const int* leaves, int nleaf, int top, int pmax, const TreeView& tv,
                        const PointsView& pv, const H3DLevels& hl, const cplx* mpole,
                        const cplx* local, const M2PParts& m2p, cplx* ufar, hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    H3DLevels h = hl;
    hipError_t er = rec_tables(&h.rec, nullptr);
    if (er != hipSuccess) return er;
    size_t lds = sizeof(cplx) * (size_t)(pmax + 3) * 64;
    if (m2p.n > 0) {
        k_h3d_m2p_part<<<m2p.n, 64, lds, st>>>(m2p.owner, m2p.poff, tv, pv, h, mpole, m2p.part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_h3d_leaf_far<<<nleaf, 64, lds, st>>>(leaves, top, tv, pv, h, local, m2p.poff, m2p.part, ufar);
    return hipGetLastError();
}


// Workgroup shape for a kernel whose item takes w consecutive threads: the
// size in {64, 128, 192, 256} that leaves the fewest lanes idle (the smaller
// one unless a larger one fills 2% more), with per-workgroup LDS lds(U, size)
// for U items at most 64 KiB.  threads = 0 when no size fits.
struct PackShape {
    int threads, per;
};
template <class F>
static PackShape pack_items(int w, F lds)
{
    PackShape best{0, 0};
    double bu = -1.0;
    for (int bt = 64; bt <= 256; bt += 64) {
        int U = bt / w;
        if (U < 1 || lds(U, bt) > 65536) continue;
        double util = (double)(U * w) / bt;
        if (util > bu + 0.02) {
            bu = util;
            best = {bt, U};
        }
    }
    return best;
}

template <int NB>
static hipError_t launch_rot_sample(const H3DTr& tr, int back, const int* eoff, const cplx* coef, hipStream_t st)
{
    int P = back ? tr.Pt : tr.Ps;
    int J = 2 * P + 1, nblk = (P + NB) / NB;
    int smax = 0;
    for (int b = 0; b < nblk; ++b) {
        int nlo = b * NB, nhi = std::min(P, nlo + NB - 1), n0 = nlo > 0 ? nlo - 1 : 0;
        smax = std::max(smax, (nhi + 1) * (nhi + 1) - n0 * n0);
    }
    size_t esz = tr.f32 ? 2 * sizeof(float) : 2 * sizeof(double);
    PackShape pk = pack_items(J, [&](int U, int) { return (size_t)U * 2 * smax * esz; });
    if (pk.threads == 0) return hipErrorInvalidValue;
    int64_t wpb = (tr.np + pk.per - 1) / pk.per;
    unsigned grid = (unsigned)(wpb * nblk);
    size_t lds = (size_t)pk.per * 2 * smax * esz;
    if (tr.f32)
        k_h3d_rot_sample<NB, float><<<grid, pk.threads, lds, st>>>(tr, back, eoff, coef, pk.per, smax);
    else
        k_h3d_rot_sample<NB, double><<<grid, pk.threads, lds, st>>>(tr, back, eoff, coef, pk.per, smax);
    return hipGetLastError();
}

// The rotation DFT of one side (P = Ps forward, Pt back): staged in LDS when a
// pair's (P+1)(P+2)/2 outputs fit one workgroup and U pairs' samples fit
// 48 KiB, else one thread per output reading the samples from memory.
static hipError_t launch_rot_dft(const H3DTr& tr, int back, const double* eq_p0, const double* eq_d0,
                                 hipStream_t st)
{
    int P = back ? tr.Pt : tr.Ps;
    int J = 2 * P + 1, nt = (P + 1) * (P + 2) / 2;
    size_t row = (size_t)2 * (P + 1) * J * sizeof(cplx), head = (size_t)(2 * J + 2) * sizeof(double);
    int U = nt <= 256 ? 256 / nt : 0;
    while (U > 0 && head + U * row > 49152) --U;
    if (U > 0) {
        int threads = (U * nt + 63) / 64 * 64;
        unsigned grid = (unsigned)((tr.np + U - 1) / U);
        k_h3d_rot_dft_lds<<<grid, threads, head + U * row, st>>>(tr, back, eq_p0, eq_d0, U);
    } else {
        int64_t n = (int64_t)tr.np * nt;
        k_h3d_rot_dft<<<blocks(n, 256), 256, sizeof(double) * 2 * J, st>>>(tr, back, eq_p0, eq_d0);
    }
    return hipGetLastError();
}

// One chunk of a translation stage: pairs [0, tr.np) of the chunk, target
// groups [0, ng) with pair ranges goff (chunk-relative).
hipError_t h3d_translate(const H3DTr& tr_in, const TreeView& tv, const int* eoff_src, const cplx* coef_src,
                         const int* gdst, const int* goff, int ng, const int* eoff_dst, cplx* coef_dst,
                         const double* eq_p0, const double* eq_d0, hipStream_t st)
{
    if (tr_in.np <= 0) return hipSuccess;
    H3DTr tr = tr_in;
    {
        hipError_t e0 = rec_tables(&tr.rec, &tr.recf);
        if (e0 != hipSuccess) return e0;
    }
    // one thread per node or per equator sample in the sampling kernels
    if (tr.nq > 128 || 2 * tr.Ps + 1 > 128 || 2 * tr.Pt + 1 > 128) return hipErrorInvalidValue;
    const int bs = 256;
    constexpr int NB = 8;
    hipError_t e;
    k_h3d_geo<<<blocks(tr.np, bs), bs, 0, st>>>(tr, tv);
    int Ps = tr.Ps, Pt = tr.Pt;
    k_h3d_rot_prep<<<blocks((int64_t)tr.np * Ps * Ps, bs), bs, 0, st>>>(tr, 0, eoff_src, coef_src);
    if ((e = launch_rot_sample<NB>(tr, 0, eoff_src, coef_src, st)) != hipSuccess) return e;
    if ((e = launch_rot_dft(tr, 0, eq_p0, eq_d0, st)) != hipSuccess) return e;
    int64_t n3 = (int64_t)tr.np * tr.nq;
    k_h3d_coax_radial<<<blocks(n3, bs), bs, 0, st>>>(tr);
    {
        // the workgroup size leaves room for its waves' tiles in the LDS bound
        PackShape pk = pack_items(tr.nq, [&](int U, int bt) { return coax_lds(U, Ps, tr.nq, bt / 64).bytes; });
        if (pk.threads == 0) return hipErrorInvalidValue;
        int64_t groups = (tr.np + pk.per - 1) / pk.per;
        k_h3d_coax<<<(unsigned)(groups * (Ps + 1)), pk.threads,
                     coax_lds(pk.per, Ps, tr.nq, pk.threads / 64).bytes, st>>>(tr, pk.per);
    }
    k_h3d_rot_prep<<<blocks((int64_t)tr.np * Pt * Pt, bs), bs, 0, st>>>(tr, 1, nullptr, nullptr);
    if ((e = launch_rot_sample<NB>(tr, 1, nullptr, nullptr, st)) != hipSuccess) return e;
    if ((e = launch_rot_dft(tr, 1, eq_p0, eq_d0, st)) != hipSuccess) return e;
    int64_t n7 = (int64_t)ng * (Pt + 1) * (Pt + 1);
    k_h3d_accum<<<blocks(n7, bs), bs, 0, st>>>(tr, gdst, goff, ng, eoff_dst, coef_dst);
    return hipGetLastError();
}

}  // namespace cfmm
