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
    for (int k = 1; k <= am; ++k) d = d * w * ir2 * (double)(2 * k - 1);
    bool neg = (m < 0 && (am & 1)) != flip;
    if (neg) d = -d;
    f(am, d);
    if (am + 1 > P) return;
    cplx a = d, b = (2.0 * am + 1.0) * (v.z * d * ir2);
    f(am + 1, b);
    for (int n = am + 2; n <= P; ++n) {
        cplx c = ((2.0 * n - 1.0) * (v.z * b) - ((double)(n + am - 1) * (double)(n - am - 1)) * a) * ir2;
        f(n, c);
        a = b;
        b = c;
    }
}

// ------------------------------------------------------------ P2M / P2L
// One workgroup per box; thread t owns order m = t - P and accumulates its
// column over the box's (or List-4 boxes') points in LDS.
template <bool IRREGULAR>
__global__ void k_l3d_p2x(const int* __restrict__ boxes, TreeView tv, PointsView pv, int useL4,
                          cplx* __restrict__ out)
{
    extern __shared__ cplx acc[];      // acc[n * blockDim.x + t]
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    double s = tv.rs[l];
    int t = threadIdx.x, st = blockDim.x, mm = t - P;
    bool act = t < 2 * P + 1;
    int am = mm < 0 ? -mm : mm;
    if (act)
        for (int n = am; n <= P; ++n) acc[n * st + t] = mk(0.0, 0.0);
    cplx c[3];
    box_centre(tv, b, c);
    int e0 = useL4 ? tv.l4off[b] : 0, e1 = useL4 ? tv.l4off[b + 1] : 1;
    for (int e = e0; e < e1; ++e) {
        int src = useL4 ? tv.l4idx[e] : b;
        for (int j = tv.pbeg[src]; j < tv.pend[src]; ++j) {
            if (!act) continue;
            Vec3 y = point_rel(pv, j, c, s);
            cplx sg = mk(pv.sre[j], pv.sim[j]);
            // (-1)^m X_n^{-m}(y): order -mm, flipped sign when mm odd
            auto f = [&](int n, cplx v) { acc[n * st + t] += v * sg; };
            if (IRREGULAR) col_I(y, -mm, P, (am & 1) != 0, f);
            else col_R(y, -mm, P, (am & 1) != 0, f);
        }
    }
    if (act) {
        cplx* o = out + tv.eoff[b];
        for (int n = am; n <= P; ++n) {
            if (useL4) o[nm(n, mm)] += acc[n * st + t];
            else o[nm(n, mm)] = acc[n * st + t];
        }
    }
}

// ------------------------------------------------------------------ M2M
// One workgroup per parent; for each child, the table R_l^q(d / w_p) (l <= P)
// and the child's multipole go to LDS; thread owns outputs (n, m).
__global__ __launch_bounds__(256) void k_l3d_m2m(const int* __restrict__ boxes, TreeView tv,
                                                 cplx* __restrict__ mpole)
{
    extern __shared__ cplx sh[];
    int p = boxes[blockIdx.x];
    int l = tv.level[p];
    int P = tv.P[l];
    int nc = (P + 1) * (P + 1);
    cplx* Rt = sh;             // nc
    cplx* Mc = sh + nc;        // nc
    double s = tv.rs[l];
    int t = threadIdx.x;
    cplx acc[4];
    for (int r = 0; r < 4; ++r) acc[r] = mk(0.0, 0.0);
    cplx cp[3];
    box_centre(tv, p, cp);
    for (int ci = 0; ci < tv.nchild[p]; ++ci) {
        int c = tv.child0[p] + ci;
        __syncthreads();
        if (t < 2 * P + 1) {
            cplx cc[3];
            box_centre(tv, c, cc);
            Vec3 d;
            d.x = (cc[0] - cp[0]) * s; d.y = (cc[1] - cp[1]) * s; d.z = (cc[2] - cp[2]) * s;
            int q = t - P;
            col_R(d, q, P, false, [&](int n, cplx v) { Rt[nm(n, q)] = v; });
        }
        for (int i = t; i < nc; i += blockDim.x) Mc[i] = mpole[tv.eoff[c] + i];
        __syncthreads();
        for (int r = 0; r < 4; ++r) {
            int o = t + r * blockDim.x;
            if (o >= nc) break;
            int n = (int)sqrt((double)o);
            while (n * n > o) --n;
            while ((n + 1) * (n + 1) <= o) ++n;
            int m = o - n * n - n;
            cplx a = mk(0.0, 0.0);
            double h = 1.0;
            for (int j = 0; j <= n; ++j, h *= 0.5) {
                int lmax = n - j;
                cplx aj = mk(0.0, 0.0);
                for (int k = -j; k <= j; ++k) {
                    int q = m - k;
                    if (q > lmax || q < -lmax) continue;
                    cplx rv = Rt[nm(lmax, -q)];
                    if (q & 1) rv = -rv;
                    aj += Mc[nm(j, k)] * rv;
                }
                a += h * aj;
            }
            acc[r] += a;
        }
    }
    for (int r = 0; r < 4; ++r) {
        int o = t + r * blockDim.x;
        if (o < nc) mpole[tv.eoff[p] + o] = acc[r];
    }
}

// ------------------------------------------------------------------ M2L
// One workgroup per target box; per source box the table I_l^q(D / w),
// l <= 2P, is built by columns (one thread per order q) in LDS.
__global__ __launch_bounds__(256) void k_l3d_m2l(const int* __restrict__ boxes, TreeView tv,
                                                 const cplx* __restrict__ mpole,
                                                 cplx* __restrict__ local)
{
    extern __shared__ cplx sh[];
    int b = boxes[blockIdx.x];
    int l = tv.level[b];
    int P = tv.P[l];
    int nc = (P + 1) * (P + 1), ni = (2 * P + 1) * (2 * P + 1);
    cplx* It = sh;             // ni
    cplx* Ms = sh + ni;        // nc
    double s = tv.rs[l];
    int t = threadIdx.x;
    cplx acc[4];
    for (int r = 0; r < 4; ++r) acc[r] = mk(0.0, 0.0);
    int jj[4], kk[4];
    for (int r = 0; r < 4; ++r) {
        int o = t + r * blockDim.x;
        int n = (int)sqrt((double)o);
        while (n * n > o) --n;
        while ((n + 1) * (n + 1) <= o) ++n;
        jj[r] = n;
        kk[r] = o - n * n - n;
    }
    cplx cb[3];
    box_centre(tv, b, cb);
    for (int e = tv.l2off[b]; e < tv.l2off[b + 1]; ++e) {
        int a = tv.l2idx[e];
        __syncthreads();
        if (t < 4 * P + 1) {
            cplx ca[3];
            box_centre(tv, a, ca);
            Vec3 d;
            d.x = (cb[0] - ca[0]) * s; d.y = (cb[1] - ca[1]) * s; d.z = (cb[2] - ca[2]) * s;
            int q = t - 2 * P;
            col_I(d, q, 2 * P, false, [&](int n, cplx v) { It[nm(n, q)] = v; });
        }
        for (int i = t; i < nc; i += blockDim.x) Ms[i] = mpole[tv.eoff[a] + i];
        __syncthreads();
        for (int r = 0; r < 4; ++r) {
            int o = t + r * blockDim.x;
            if (o >= nc) break;
            int j = jj[r], k = kk[r];
            cplx a2 = mk(0.0, 0.0);
            for (int n = 0; n <= P; ++n) {
                const cplx* Irow = It + (j + n) * (j + n) + (j + n) - k;   // It[nm(j+n, m-k)] = Irow[m]
                const cplx* Mrow = Ms + n * n + n;
                for (int m = -n; m <= n; ++m) a2 += Mrow[m] * Irow[m];
            }
            acc[r] += a2;
        }
    }
    for (int r = 0; r < 4; ++r) {
        int o = t + r * blockDim.x;
        if (o < nc) {
            cplx v = acc[r];
            if ((jj[r] + kk[r]) & 1) v = -v;
            local[tv.eoff[b] + o] = v;
        }
    }
}

// ------------------------------------------------------------------ L2L
__global__ __launch_bounds__(256) void k_l3d_l2l(const int* __restrict__ boxes, TreeView tv,
                                                 cplx* __restrict__ local)
{
    extern __shared__ cplx sh[];
    int c = boxes[blockIdx.x];
    int p = tv.parent[c];
    int lp = tv.level[p];
    int P = tv.P[lp];
    int nc = (P + 1) * (P + 1);
    cplx* Rt = sh;
    cplx* Lp = sh + nc;
    double s = tv.rs[lp];
    int t = threadIdx.x;
    if (t < 2 * P + 1) {
        cplx cp[3], cc[3];
        box_centre(tv, p, cp);
        box_centre(tv, c, cc);
        Vec3 d;
        d.x = (cc[0] - cp[0]) * s; d.y = (cc[1] - cp[1]) * s; d.z = (cc[2] - cp[2]) * s;
        int q = t - P;
        col_R(d, q, P, false, [&](int n, cplx v) { Rt[nm(n, q)] = v; });
    }
    for (int i = t; i < nc; i += blockDim.x) Lp[i] = local[tv.eoff[p] + i];
    __syncthreads();
    for (int o = t; o < nc; o += blockDim.x) {
        int j = (int)sqrt((double)o);
        while (j * j > o) --j;
        while ((j + 1) * (j + 1) <= o) ++j;
        int k = o - j * j - j;
        cplx a = mk(0.0, 0.0);
        for (int n = j; n <= P; ++n) {
            int lmax = n - j;
            for (int m = -n; m <= n; ++m) {
                int q = m - k;
                if (q > lmax || q < -lmax) continue;
                a += Lp[nm(n, m)] * Rt[nm(lmax, q)];
            }
        }
        local[tv.eoff[c] + o] += ldexp(1.0, -(j + 1)) * a;
    }
}

// ------------------------------------------------------------- L2P + M2P
__global__ __launch_bounds__(64) void k_l3d_leaf_far(const int* __restrict__ leaves, int top,
                                                     TreeView tv, PointsView pv,
                                                     const cplx* __restrict__ mpole,
                                                     const cplx* __restrict__ local,
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
            Vec3 x = point_rel(pv, i, c, s);
            const cplx* L = local + tv.eoff[b];
            cplx ul = mk(0.0, 0.0);
            for (int m = -P; m <= P; ++m)
                col_R(x, m, P, false, [&](int n, cplx v) { ul += L[nm(n, m)] * v; });
            u = s * ul;
            for (int e = tv.l3off[b]; e < tv.l3off[b + 1]; ++e) {
                int a = tv.l3idx[e];
                int la = tv.level[a];
                int Pa = tv.P[la];
                double sa = tv.rs[la];
                box_centre(tv, a, c);
                Vec3 y = point_rel(pv, i, c, sa);
                const cplx* M = mpole + tv.eoff[a];
                cplx um = mk(0.0, 0.0);
                for (int m = -Pa; m <= Pa; ++m)
                    col_I(y, m, Pa, false, [&](int n, cplx v) { um += M[nm(n, m)] * v; });
                u += sa * um;
            }
        }
        ufar[i] = u;
    }
}


// ---------------------------------------------------------------- launchers
static size_t lds_bytes(int nelem) { return (size_t)nelem * sizeof(cplx); }

hipError_t l3d_p2m(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   cplx* mpole, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    int th = ((2 * P + 1 + 63) / 64) * 64;
    k_l3d_p2x<false><<<nb, th, lds_bytes((P + 1) * th), st>>>(boxes, tv, pv, 0, mpole);
    return hipGetLastError();
}

hipError_t l3d_p2l(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    int th = ((2 * P + 1 + 63) / 64) * 64;
    k_l3d_p2x<true><<<nb, th, lds_bytes((P + 1) * th), st>>>(boxes, tv, pv, 1, local);
    return hipGetLastError();
}

hipError_t l3d_m2m(const int* boxes, int nb, int P, const TreeView& tv, cplx* mpole, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_l3d_m2m<<<nb, 256, lds_bytes(2 * (P + 1) * (P + 1)), st>>>(boxes, tv, mpole);
    return hipGetLastError();
}

hipError_t l3d_m2l(const int* boxes, int nb, int P, const TreeView& tv, const cplx* mpole,
                   cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    size_t lds = lds_bytes((2 * P + 1) * (2 * P + 1) + (P + 1) * (P + 1));
    k_l3d_m2l<<<nb, 256, lds, st>>>(boxes, tv, mpole, local);
    return hipGetLastError();
}

hipError_t l3d_l2l(const int* boxes, int nb, int P, const TreeView& tv, cplx* local, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    k_l3d_l2l<<<nb, 256, lds_bytes(2 * (P + 1) * (P + 1)), st>>>(boxes, tv, local);
    return hipGetLastError();
}

hipError_t l3d_leaf_far(const int* leaves, int nleaf, int top, const TreeView& tv,
                        const PointsView& pv, const cplx* mpole, const cplx* local, cplx* ufar,
                        hipStream_t st)
{
    if (nleaf <= 0) return hipSuccess;
    k_l3d_leaf_far<<<nleaf, 64, 0, st>>>(leaves, top, tv, pv, mpole, local, ufar);
    return hipGetLastError();
}


size_t l3d_max_lds_m2l(int P) { return lds_bytes((2 * P + 1) * (2 * P + 1) + (P + 1) * (P + 1)); }

// Largest P the kernels take: 4 outputs per thread of a 256-thread M2L
// workgroup ((P+1)^2 <= 1024) and the M2L tables within the device's LDS.
int l3d_pmax_supported()
{
    int dev = 0, lds = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lds = v;
    }
    int P = 31;
    while (P > 1 && l3d_max_lds_m2l(P) > (size_t)lds) --P;
    return P;
}

}  // namespace cfmm
