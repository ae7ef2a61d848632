// Tree construction kernels (Sec. 6.1): real-part bounding box, Morton keys,
// a stable LSD radix sort of (key, index) built on wavefront ballots, point
// and density gathers into sorted SoA order, and the complexified box centres.
#include "common.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace cfmm {

// ------------------------------------------------------------ bounding box
// partial[blk * (2*dim+1) + ...] = { min_d..., max_d..., nonfinite flag }
__global__ void k_bbox_partial(const double* __restrict__ pts, int64_t n, int dim,
                               double* __restrict__ partial)
{
    __shared__ double smin[3][256], smax[3][256];
    __shared__ int sbad[256];
    int t = threadIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < dim; ++d) {
            double re = pts[(i * dim + d) * 2], im = pts[(i * dim + d) * 2 + 1];
            if (!isfinite(re) || !isfinite(im)) bad = 1;
            mn[d] = fmin(mn[d], re);
            mx[d] = fmax(mx[d], re);
        }
    }
    for (int d = 0; d < 3; ++d) { smin[d][t] = mn[d]; smax[d][t] = mx[d]; }
    sbad[t] = bad;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
            for (int d = 0; d < 3; ++d) {
                smin[d][t] = fmin(smin[d][t], smin[d][t + s]);
                smax[d][t] = fmax(smax[d][t], smax[d][t + s]);
            }
            sbad[t] |= sbad[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = partial + (size_t)blockIdx.x * (2 * dim + 1);
        for (int d = 0; d < dim; ++d) { o[d] = smin[d][0]; o[dim + d] = smax[d][0]; }
        o[2 * dim] = (double)sbad[0];
    }
}

// one block of 256 threads over the per-block partials (min and max are
// exact, so the order of the reduction does not matter)
__global__ void k_bbox_final(const double* __restrict__ partial, int nb, int dim, double* __restrict__ out)
{
    __shared__ double smin[3][256], smax[3][256], sbad[256];
    int t = threadIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0.0;
    for (int b = t; b < nb; b += blockDim.x) {
        const double* p = partial + (size_t)b * (2 * dim + 1);
        for (int d = 0; d < dim; ++d) { mn[d] = fmin(mn[d], p[d]); mx[d] = fmax(mx[d], p[dim + d]); }
        bad = fmax(bad, p[2 * dim]);
    }
    for (int d = 0; d < 3; ++d) { smin[d][t] = mn[d]; smax[d][t] = mx[d]; }
    sbad[t] = bad;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
            for (int d = 0; d < 3; ++d) {
                smin[d][t] = fmin(smin[d][t], smin[d][t + s]);
                smax[d][t] = fmax(smax[d][t], smax[d][t + s]);
            }
            sbad[t] = fmax(sbad[t], sbad[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int d = 0; d < dim; ++d) { out[d] = smin[d][0]; out[dim + d] = smax[d][0]; }
        out[2 * dim] = sbad[0];
    }
}

// ------------------------------------------------------------- Morton keys
__device__ inline uint64_t spread2(uint64_t v)   // bit b -> bit 2b
{
    v &= 0x7fffffffull;
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}
__device__ inline uint64_t spread3(uint64_t v)   // bit b -> bit 3b
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x001f00000000ffffull;
    v = (v | (v << 16)) & 0x001f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_morton(const double* __restrict__ pts, int64_t n, int dim, KeyParams kp,
                         uint64_t* __restrict__ keys, int* __restrict__ idx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t key = 0;
    double top = kp.top;
    for (int d = 0; d < dim; ++d) {
        double re = pts[(i * dim + d) * 2];
        double t = (re - kp.lo[d]) * kp.scale;   // no contraction: same rounding as the host
        double q = floor(t);
        q = q < 0.0 ? 0.0 : (q > top ? top : q);
        uint64_t qi = (uint64_t)q;
        key |= (dim == 2 ? spread2(qi) : spread3(qi)) << d;
    }
    keys[i] = key;
    idx[i] = (int)i;
}

// ---------------------------------------------------------------- radix sort
// Tile of kRsThreads * kRsRounds keys per block; 8-bit digits.
__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                          unsigned* __restrict__ hist, int nblk)
{
    __shared__ unsigned cnt[256];
    int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        int64_t i = base + (int64_t)r * kRsThreads + t;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)t * nblk + blockIdx.x] = cnt[t];
}

// exclusive scan, 2048 elements per block; block totals to `sums`
__global__ void k_scan_block(unsigned* __restrict__ a, int64_t m, unsigned* __restrict__ sums)
{
    __shared__ unsigned s[256];
    int t = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * 2048 + (int64_t)t * 8;
    unsigned v[8], run = 0;
    for (int k = 0; k < 8; ++k) {
        v[k] = (base + k < m) ? a[base + k] : 0u;
        unsigned x = v[k];
        v[k] = run;
        run += x;
    }
    s[t] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {      // inclusive Hillis-Steele
        unsigned x = (t >= off) ? s[t - off] : 0u;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    unsigned excl = (t > 0) ? s[t - 1] : 0u;
    for (int k = 0; k < 8; ++k)
        if (base + k < m) a[base + k] = v[k] + excl;
    if (t == 255 && sums) sums[blockIdx.x] = s[255];
}

__global__ void k_scan_add(unsigned* __restrict__ a, int64_t m, const unsigned* __restrict__ offs)
{
    int64_t i = (int64_t)blockIdx.x * 2048 + threadIdx.x;
    unsigned o = offs[blockIdx.x];
    for (int k = 0; k < 8; ++k, i += 256)
        if (i < m) a[i] += o;
}

__global__ void k_rs_scatter(const uint64_t* __restrict__ kin, const int* __restrict__ vin,
                             uint64_t* __restrict__ kout, int* __restrict__ vout, int64_t n,
                             int shift, const unsigned* __restrict__ hist, int nblk)
{
    __shared__ unsigned running[256];
    __shared__ unsigned wcnt[kRsThreads / 64][256];
    int t = threadIdx.x;
    int lane = t & 63, wave = t >> 6;
    running[t] = hist[(size_t)t * nblk + blockIdx.x];
    for (int w = 0; w < kRsThreads / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < kRsRounds; ++r) {
        int64_t i = base + (int64_t)r * kRsThreads + t;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        int val = valid ? vin[i] : 0;
        unsigned d = (unsigned)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        unsigned rank = (unsigned)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (unsigned)__popcll(peers);
        __syncthreads();
        if (valid) {
            unsigned off = running[d] + rank;
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        unsigned add = 0;
        for (int w = 0; w < kRsThreads / 64; ++w) { add += wcnt[w][t]; wcnt[w][t] = 0; }
        running[t] += add;
        __syncthreads();
    }
}

// -------------------------------------------------------------- gathers
__global__ void k_gather_points(const double* __restrict__ pts, const int* __restrict__ perm,
                                int64_t n, int dim, double* __restrict__ xre, double* __restrict__ xim)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t p = perm[i];
    for (int d = 0; d < dim; ++d) {
        xre[d * n + i] = pts[(p * dim + d) * 2];
        xim[d * n + i] = pts[(p * dim + d) * 2 + 1];
    }
}

// sigma into sorted order; target-only tree points carry zero density
__global__ void k_gather_density(const double* __restrict__ sig, IoMap io,
                                 int64_t n, double* __restrict__ sre, double* __restrict__ sim)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t p = io.perm[i];
    bool src = p < io.nsrc;
    sre[i] = src ? sig[2 * p] : 0.0;
    sim[i] = src ? sig[2 * p + 1] : 0.0;
}

// Complexified centres (a4): the mean imaginary part of each box's points and
// their largest imaginary spread about it.  Boxes are cut into chunks of at
// most kCentreChunk points (the root holds all N), so every level runs in
// parallel: per chunk a block sum, per box the chunk sums in order, then per
// chunk the largest squared spread and per box its maximum.
__global__ void k_chunk_sum(const int* __restrict__ cbeg, const int* __restrict__ cend, int64_t n, int dim,
                            const double* __restrict__ xim, double* __restrict__ part)
{
    __shared__ double s[3][256];
    int c = blockIdx.x, t = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = cbeg[c] + t; i < cend[c]; i += blockDim.x)
        for (int d = 0; d < dim; ++d) acc[d] += xim[d * n + i];
    for (int d = 0; d < 3; ++d) s[d][t] = acc[d];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (t < st)
            for (int d = 0; d < 3; ++d) s[d][t] += s[d][t + st];
        __syncthreads();
    }
    if (t == 0)
        for (int d = 0; d < 3; ++d) part[3 * c + d] = s[d][0];
}

__global__ void k_box_mean(const int* __restrict__ coff, const int* __restrict__ pbeg,
                           const int* __restrict__ pend, int nbox, int dim, const double* __restrict__ part,
                           double* __restrict__ cim)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int c = coff[b]; c < coff[b + 1]; ++c)
        for (int d = 0; d < 3; ++d) acc[d] += part[3 * c + d];
    double inv = 1.0 / (double)(pend[b] - pbeg[b]);
    for (int d = 0; d < dim; ++d) cim[d * nbox + b] = acc[d] * inv;
}

__global__ void k_chunk_spread(const int* __restrict__ cbox, const int* __restrict__ cbeg,
                               const int* __restrict__ cend, int nbox, int64_t n, int dim,
                               const double* __restrict__ xim, const double* __restrict__ cim,
                               double* __restrict__ pmax)
{
    __shared__ double s[256];
    int c = blockIdx.x, t = threadIdx.x, b = cbox[c];
    double mean[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < dim; ++d) mean[d] = cim[d * nbox + b];
    double dm = 0.0;
    for (int i = cbeg[c] + t; i < cend[c]; i += blockDim.x) {
        double q = 0.0;
        for (int d = 0; d < dim; ++d) {
            double e = xim[d * n + i] - mean[d];
            q += e * e;
        }
        dm = fmax(dm, q);
    }
    s[t] = dm;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (t < st) s[t] = fmax(s[t], s[t + st]);
        __syncthreads();
    }
    if (t == 0) pmax[c] = s[0];
}

__global__ void k_box_delta(const int* __restrict__ coff, int nbox, const double* __restrict__ pmax,
                            double* __restrict__ delta)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    double m = 0.0;
    for (int c = coff[b]; c < coff[b + 1]; ++c) m = fmax(m, pmax[c]);
    delta[b] = sqrt(m);
}

// Flags a near pair (List 1) with Re r^2 <= 0 and r^2 != 0: the principal
// branch of the complexified distance is then not the continuation the
// expansions assume (the Lipschitz condition of Sec. 4.1 / 5.1 fails).
__global__ __launch_bounds__(64) void k_check_near(const int* __restrict__ leaves, const int* __restrict__ pbeg,
                                                   const int* __restrict__ pend, const int* __restrict__ l1off,
                                                   const int* __restrict__ l1idx, int64_t n, int dim,
                                                   const double* __restrict__ xre, const double* __restrict__ xim,
                                                   int* __restrict__ flag)
{
    // source tiles of 64 points staged in LDS (coalesced loads), read at one
    // address by the whole wavefront
    __shared__ double tre[3][64], tim[3][64];
    int b = leaves[blockIdx.x];
    int t = threadIdx.x;
    int bad = 0;
    for (int i0 = pbeg[b]; i0 < pend[b]; i0 += 64) {
        int i = i0 + t;
        bool ok = i < pend[b];
        double xr[3] = {0.0, 0.0, 0.0}, xi[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < dim; ++d)
            if (ok) {
                xr[d] = xre[d * n + i];
                xi[d] = xim[d * n + i];
            }
        for (int e = l1off[b]; e < l1off[b + 1]; ++e) {
            int a = l1idx[e];
            // List 1 is symmetric and s is the same for (i, j) and (j, i): each
            // unordered leaf pair is checked once, from its lower leaf
            if (a < b) continue;
            for (int j0 = pbeg[a]; j0 < pend[a]; j0 += 64) {
                int cnt = min(64, pend[a] - j0);
                __syncthreads();
                if (t < cnt)
                    for (int d = 0; d < dim; ++d) {
                        tre[d][t] = xre[d * n + j0 + t];
                        tim[d][t] = xim[d * n + j0 + t];
                    }
                __syncthreads();
                if (!ok) continue;
                for (int q = 0; q < cnt; ++q) {
                    double dr = xr[0] - tre[0][q], di = xi[0] - tim[0][q];
                    double sr = dr * dr - di * di, si = dr * di;
                    for (int d = 1; d < dim; ++d) {
                        dr = xr[d] - tre[d][q];
                        di = xi[d] - tim[d][q];
                        sr = fma(dr, dr, sr);
                        sr = fma(-di, di, sr);
                        si = fma(dr, di, si);
                    }
                    // s = 0 is allowed only for coincident points, which
                    // share a leaf (equal real parts, equal keys)
                    if (sr <= 0.0 && (a != b || !(sr == 0.0 && si == 0.0))) bad = 1;
                }
            }
        }
    }
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------- launchers
hipError_t launch_bbox(const double* pts, int64_t n, int dim, double* partial, int nb,
                       double* out, hipStream_t st)
{
    k_bbox_partial<<<nb, 256, 0, st>>>(pts, n, dim, partial);
    k_bbox_final<<<1, 256, 0, st>>>(partial, nb, dim, out);
    return hipGetLastError();
}

hipError_t launch_morton(const double* pts, int64_t n, int dim, const KeyParams& kp,
                         uint64_t* keys, int* idx, hipStream_t st)
{
    int nb = (int)((n + 255) / 256);
    k_morton<<<nb, 256, 0, st>>>(pts, n, dim, kp, keys, idx);
    return hipGetLastError();
}

static void scan_exclusive(unsigned* a, int64_t m, unsigned* tmp, hipStream_t st)
{
    int nb = (int)((m + 2047) / 2048);
    if (nb == 1) {
        k_scan_block<<<1, 256, 0, st>>>(a, m, nullptr);
        return;
    }
    k_scan_block<<<nb, 256, 0, st>>>(a, m, tmp);
    scan_exclusive(tmp, nb, tmp + nb, st);
    k_scan_add<<<nb, 256, 0, st>>>(a, m, tmp);
}

size_t scan_scratch_elems(int64_t m)
{
    int64_t tmp = 0, mm = m;
    while (mm > 2048) { mm = (mm + 2047) / 2048; tmp += mm; }
    return (size_t)tmp + 16;
}

void launch_scan_exclusive(unsigned* a, int64_t m, unsigned* tmp, hipStream_t st)
{
    scan_exclusive(a, m, tmp, st);
}

size_t radix_sort_scratch_bytes(int64_t n)
{
    int64_t nblk = (n + kRsTile - 1) / kRsTile;
    int64_t m = 256 * nblk;
    int64_t tmp = 0, mm = m;
    while (mm > 2048) { mm = (mm + 2047) / 2048; tmp += mm; }
    tmp += 16;
    return (size_t)(m + tmp) * sizeof(unsigned) + 256;
}

hipError_t launch_radix_sort(uint64_t* keys, int* vals, uint64_t* keys_alt, int* vals_alt,
                             int64_t n, int key_bits, void* scratch, hipStream_t st)
{
    int nblk = (int)((n + kRsTile - 1) / kRsTile);
    unsigned* hist = (unsigned*)scratch;
    unsigned* tmp = hist + (size_t)256 * nblk;
    uint64_t* ki = keys; int* vi = vals;
    uint64_t* ko = keys_alt; int* vo = vals_alt;
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        k_rs_hist<<<nblk, kRsThreads, 0, st>>>(ki, n, shift, hist, nblk);
        scan_exclusive(hist, (int64_t)256 * nblk, tmp, st);
        k_rs_scatter<<<nblk, kRsThreads, 0, st>>>(ki, vi, ko, vo, n, shift, hist, nblk);
        uint64_t* tk = ki; ki = ko; ko = tk;
        int* tv = vi; vi = vo; vo = tv;
    }
    if (ki != keys) {
        hipMemcpyAsync(keys, ki, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
        hipMemcpyAsync(vals, vi, n * sizeof(int), hipMemcpyDeviceToDevice, st);
    }
    return hipGetLastError();
}

hipError_t launch_gather_points(const double* pts, const int* perm, int64_t n, int dim,
                                double* xre, double* xim, hipStream_t st)
{
    k_gather_points<<<(int)((n + 255) / 256), 256, 0, st>>>(pts, perm, n, dim, xre, xim);
    return hipGetLastError();
}

hipError_t launch_gather_density(const double* sig, const IoMap& io, int64_t n, double* sre,
                                 double* sim, hipStream_t st)
{
    k_gather_density<<<(int)((n + 255) / 256), 256, 0, st>>>(sig, io, n, sre, sim);
    return hipGetLastError();
}

hipError_t launch_centres(const CentreChunks& ch, const int* pbeg, const int* pend, int nbox, int64_t n,
                          int dim, const double* xim, double* cim, double* delta, hipStream_t st)
{
    if (nbox <= 0 || ch.n <= 0) return hipSuccess;
    k_chunk_sum<<<ch.n, 256, 0, st>>>(ch.beg, ch.end, n, dim, xim, ch.part);
    k_box_mean<<<(nbox + 255) / 256, 256, 0, st>>>(ch.off, pbeg, pend, nbox, dim, ch.part, cim);
    k_chunk_spread<<<ch.n, 256, 0, st>>>(ch.box, ch.beg, ch.end, nbox, n, dim, xim, cim, ch.pmax);
    k_box_delta<<<(nbox + 255) / 256, 256, 0, st>>>(ch.off, nbox, ch.pmax, delta);
    return hipGetLastError();
}

hipError_t launch_check_near(const int* leaves, int nleaf, const int* pbeg, const int* pend,
                             const int* l1off, const int* l1idx, int64_t n, int dim,
                             const double* xre, const double* xim, int* flag, hipStream_t st)
{
    if (nleaf == 0) return hipSuccess;
    k_check_near<<<nleaf, 64, 0, st>>>(leaves, pbeg, pend, l1off, l1idx, n, dim, xre, xim, flag);
    return hipGetLastError();
}

}  // namespace cfmm
