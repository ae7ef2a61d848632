// Tree topology (Sec. 6.1) and Lists 1-4 (Sec. 6.2) on the device.
//
// Readings (the same as the host builder's):
//  * a box with more than N_s points splits into its non-empty children;
//  * near: ||c_a - c_b||_inf <= (k/2)(w_a + w_b), tested exactly in integer
//    units of the finest grid; boxes coarser than the top level of the far
//    field are near everything;
//  * level restriction: a leaf near a leaf two or more levels finer splits,
//    in passes until no such pair is left.
//
// Splitting is a pass over the points: every point carries the box that
// holds it, a point opens a child where its key prefix one level down changes
// inside a box that splits, an exclusive scan of those flags numbers the new
// children, and each point then moves to the last child opened at or before
// it.  The occupancy split runs one such pass per level; each level
// restriction pass marks the offending coarse leaves through a hash table of
// (level, prefix) -> box and splits them all at once.  Boxes are finally put
// in (level, first point) order by the radix sort, which is (level, prefix)
// order.
//
// Each list is counted per box, the counts scanned into offsets, the entries
// written per box as (box, entry) pairs and the pairs put in order by the
// radix sort, so every list is sorted by box index.  The neighbours of a box
// are found by looking up the coordinates around it:
//  * List 1 (leaf b at level l >= top): the leaves coarser than the top
//    level, and the geometrically near leaves of levels l - 1, l and l + 1
//    (the level restriction leaves no others); a leaf coarser than the top
//    level has every leaf in its List 1;
//  * List 2 (b, parent p): the children of p's colleagues not near b; when p
//    is coarser than the top level, every box of b's level not near b;
//  * List 3 (leaf b): by descent from b's colleagues through the boxes near
//    b, the children that are not near b;
//  * List 4: List 3 transposed.
#include "common.hpp"
#include "kernels.hpp"
#include "tree_device.hpp"

#include <algorithm>

namespace cfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kStack = 256;      // List 3 descent stack (at most 7 per level + 1)

inline int nblocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

// ------------------------------------------------------------ coordinates
__device__ inline void pre_coords(uint64_t p, int l, int dim, int64_t* q)
{
    q[0] = q[1] = q[2] = 0;
    for (int b = 0; b < l; ++b)
        for (int d = 0; d < dim; ++d) q[d] |= (int64_t)((p >> (b * dim + d)) & 1ull) << b;
}

__device__ inline uint64_t coords_pre(const int64_t* q, int l, int dim)
{
    uint64_t p = 0;
    for (int b = 0; b < l; ++b)
        for (int d = 0; d < dim; ++d) p |= (uint64_t)((q[d] >> b) & 1) << (b * dim + d);
    return p;
}

// geometric near test of a box at level la, coordinates qa and one at lb, qb
__device__ inline bool geo_near(int la, const int64_t* qa, int lb, const int64_t* qb, int dim, int B, int k)
{
    int64_t wa = (int64_t)1 << (B + 1 - la), wb = (int64_t)1 << (B + 1 - lb);
    for (int d = 0; d < dim; ++d) {
        int64_t ca = (2 * qa[d] + 1) << (B - la), cb = (2 * qb[d] + 1) << (B - lb);
        int64_t dd = ca > cb ? ca - cb : cb - ca;
        if (2 * dd > (int64_t)k * (wa + wb)) return false;
    }
    return true;
}

// ------------------------------------------------------------------- hash
// Key: the prefix with a marker bit above its dim * l bits, unique per
// (level, prefix) and never zero (zero marks an empty slot).  Slots by the
// 64-bit finaliser of MurmurHash3, linear probing; the table is kept at most
// half full.
__device__ inline uint64_t box_key(int l, uint64_t pre, int dim) { return pre | (1ull << (dim * l)); }

__device__ inline unsigned slot_of(uint64_t k, unsigned mask)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (unsigned)k & mask;
}

__device__ inline int find_box(const uint64_t* hk, const int* hv, unsigned mask, uint64_t k)
{
    unsigned s = slot_of(k, mask);
    for (unsigned it = 0; it <= mask; ++it) {
        uint64_t x = hk[s];
        if (x == k) return hv[s];
        if (x == 0ull) return -1;
        s = (s + 1) & mask;
    }
    return -1;
}

__global__ void k_hash_insert(int b0, int b1, const int* __restrict__ lev, const uint64_t* __restrict__ pre,
                              int dim, uint64_t* hk, int* hv, unsigned mask)
{
    int b = b0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= b1) return;
    uint64_t k = box_key(lev[b], pre[b], dim);
    unsigned s = slot_of(k, mask);
    for (unsigned it = 0; it <= mask; ++it) {
        unsigned long long prev = atomicCAS((unsigned long long*)&hk[s], 0ull, (unsigned long long)k);
        if (prev == 0ull || prev == k) {
            hv[s] = b;
            return;
        }
        s = (s + 1) & mask;
    }
}

__global__ void k_hash_remap(uint64_t* __restrict__ hk, int* __restrict__ hv, unsigned m,
                             const int* __restrict__ rank)
{
    unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < m && hk[s] != 0ull) hv[s] = rank[hv[s]];
}

template <class T>
__global__ void k_fill(T* __restrict__ a, int64_t n, T v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// ----------------------------------------------------------------- split
struct Boxes {
    int* lev;
    uint64_t* pre;
    int* pb;
    int* pe;
    int* par;
    int* first;
    int* nch;
    unsigned char* mark;
};

__global__ void k_root(Boxes bx, int64_t n)
{
    bx.lev[0] = 0; bx.pre[0] = 0; bx.pb[0] = 0; bx.pe[0] = (int)n;
    bx.par[0] = -1; bx.first[0] = -1; bx.nch[0] = 0; bx.mark[0] = 0;
}

// mode 0: occupancy (more than ns points, below the finest level); mode 1: marked
__device__ inline bool splits(const Boxes& bx, int b, int mode, int ns, int B)
{
    return mode == 0 ? (bx.pe[b] - bx.pb[b] > ns && bx.lev[b] < B) : bx.mark[b] != 0;
}

__global__ void k_split_flags(const uint64_t* __restrict__ keys, int64_t n, const int* __restrict__ pbox, Boxes bx,
                              int mode, int ns, int dim, int B, unsigned* __restrict__ flag,
                              unsigned* __restrict__ pos)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    unsigned f = 0;
    if (i < n) {
        int b = pbox[i];
        if (b >= 0 && splits(bx, b, mode, ns, B)) {
            int sh = dim * (B - bx.lev[b] - 1);
            f = (i == bx.pb[b] || (keys[i] >> sh) != (keys[i - 1] >> sh)) ? 1u : 0u;
        }
    }
    flag[i] = f;
    pos[i] = f;
}

__global__ void k_split_children(const uint64_t* __restrict__ keys, int64_t n, const int* __restrict__ pbox,
                                 const unsigned* __restrict__ flag, const unsigned* __restrict__ pos, int base,
                                 int dim, int B, Boxes bx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    int b = pbox[i];
    int c = base + (int)pos[i];
    int l = bx.lev[b] + 1;
    bx.lev[c] = l;
    bx.pre[c] = keys[i] >> (dim * (B - l));
    bx.pb[c] = (int)i;
    bx.par[c] = b;
    bx.first[c] = -1;
    bx.nch[c] = 0;
    bx.mark[c] = 0;
    if ((int)i == bx.pb[b]) bx.first[b] = c;
}

__global__ void k_split_close(int base, int cnt, Boxes bx)
{
    int c = base + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= base + cnt) return;
    int b = bx.par[c];
    bool last = c + 1 == base + cnt || bx.par[c + 1] != b;
    bx.pe[c] = last ? bx.pe[b] : bx.pb[c + 1];
    if (last) bx.nch[b] = c - bx.first[b] + 1;
}

// after an occupancy pass: each point to its child, or out of the active set
__global__ void k_split_move(int64_t n, int* __restrict__ pbox, const unsigned* __restrict__ flag,
                             const unsigned* __restrict__ pos, int base, Boxes bx, int ns, int B)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = pbox[i];
    if (b < 0) return;
    pbox[i] = (bx.pe[b] - bx.pb[b] > ns && bx.lev[b] < B) ? base + (int)(pos[i] + flag[i]) - 1 : -1;
}

// -------------------------------------------------------- level restriction
__global__ void k_has_leaf(int nbox, Boxes bx, int* __restrict__ hl)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox && bx.nch[b] == 0) hl[bx.lev[b]] = 1;
}

__global__ void k_marks(int nbox, Boxes bx, const int* __restrict__ hl, int dim, int B, int k,
                        const uint64_t* __restrict__ hk, const int* __restrict__ hv, unsigned mask)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox || bx.nch[b] != 0 || bx.lev[b] < 2) return;
    int l = bx.lev[b];
    int64_t qb[3];
    pre_coords(bx.pre[b], l, dim, qb);
    int side = 2 * k + 1, ncand = dim == 2 ? side * side : side * side * side;
    for (int lp = l - 2; lp >= 0; --lp) {
        if (!hl[lp]) continue;
        int64_t A[3] = {qb[0] >> (l - lp), qb[1] >> (l - lp), qb[2] >> (l - lp)};
        int64_t lim = ((int64_t)1 << lp) - 1;
        for (int q = 0; q < ncand; ++q) {
            int rem = q;
            int64_t cc[3] = {0, 0, 0};
            bool ok = true;
            for (int d = 0; d < dim; ++d) {
                cc[d] = A[d] + (rem % side) - k;
                rem /= side;
                if (cc[d] < 0 || cc[d] > lim) ok = false;
            }
            if (!ok) continue;
            int a = find_box(hk, hv, mask, box_key(lp, coords_pre(cc, lp, dim), dim));
            if (a >= 0 && bx.nch[a] == 0 && geo_near(lp, cc, l, qb, dim, B, k)) bx.mark[a] = 1;
        }
    }
}

__global__ void k_collect_marks(int nbox, Boxes bx, int* __restrict__ list, int* __restrict__ cnt)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox && bx.mark[b]) list[atomicAdd(cnt, 1)] = b;
}

__global__ void k_mark_points(const int* __restrict__ list, Boxes bx, int* __restrict__ pbox)
{
    int a = list[blockIdx.x];
    for (int i = bx.pb[a] + threadIdx.x; i < bx.pe[a]; i += blockDim.x) pbox[i] = a;
}

__global__ void k_clear_marks(const int* __restrict__ list, int m, Boxes bx)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) bx.mark[list[j]] = 0;
}

// -------------------------------------------------------- final numbering
__global__ void k_order_keys(int nbox, Boxes bx, uint64_t* __restrict__ key, int* __restrict__ val)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nbox) return;
    key[c] = ((uint64_t)bx.lev[c] << 32) | (uint64_t)(uint32_t)bx.pb[c];
    val[c] = c;
}

__global__ void k_rank(int nbox, const int* __restrict__ order, int* __restrict__ rank)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbox) rank[order[i]] = i;
}

__global__ void k_final(int nbox, const int* __restrict__ order, const int* __restrict__ rank, Boxes bx,
                        int* level, uint64_t* prefix, int* pbeg, int* pend, int* parent, int* child0, int* nchild)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbox) return;
    int c = order[i];
    level[i] = bx.lev[c];
    prefix[i] = bx.pre[c];
    pbeg[i] = bx.pb[c];
    pend[i] = bx.pe[c];
    nchild[i] = bx.nch[c];
    parent[i] = bx.par[c] >= 0 ? rank[bx.par[c]] : -1;
    child0[i] = bx.nch[c] > 0 ? rank[bx.first[c]] : -1;
}

// ------------------------------------------------------------------ lists
struct ListCtx {
    int dim, B, k, top, nbox;
    const int* level;
    const uint64_t* prefix;
    const int* child0;
    const int* nchild;
    const int* parent;
    const uint64_t* hk;
    const int* hv;
    unsigned mask;
    const int* lvl_beg;
    const int* leaves;
    int nleaf;
    const int* coarse;    // leaves coarser than the top level
    int ncoarse;
    int* overflow;        // set if a descent outgrows its stack
};

__device__ inline int lookup(const ListCtx& c, int l, const int64_t* q)
{
    return find_box(c.hk, c.hv, c.mask, box_key(l, coords_pre(q, l, c.dim), c.dim));
}

// visit f(a, qa) for the boxes at level l with coordinates within r of q
template <class F>
__device__ inline void around(const ListCtx& c, int l, const int64_t* q, int r, F f)
{
    int side = 2 * r + 1, ncand = c.dim == 2 ? side * side : side * side * side;
    int64_t lim = ((int64_t)1 << l) - 1;
    for (int t = 0; t < ncand; ++t) {
        int rem = t;
        int64_t cc[3] = {0, 0, 0};
        bool ok = true;
        for (int d = 0; d < c.dim; ++d) {
            cc[d] = q[d] + (rem % side) - r;
            rem /= side;
            if (cc[d] < 0 || cc[d] > lim) ok = false;
        }
        if (!ok) continue;
        int a = lookup(c, l, cc);
        if (a >= 0) f(a, cc);
    }
}

template <class E>
__device__ void list1(const ListCtx& c, int b, E& emit)
{
    if (c.nchild[b] != 0) return;
    int l = c.level[b];
    if (l < c.top) {
        for (int i = 0; i < c.nleaf; ++i) emit(c.leaves[i]);
        return;
    }
    for (int i = 0; i < c.ncoarse; ++i) emit(c.coarse[i]);
    int64_t qb[3];
    pre_coords(c.prefix[b], l, c.dim, qb);
    if (l - 1 >= c.top) {
        int64_t A[3] = {qb[0] >> 1, qb[1] >> 1, qb[2] >> 1};
        around(c, l - 1, A, c.k + 1, [&](int a, const int64_t* qa) {
            if (c.nchild[a] == 0 && geo_near(l - 1, qa, l, qb, c.dim, c.B, c.k)) emit(a);
        });
    }
    around(c, l, qb, c.k, [&](int a, const int64_t* qa) {
        if (!geo_near(l, qa, l, qb, c.dim, c.B, c.k)) return;
        if (c.nchild[a] == 0) {
            emit(a);
            return;
        }
        for (int ch = c.child0[a]; ch < c.child0[a] + c.nchild[a]; ++ch) {
            if (c.nchild[ch] != 0) continue;
            int64_t qc[3];
            pre_coords(c.prefix[ch], l + 1, c.dim, qc);
            if (geo_near(l + 1, qc, l, qb, c.dim, c.B, c.k)) emit(ch);
        }
    });
}

template <class E>
__device__ void list2(const ListCtx& c, int b, E& emit)
{
    int p = c.parent[b];
    int l = c.level[b];
    if (p < 0 || l < c.top) return;
    int64_t qb[3];
    pre_coords(c.prefix[b], l, c.dim, qb);
    if (c.level[p] < c.top) {
        for (int a = c.lvl_beg[l]; a < c.lvl_beg[l + 1]; ++a) {
            int64_t qa[3];
            pre_coords(c.prefix[a], l, c.dim, qa);
            if (!geo_near(l, qa, l, qb, c.dim, c.B, c.k)) emit(a);
        }
        return;
    }
    int64_t qp[3] = {qb[0] >> 1, qb[1] >> 1, qb[2] >> 1};
    around(c, l - 1, qp, c.k, [&](int a, const int64_t* qa) {
        if (!geo_near(l - 1, qa, l - 1, qp, c.dim, c.B, c.k)) return;
        for (int ch = c.child0[a]; ch < c.child0[a] + c.nchild[a]; ++ch) {
            int64_t qc[3];
            pre_coords(c.prefix[ch], l, c.dim, qc);
            if (!geo_near(l, qc, l, qb, c.dim, c.B, c.k)) emit(ch);
        }
    });
}

template <class E>
__device__ void list3(const ListCtx& c, int b, E& emit)
{
    if (c.nchild[b] != 0) return;
    int l = c.level[b];
    if (l < c.top) return;
    int64_t qb[3];
    pre_coords(c.prefix[b], l, c.dim, qb);
    int stack[kStack];
    around(c, l, qb, c.k, [&](int a, const int64_t* qa) {
        if (c.nchild[a] == 0 || !geo_near(l, qa, l, qb, c.dim, c.B, c.k)) return;
        int sp = 0;
        stack[sp++] = a;
        while (sp > 0) {
            int x = stack[--sp];
            int lc = c.level[x] + 1;
            for (int ch = c.child0[x]; ch < c.child0[x] + c.nchild[x]; ++ch) {
                int64_t qc[3];
                pre_coords(c.prefix[ch], lc, c.dim, qc);
                if (!geo_near(lc, qc, l, qb, c.dim, c.B, c.k)) {
                    emit(ch);
                } else if (c.nchild[ch] != 0) {
                    if (sp < kStack) stack[sp++] = ch;
                    else *c.overflow = 1;
                }
            }
        }
    });
}

// count (FILL = false) or write the (box, entry) pairs of list Q per box
template <int Q, bool FILL>
__global__ void k_list(ListCtx c, unsigned* __restrict__ cnt, const unsigned* __restrict__ off,
                       uint64_t* __restrict__ out, int s)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= c.nbox) return;
    unsigned k = 0;
    uint64_t hi = (uint64_t)b << s;
    size_t o = FILL ? off[b] : 0;
    auto emit = [&](int a) {
        if (FILL) out[o + k] = hi | (uint64_t)(uint32_t)a;
        ++k;
    };
    if (Q == 0) list1(c, b, emit);
    if (Q == 1) list2(c, b, emit);
    if (Q == 2) list3(c, b, emit);
    if (!FILL) cnt[b] = k;
}

// List 4 from the sorted List 3 pairs: swap the halves and count per entry box
__global__ void k_transpose(const uint64_t* __restrict__ p3, int64_t m, int s, uint64_t* __restrict__ p4,
                            unsigned* __restrict__ cnt4)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    uint64_t lo = p3[j] & ((1ull << s) - 1), hi = p3[j] >> s;
    p4[j] = (lo << s) | hi;
    atomicAdd(&cnt4[lo], 1u);
}

__global__ void k_extract(const uint64_t* __restrict__ p, int64_t m, int s, int* __restrict__ idx)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) idx[j] = (int)(p[j] & ((1ull << s) - 1));
}

__global__ void k_u2i(const unsigned* __restrict__ a, int64_t m, int* __restrict__ b)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) b[j] = (int)a[j];
}

int bits_for(int64_t v)
{
    int s = 1;
    while (((int64_t)1 << s) <= v) ++s;
    return s;
}

}  // namespace

// ------------------------------------------------------------------- host
template <class T>
hipError_t DeviceTree::grab(T** p, size_t count)
{
    void* q = nullptr;
    hipError_t e = hipMallocAsync(&q, (count ? count : 1) * sizeof(T), st_);
    if (e != hipSuccess) return e;
    mem_.push_back(q);
    *p = (T*)q;
    return hipSuccess;
}

void DeviceTree::release()
{
    for (void* q : mem_) (void)hipFreeAsync(q, st_);
    mem_.clear();
}

#define DTCHK(x)                                   \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return e_;           \
    } while (0)

hipError_t DeviceTree::grow_boxes(int need)
{
    if (need <= cap_) return hipSuccess;
    int cap = cap_ ? cap_ : 1024;
    while (cap < need) cap *= 2;
    int *lev, *pb, *pe, *par, *first, *nch;
    uint64_t* pre;
    unsigned char* mark;
    DTCHK(grab(&lev, cap)); DTCHK(grab(&pb, cap)); DTCHK(grab(&pe, cap)); DTCHK(grab(&par, cap));
    DTCHK(grab(&first, cap)); DTCHK(grab(&nch, cap)); DTCHK(grab(&pre, cap)); DTCHK(grab(&mark, cap));
    if (nbox_ > 0) {
        size_t m = nbox_;
        DTCHK(hipMemcpyAsync(lev, lev_, m * sizeof(int), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(pb, pb_, m * sizeof(int), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(pe, pe_, m * sizeof(int), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(par, par_, m * sizeof(int), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(first, first_, m * sizeof(int), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(nch, nch_, m * sizeof(int), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(pre, pre_, m * sizeof(uint64_t), hipMemcpyDeviceToDevice, st_));
        DTCHK(hipMemcpyAsync(mark, mark_, m, hipMemcpyDeviceToDevice, st_));
    }
    lev_ = lev; pb_ = pb; pe_ = pe; par_ = par; first_ = first; nch_ = nch; pre_ = pre; mark_ = mark;
    cap_ = cap;
    return hipSuccess;
}

// one split pass over the points; *added = the number of children made
hipError_t DeviceTree::split_pass(int mode, int, int* added)
{
    Boxes bx{lev_, pre_, pb_, pe_, par_, first_, nch_, mark_};
    k_split_flags<<<nblocks(n_ + 1), kThreads, 0, st_>>>(keys_, n_, pbox_, bx, mode, ns_, dim_, B_, flag_, pos_);
    launch_scan_exclusive(pos_, n_ + 1, scan_tmp_, st_);
    unsigned total = 0;
    DTCHK(hipMemcpyAsync(&total, pos_ + n_, sizeof(unsigned), hipMemcpyDeviceToHost, st_));
    DTCHK(hipStreamSynchronize(st_));
    *added = (int)total;
    if (total == 0) return hipGetLastError();
    int base = nbox_;
    DTCHK(grow_boxes(base + (int)total));
    bx = Boxes{lev_, pre_, pb_, pe_, par_, first_, nch_, mark_};
    k_split_children<<<nblocks(n_), kThreads, 0, st_>>>(keys_, n_, pbox_, flag_, pos_, base, dim_, B_, bx);
    k_split_close<<<nblocks(total), kThreads, 0, st_>>>(base, (int)total, bx);
    if (mode == 0) k_split_move<<<nblocks(n_), kThreads, 0, st_>>>(n_, pbox_, flag_, pos_, base, bx, ns_, B_);
    nbox_ = base + (int)total;
    return hipGetLastError();
}

hipError_t DeviceTree::sort_pairs(uint64_t* keys, int64_t m, int key_bits)
{
    if (m <= 1) return hipSuccess;
    uint64_t* kalt;
    int *v, *valt;
    unsigned char* scr;
    DTCHK(grab(&kalt, m)); DTCHK(grab(&v, m)); DTCHK(grab(&valt, m));
    DTCHK(grab(&scr, radix_sort_scratch_bytes(m)));
    k_fill<int><<<nblocks(m), kThreads, 0, st_>>>(v, m, 0);
    return launch_radix_sort(keys, v, kalt, valt, m, key_bits, scr, st_);
}

hipError_t DeviceTree::build(const uint64_t* keys, int64_t n, int dim, int B, int leaf_size, int sep,
                             hipStream_t st)
{
    release();
    st_ = st; keys_ = keys; n_ = n; dim_ = dim; B_ = B; ns_ = leaf_size; sep_ = sep;
    nbox_ = 0; cap_ = 0;
    DTCHK(grab(&pbox_, n)); DTCHK(grab(&flag_, n + 1)); DTCHK(grab(&pos_, n + 1));
    DTCHK(grab(&scan_tmp_, scan_scratch_elems(n + 1)));
    DTCHK(grab(&counter_, 64));
    int64_t cap0 = std::max<int64_t>(1024, 4 * (n / std::max(1, leaf_size)) + 64);
    DTCHK(grow_boxes((int)std::min<int64_t>(cap0, 1 << 30)));
    k_root<<<1, 1, 0, st_>>>(Boxes{lev_, pre_, pb_, pe_, par_, first_, nch_, mark_}, n);
    k_fill<int><<<nblocks(n), kThreads, 0, st_>>>(pbox_, n, 0);
    nbox_ = 1;
    // occupancy split, one level per pass
    for (int l = 0; l < B; ++l) {
        int added = 0;
        DTCHK(split_pass(0, l, &added));
        if (!added) break;
    }
    // level restriction to a fixed point
    unsigned hcap = 1024;
    int hashed = 0;
    int* hl = counter_ + 1;          // [32] levels holding a leaf
    int* mcnt = counter_;            // marked leaves
    int* mlist = nullptr;
    int mcap = 0;
    for (;;) {
        if ((unsigned)nbox_ * 2u > hcap || !hk_) {
            while ((unsigned)nbox_ * 2u > hcap) hcap *= 2;
            DTCHK(grab(&hk_, hcap)); DTCHK(grab(&hv_, hcap));
            hmask_ = hcap - 1;
            k_fill<uint64_t><<<nblocks(hcap), kThreads, 0, st_>>>(hk_, hcap, 0ull);
            hashed = 0;
        }
        if (hashed < nbox_)
            k_hash_insert<<<nblocks(nbox_ - hashed), kThreads, 0, st_>>>(hashed, nbox_, lev_, pre_, dim_, hk_, hv_,
                                                                         hmask_);
        hashed = nbox_;
        Boxes bx{lev_, pre_, pb_, pe_, par_, first_, nch_, mark_};
        k_fill<int><<<1, 64, 0, st_>>>(counter_, 33, 0);
        k_has_leaf<<<nblocks(nbox_), kThreads, 0, st_>>>(nbox_, bx, hl);
        k_marks<<<nblocks(nbox_), kThreads, 0, st_>>>(nbox_, bx, hl, dim_, B_, sep_, hk_, hv_, hmask_);
        if (mcap < nbox_) {
            mcap = 2 * nbox_;
            DTCHK(grab(&mlist, mcap));
        }
        k_collect_marks<<<nblocks(nbox_), kThreads, 0, st_>>>(nbox_, bx, mlist, mcnt);
        int m = 0;
        DTCHK(hipMemcpyAsync(&m, mcnt, sizeof(int), hipMemcpyDeviceToHost, st_));
        DTCHK(hipStreamSynchronize(st_));
        if (m == 0) break;
        k_fill<int><<<nblocks(n), kThreads, 0, st_>>>(pbox_, n, -1);
        k_mark_points<<<m, kThreads, 0, st_>>>(mlist, bx, pbox_);
        int added = 0;
        DTCHK(split_pass(1, 0, &added));
        bx = Boxes{lev_, pre_, pb_, pe_, par_, first_, nch_, mark_};
        k_clear_marks<<<nblocks(m), kThreads, 0, st_>>>(mlist, m, bx);
    }
    // final (level, prefix) numbering
    uint64_t* okey;
    int *order, *rank;
    DTCHK(grab(&okey, nbox_)); DTCHK(grab(&order, nbox_)); DTCHK(grab(&rank, nbox_));
    uint64_t* kalt;
    int* valt;
    unsigned char* scr;
    DTCHK(grab(&kalt, nbox_)); DTCHK(grab(&valt, nbox_)); DTCHK(grab(&scr, radix_sort_scratch_bytes(nbox_)));
    Boxes bx{lev_, pre_, pb_, pe_, par_, first_, nch_, mark_};
    k_order_keys<<<nblocks(nbox_), kThreads, 0, st_>>>(nbox_, bx, okey, order);
    DTCHK(launch_radix_sort(okey, order, kalt, valt, nbox_, 40, scr, st_));
    k_rank<<<nblocks(nbox_), kThreads, 0, st_>>>(nbox_, order, rank);
    DTCHK(grab(&f_level_, nbox_)); DTCHK(grab(&f_prefix_, nbox_)); DTCHK(grab(&f_pbeg_, nbox_));
    DTCHK(grab(&f_pend_, nbox_)); DTCHK(grab(&f_parent_, nbox_)); DTCHK(grab(&f_child0_, nbox_));
    DTCHK(grab(&f_nchild_, nbox_));
    k_final<<<nblocks(nbox_), kThreads, 0, st_>>>(nbox_, order, rank, bx, f_level_, f_prefix_, f_pbeg_, f_pend_,
                                                  f_parent_, f_child0_, f_nchild_);
    k_hash_remap<<<nblocks(hcap), kThreads, 0, st_>>>(hk_, hv_, hcap, rank);
    return hipGetLastError();
}

hipError_t DeviceTree::export_topology(int* level, int* parent, int* child0, int* nchild, int* pbeg, int* pend,
                                       std::vector<int32_t>& h_level, std::vector<int32_t>& h_parent,
                                       std::vector<int32_t>& h_child0, std::vector<int32_t>& h_nchild,
                                       std::vector<int32_t>& h_pbeg, std::vector<int32_t>& h_pend,
                                       std::vector<uint64_t>& h_prefix)
{
    size_t m = nbox_, b4 = m * sizeof(int);
    const int* src[6] = {f_level_, f_parent_, f_child0_, f_nchild_, f_pbeg_, f_pend_};
    int* dst[6] = {level, parent, child0, nchild, pbeg, pend};
    std::vector<int32_t>* hst[6] = {&h_level, &h_parent, &h_child0, &h_nchild, &h_pbeg, &h_pend};
    for (int k = 0; k < 6; ++k) {
        if (dst[k]) DTCHK(hipMemcpyAsync(dst[k], src[k], b4, hipMemcpyDeviceToDevice, st_));
        hst[k]->resize(m);
        DTCHK(hipMemcpyAsync(hst[k]->data(), src[k], b4, hipMemcpyDeviceToHost, st_));
    }
    h_prefix.resize(m);
    DTCHK(hipMemcpyAsync(h_prefix.data(), f_prefix_, m * sizeof(uint64_t), hipMemcpyDeviceToHost, st_));
    return hipStreamSynchronize(st_);
}

hipError_t DeviceTree::count_lists(int top, const std::vector<int32_t>& lvl_beg, int64_t cnt[4])
{
    top_ = top;
    std::vector<int32_t> h_nchild(nbox_), h_level(nbox_);
    DTCHK(hipMemcpyAsync(h_nchild.data(), f_nchild_, nbox_ * sizeof(int), hipMemcpyDeviceToHost, st_));
    DTCHK(hipMemcpyAsync(h_level.data(), f_level_, nbox_ * sizeof(int), hipMemcpyDeviceToHost, st_));
    DTCHK(hipStreamSynchronize(st_));
    std::vector<int32_t> leaves, coarse;
    for (int b = 0; b < nbox_; ++b)
        if (h_nchild[b] == 0) {
            leaves.push_back(b);
            if (h_level[b] < top) coarse.push_back(b);
        }
    nleaf_ = (int)leaves.size();
    ncoarse_ = (int)coarse.size();
    DTCHK(grab(&leaves_, leaves.size())); DTCHK(grab(&coarse_, coarse.size()));
    DTCHK(grab(&lvl_beg_d_, lvl_beg.size()));
    DTCHK(hipMemcpyAsync(leaves_, leaves.data(), leaves.size() * sizeof(int), hipMemcpyHostToDevice, st_));
    if (!coarse.empty())
        DTCHK(hipMemcpyAsync(coarse_, coarse.data(), coarse.size() * sizeof(int), hipMemcpyHostToDevice, st_));
    DTCHK(hipMemcpyAsync(lvl_beg_d_, lvl_beg.data(), lvl_beg.size() * sizeof(int), hipMemcpyHostToDevice, st_));
    ListCtx c{dim_, B_, sep_, top, nbox_, f_level_, f_prefix_, f_child0_, f_nchild_, f_parent_, hk_, hv_, hmask_,
              lvl_beg_d_, leaves_, nleaf_, coarse_, ncoarse_, counter_};
    k_fill<int><<<1, 64, 0, st_>>>(counter_, 1, 0);
    for (int q = 0; q < 4; ++q) DTCHK(grab(&lcnt_[q], (size_t)nbox_ + 1));
    int nb = nblocks(nbox_);
    k_list<0, false><<<nb, kThreads, 0, st_>>>(c, lcnt_[0], nullptr, nullptr, 0);
    k_list<1, false><<<nb, kThreads, 0, st_>>>(c, lcnt_[1], nullptr, nullptr, 0);
    k_list<2, false><<<nb, kThreads, 0, st_>>>(c, lcnt_[2], nullptr, nullptr, 0);
    unsigned* tmp;
    DTCHK(grab(&tmp, scan_scratch_elems(nbox_ + 1)));
    unsigned tot[3] = {0, 0, 0};
    for (int q = 0; q < 3; ++q) {
        k_fill<unsigned><<<1, 64, 0, st_>>>(lcnt_[q] + nbox_, 1, 0u);
        launch_scan_exclusive(lcnt_[q], nbox_ + 1, tmp, st_);
        DTCHK(hipMemcpyAsync(&tot[q], lcnt_[q] + nbox_, sizeof(unsigned), hipMemcpyDeviceToHost, st_));
    }
    int ovf = 0;
    DTCHK(hipMemcpyAsync(&ovf, counter_, sizeof(int), hipMemcpyDeviceToHost, st_));
    DTCHK(hipStreamSynchronize(st_));
    if (ovf) return hipErrorIllegalState;
    for (int q = 0; q < 3; ++q) cnt[q] = lsize_[q] = tot[q];
    cnt[3] = lsize_[3] = tot[2];
    return hipGetLastError();
}

hipError_t DeviceTree::fill_lists(int* const off[4], int* const idx[4], std::vector<int32_t> h_off[4],
                                  std::vector<int32_t> h_idx[4])
{
    ListCtx c{dim_, B_, sep_, top_, nbox_, f_level_, f_prefix_, f_child0_, f_nchild_, f_parent_, hk_, hv_, hmask_,
              lvl_beg_d_, leaves_, nleaf_, coarse_, ncoarse_, counter_};
    int s = bits_for(nbox_);
    int nb = nblocks(nbox_);
    uint64_t* pairs[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int q = 0; q < 4; ++q) DTCHK(grab(&pairs[q], (size_t)std::max<int64_t>(lsize_[q], 1)));
    k_list<0, true><<<nb, kThreads, 0, st_>>>(c, nullptr, lcnt_[0], pairs[0], s);
    k_list<1, true><<<nb, kThreads, 0, st_>>>(c, nullptr, lcnt_[1], pairs[1], s);
    k_list<2, true><<<nb, kThreads, 0, st_>>>(c, nullptr, lcnt_[2], pairs[2], s);
    for (int q = 0; q < 3; ++q) DTCHK(sort_pairs(pairs[q], lsize_[q], 2 * s));
    // List 4 = List 3 transposed
    k_fill<unsigned><<<nblocks(nbox_ + 1), kThreads, 0, st_>>>(lcnt_[3], nbox_ + 1, 0u);
    if (lsize_[2] > 0)
        k_transpose<<<nblocks(lsize_[2]), kThreads, 0, st_>>>(pairs[2], lsize_[2], s, pairs[3], lcnt_[3]);
    unsigned* tmp;
    DTCHK(grab(&tmp, scan_scratch_elems(nbox_ + 1)));
    launch_scan_exclusive(lcnt_[3], nbox_ + 1, tmp, st_);
    DTCHK(sort_pairs(pairs[3], lsize_[3], 2 * s));
    for (int q = 0; q < 4; ++q) {
        k_u2i<<<nblocks(nbox_ + 1), kThreads, 0, st_>>>(lcnt_[q], nbox_ + 1, off[q]);
        if (lsize_[q] > 0) k_extract<<<nblocks(lsize_[q]), kThreads, 0, st_>>>(pairs[q], lsize_[q], s, idx[q]);
        h_off[q].resize(nbox_ + 1);
        h_idx[q].resize(lsize_[q]);
        DTCHK(hipMemcpyAsync(h_off[q].data(), off[q], (nbox_ + 1) * sizeof(int), hipMemcpyDeviceToHost, st_));
        if (lsize_[q] > 0)
            DTCHK(hipMemcpyAsync(h_idx[q].data(), idx[q], lsize_[q] * sizeof(int), hipMemcpyDeviceToHost, st_));
    }
    int ovf = 0;
    DTCHK(hipMemcpyAsync(&ovf, counter_, sizeof(int), hipMemcpyDeviceToHost, st_));
    DTCHK(hipStreamSynchronize(st_));
    if (ovf) return hipErrorIllegalState;
    return hipGetLastError();
}

}  // namespace cfmm
