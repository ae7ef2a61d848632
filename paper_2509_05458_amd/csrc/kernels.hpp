// Launch interfaces of the cfmm kernels (host side).
#pragma once
#include "common.hpp"

namespace cfmm {

constexpr int kRsThreads = 256;
constexpr int kRsRounds = 8;
constexpr int kRsTile = kRsThreads * kRsRounds;

struct KeyParams {
    double lo[3];
    double scale;   // 2^B / D
    double top;     // 2^B - 1
};

// tree construction (tree_kernels.hip)
hipError_t launch_bbox(const double* pts, int64_t n, int dim, double* partial, int nb,
                       double* out, hipStream_t st);
hipError_t launch_morton(const double* pts, int64_t n, int dim, const KeyParams& kp,
                         uint64_t* keys, int* idx, hipStream_t st);
size_t radix_sort_scratch_bytes(int64_t n);
// in-place exclusive scan of m unsigned values; tmp holds scan_scratch_elems(m)
size_t scan_scratch_elems(int64_t m);
void launch_scan_exclusive(unsigned* a, int64_t m, unsigned* tmp, hipStream_t st);
hipError_t launch_radix_sort(uint64_t* keys, int* vals, uint64_t* keys_alt, int* vals_alt,
                             int64_t n, int key_bits, void* scratch, hipStream_t st);
hipError_t launch_gather_points(const double* pts, const int* perm, int64_t n, int dim,
                                double* xre, double* xim, hipStream_t st);
// Caller order <-> sorted tree order.  Tree points are the sources
// (0 .. nsrc-1), then the distinct targets; obase is the tree index of the
// first target (0 when the targets are the sources).  A final pass that writes
// a non-finite potential sets *nonfinite.
struct IoMap {
    const int* perm;       // sorted position -> tree point index
    int64_t nsrc;
    int64_t obase;
    int* nonfinite;
};
hipError_t launch_gather_density(const double* sig, const IoMap& io, int64_t n, double* sre,
                                 double* sim, hipStream_t st);
// Boxes cut into chunks of at most kCentreChunk points for the centre pass.
constexpr int kCentreChunk = 4096;
struct CentreChunks {
    int n;                 // chunks
    const int* box;        // [n] owning box
    const int* beg;        // [n] point range
    const int* end;
    const int* off;        // [nbox + 1] chunks of each box
    double* part;          // [3 n] scratch: per-chunk sums
    double* pmax;          // [n] scratch: per-chunk largest squared spread
};
hipError_t launch_centres(const CentreChunks& ch, const int* pbeg, const int* pend, int nbox, int64_t n,
                          int dim, const double* xim, double* cim, double* delta, hipStream_t st);
hipError_t launch_check_near(const int* leaves, int nleaf, const int* pbeg, const int* pend,
                             const int* l1off, const int* l1idx, int64_t n, int dim,
                             const double* xre, const double* xim, int* flag, hipStream_t st);

// Device views shared by the evaluation kernels.
struct TreeView {
    int nbox;
    const int* pbeg;
    const int* pend;
    const int* level;
    const int* parent;
    const int* child0;
    const int* nchild;
    const double* cre;     // centre real parts, [d * nbox + b]
    const double* cim;     // centre imaginary parts
    const int* eoff;       // expansion offset (complex units) per box, -1 if none
    const int* P;          // expansion length per level
    const double* rs;      // expansion scaling per level
    const int* l1off; const int* l1idx;
    const int* l2off; const int* l2idx;
    const int* l3off; const int* l3idx;
    const int* l4off; const int* l4idx;
};

// M2P by List-3 entries (3D): per entry its owner leaf and the offset of its
// per-point partial sums.
struct M2PParts {
    int n;                 // List-3 entries
    const int* owner;      // [n]
    const int64_t* poff;   // [n + 1]
    cplx* part;            // [poff[n]]
};

struct PointsView {
    int64_t n;
    const double* xre;     // [d * n + i], sorted order
    const double* xim;
    const double* sre;     // densities, sorted order
    const double* sim;
};

// Plan-time operator tables of the 2D Helmholtz translations.
constexpr int kPwStride = 4 * 64;          // per-level powers r^e, e < kPwStride
struct H2DOps {
    const cplx* g_m2l;      // per List-2 entry: 4P+1 generator values, k = -2P..2P
    const int64_t* o_m2l;   // offset of each entry's generator
    const cplx* g_m2m;      // per box: 2K+1 values, K = P(parent) + P(box)
    const cplx* g_l2l;
    const int64_t* o_tr;    // per box offset into g_m2m / g_l2l (-1 if none)
    const double* pw;       // pw[l * kPwStride + e] = r_l^e
    const int* m2l_src;     // per List-2 entry: expansion offset of the source box
};

// 2D Helmholtz evaluation (h2d_kernels.hip)
hipError_t h2d_init_tables(int device);
hipError_t h2d_gen_ops(const int* pair_b, int npairs, const int* tr_boxes, int ntr,
                       const TreeView& tv, double kappa, int lwin, const int64_t* o_m2l, cplx* g_m2l,
                       const int64_t* o_tr, cplx* g_m2m, cplx* g_l2l, hipStream_t st);
hipError_t h2d_p2m(const int* leaves, int nleaf, int pmax, const TreeView& tv, const PointsView& pv,
                   double kappa, cplx* mpole, hipStream_t st);
hipError_t h2d_m2m(const int* boxes, int nb, int ncoef, const TreeView& tv, const H2DOps& ops, cplx* mpole,
                   hipStream_t st);
// M2L: boxes[0 .. nwin) grouped by grp (first box, count) for the window
// kernel, boxes[nwin .. total) by the scaled kernel
int h2d_m2l_w_slots(int P);
int h2d_m2l_w_waves();
size_t h2d_m2l_w_lds(int P, int W);
hipError_t h2d_m2l(const int* boxes, const int2* grp, int ngrp1, int ngrp, size_t lds1, size_t ldsw, int nwin,
                   int total, const TreeView& tv, const H2DOps& ops, const cplx* mpole, cplx* local,
                   hipStream_t st);
hipError_t h2d_p2l(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   double kappa, cplx* local, hipStream_t st);
hipError_t h2d_l2l(const int* boxes, int nb, int ncoef, const TreeView& tv, const H2DOps& ops, cplx* local,
                   hipStream_t st);
hipError_t h2d_leaf_far(const int* leaves, int nleaf, const M2PParts& m2p, int m2p_pmax, int top,
                        const TreeView& tv, const PointsView& pv, double kappa, const cplx* mpole,
                        const cplx* local, cplx* ufar, hipStream_t st);
// Near-field work of the 2D Helmholtz plan: List-1 entries as work items
// (symmetric pair items, series row items, general row items) and the
// partial-sum buffer C they write.
struct H2DNear {
    const int* sym; const int* sym_k; int nsym;
    const int* diag; const int* diag_k; int ndiag;
    const int* ser; const int* ser_k; int nser;
    const int* gen; int ngen;
    const int* row_of; const int* partner; const int64_t* coff; cplx* C;
};
// laplace = 1: the 2D Laplace near field (Log s by every item kind; no
// general items), final constant -(1/4 pi) instead of (i/4)
hipError_t h2d_p2p(const H2DNear& nr, const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv,
                   double kappa, const cplx* ufar, const IoMap& io, double* out, int laplace, hipStream_t st);

// 2D Laplace evaluation (l2d_kernels.hip): expansions of 2P+1 values per box
// (two power series, in z = x1 + i x2 and w = x1 - i x2), P the same on
// every level, tv.rs[l] = 1 / w_l
hipError_t l2d_init_tables(int device);
hipError_t l2d_p2m(const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv, cplx* mpole,
                   hipStream_t st);
hipError_t l2d_m2m(const int* boxes, int nb, const TreeView& tv, cplx* mpole, hipStream_t st);
hipError_t l2d_m2l(const int* boxes, int nb, const TreeView& tv, const cplx* mpole, cplx* local, hipStream_t st);
hipError_t l2d_p2l(const int* boxes, int nb, const TreeView& tv, const PointsView& pv, cplx* local,
                   hipStream_t st);
hipError_t l2d_l2l(const int* boxes, int nb, const TreeView& tv, cplx* local, hipStream_t st);
hipError_t l2d_leaf_far(const int* leaves, int nleaf, const M2PParts& m2p, int top, const TreeView& tv,
                        const PointsView& pv, const cplx* mpole, const cplx* local, cplx* ufar, hipStream_t st);

// 3D Laplace evaluation (l3d_kernels.hip); P is the common expansion length
hipError_t l3d_p2m(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   cplx* mpole, hipStream_t st);
hipError_t l3d_p2l(const int* boxes, int nb, int P, const TreeView& tv, const PointsView& pv,
                   cplx* local, hipStream_t st);
// M2M into the nb parents `boxes` from all their children; L2L from the nb
// parents `parents` into all their children
hipError_t l3d_m2m(const int* boxes, int nb, int P, const TreeView& tv, cplx* mpole, hipStream_t st);
// Source expansion length of an M2L pair by the max-norm distance d of the
// box centres in box widths: p[min(d, 7)] (Sec. 6.3's rule with the pair's
// own nearest target distance (d - 1/2) w in place of (k + 1/2) w).
struct L3PairP {
    int p[8];
    // point-and-shoot M2L: the expansion length P (0: off) and the bound
    // P ln(K^2) <= pns_logb on the pair's phases, K the largest of
    // |e^{+-ia}|, |e^{+-ib}|
    int pns_P;
    double pns_logb;
};
// The table constants of every List-2 pair of the boxes (5 complex per entry)
// and its source expansion length, formed once per plan; rows64 / rows32: per
// source length Ps the rows n <= Ps each wavefront of the FP64 (4 waves) or
// FP32 (2 waves) M2L contracts, as bit masks [Ps * W + w].
struct L3Pairs {
    const cplx* c;         // [5 * n_list2]
    const int* ps;         // [n_list2]
    const int* src;        // [n_list2] expansion offset of the source box
    const unsigned* rows64;
    const unsigned* rows32;
};
// wavefronts per workgroup of the FP64 (fp32 = 0) or FP32 M2L
int l3d_m2l_waves(int fp32);
hipError_t l3d_m2l_pairs(const int* boxes, int nb, const TreeView& tv, const L3PairP& pp, cplx* c, int* ps,
                         int* src, hipStream_t st);
// The direct-form M2L over the pairs with ps >= 0 (the others are left to
// l3d_m2l_pns): writes the boxes' locals, or adds to them with accum.
hipError_t l3d_m2l(const int* boxes, int nb, int P, const TreeView& tv, const int* map, int ntab, int R,
                   const L3Pairs& pr, int mixed, int accum, const cplx* mpole, cplx* local, hipStream_t st);
// The point-and-shoot M2L over the pairs with ps < 0 (P <= l3d_pns_max_p()),
// listed per box b as ent[off[b] .. off[b+1]-1] = (List-2 entry, source
// expansion offset, Ps, 0): writes the boxes' locals (zero for a box with no
// such pair).
int l3d_pns_max_p();
hipError_t l3d_m2l_pns(const int* boxes, int nb, int P, const TreeView& tv, const cplx* pc, const int* off,
                       const int4* ent, const cplx* mpole, cplx* local, hipStream_t st);
hipError_t l3d_l2l(const int* parents, int nb, int P, const TreeView& tv, cplx* local, hipStream_t st);
hipError_t l3d_leaf_far(const int* leaves, int nleaf, int top, const TreeView& tv,
                        const PointsView& pv, const cplx* mpole, const cplx* local, const M2PParts& m2p,
                        cplx* ufar, hipStream_t st);
size_t l3d_m2l_lds(int P, int ntab);
// Layer potentials (3D Laplace): dipoles v in sorted SoA dre/dim [3][n];
// P2M (irregular = 0) or P2L over List 4 (irregular = 1) with charges and
// dipoles; L2P + M2P with gradients (m2p4: 4 complex per point per List-3
// entry); the near field by target leaf, writing pot[n_out] and
// grad[n_out][3] (either may be NULL) with the far field and 1/(4 pi).
hipError_t l3d_p2x_dip(const int* boxes, int nb, int P, int irregular, const TreeView& tv, const PointsView& pv,
                       const double* dre, const double* dim, cplx* out, hipStream_t st);
hipError_t l3d_leaf_far_grad(const int* leaves, int nleaf, int top, const TreeView& tv, const PointsView& pv,
                             const cplx* mpole, const cplx* local, const M2PParts& m2p4, cplx* ufar, cplx* gfar,
                             hipStream_t st);
hipError_t l3d_near_layer(const int* leaves, int nleaf, const TreeView& tv, const PointsView& pv, const double* dre,
                          const double* dim, int has_dip, const cplx* ufar, const cplx* gfar, const IoMap& io,
                          double* pot, double* grad, hipStream_t st);
hipError_t launch_gather_dipole(const double* dip, const IoMap& io, int64_t n, double* dre, double* dim,
                                hipStream_t st);
int l3d_pmax_supported();

// 3D Helmholtz evaluation (h3d_kernels.hip)
struct H3DLevels {
    const double* kw;      // kappa * w_l per level
    const double* sc;      // min(1, kappa * w_l)
    const void* rec;       // column recurrence table (set by the launchers)
};

// One chunk of a translation stage (M2M, M2L or L2L at one level): its pairs,
// the per-stage constants and the scratch regions (per-pair strides in
// complex units).
struct H3DTr {
    int np;                 // pairs in the chunk
    const int* src;         // source box per pair
    const int* dst;         // target box per pair
    int Ps, Pt, nq;         // source / target expansion lengths, coaxial nodes
    int src_h, trg_h;       // 1: singular (multipole) expansion, 0: regular (local)
    int f32;                // 1: rotation sampling in FP32 (mixed-precision M2L)
    const void* rec;        // column recurrence tables, FP64 and FP32 (set by h3d_translate)
    const void* recf;
    double ks, sc;          // kappa w_src and the source level's scale
    double rs;              // coaxial sampling radius / w_src
    double inv_w;           // 1 / w_src
    const double* sth;      // sin t_j, cos t_j of the Gauss-Legendre nodes
    const double* cth;
    const double* W;        // [(n(n+1)/2 + m) * nq + j] = (2n+1)/2 w_j S_n^m(s_j)
    const cplx* Tc;         // conj(T_n) / (|T_n|^2 + |T'_n|^2)
    const cplx* Tdc;        // conj(T'_n) / (|T_n|^2 + |T'_n|^2)
    cplx* geo;  // [np][10]: Q (row major), rho_D
    cplx* FG;  int64_t sFG;
    cplx* A;   int64_t sA;
    cplx* R;   int64_t sR;
    cplx* B;   int64_t sB;
};

hipError_t h3d_init_tables(int device);
hipError_t l3d_init_tables(int device);
hipError_t h3d_p2m(const int* boxes, int nb, int pmax, const TreeView& tv, const PointsView& pv,
                   const H3DLevels& hl, cplx* mpole, hipStream_t st);
hipError_t h3d_p2l(const int* boxes, int nb, int pmax, const TreeView& tv, const PointsView& pv,
                   const H3DLevels& hl, cplx* local, hipStream_t st);
hipError_t h3d_leaf_far(const int* leaves, int nleaf, int top, int pmax, const TreeView& tv,
                        const PointsView& pv, const H3DLevels& hl, const cplx* mpole,
                        const cplx* local, const M2PParts& m2p, cplx* ufar, hipStream_t st);
hipError_t h3d_translate(const H3DTr& tr, const TreeView& tv, const int* eoff_src, const cplx* coef_src,
                         const int* gdst, const int* goff, int ng, const int* eoff_dst, cplx* coef_dst,
                         const double* eq_p0, const double* eq_d0, hipStream_t st);

// 3D near field by List-1 entries (near3d.hip)
struct Near3Map {
    const int* row_of;      // target leaf of each List-1 entry
    const int* partner;     // entry (a, b) for entry (b, a)
    const int64_t* coff;    // offset of each entry's partial sums in C
    cplx* C;
};
struct Near3Work {
    const int* items[4];    // neighbour, diagonal, neighbour (wide phase), diagonal (wide phase)
    int nitems[4];
    const int* row_of; const int* partner; const int64_t* coff; cplx* C;
};
hipError_t near3_p2p(const Near3Work& w, int kernel, int mixed, const int* leaves, int nleaf, const TreeView& tv,
                     const PointsView& pv, double kappa, const cplx* ufar, const IoMap& io, double* out,
                     hipStream_t st);

// Static staging of cfmm_eval_static (scratch.hip): kStaticScratch complex
// values per device, resolved once per device with that device current.
constexpr int64_t kStaticScratch = (int64_t)1 << 22;
hipError_t static_scratch_init(int device);
cplx* static_scratch(int device);

// host-side special functions for the expansion-length rule
double h2d_nterms_crit(double kappa, double R, double r, int n);

}  // namespace cfmm
