/*
 * cfmm -- complex-coordinate fast multipole method on MI355X (gfx950).
 *
 * Evaluates the discrete single-layer sum of the complex-coordinate FMM
 * paper (Sec. 2.3, the M-body sum)
 *
 *     u(x_i) = sum_j G(x_i, y_j) sigma_j ,   i = 0 .. n_trg-1,  j = 0 .. n_src-1
 *
 * at complex targets x and sources y in C^d, with the complexified distance
 * r = sqrt(sum_d (x_{i,d} - y_{j,d})^2) on the principal branch (Sec. 2.1;
 * complex polar / spherical coordinates of Sec. 3.1).  When no targets are
 * given, the targets are the sources and the self term j = i is left out.
 * A pair at squared distance exactly 0 contributes nothing.  Kernels:
 *
 *     dim 2, CFMM_LAPLACE   :  G = -(1/(2 pi)) log r           (Sec. 4.2)
 *     dim 2, CFMM_HELMHOLTZ :  G = (i/4) H0^(1)(kappa r)        (Sec. 4.3)
 *     dim 3, CFMM_LAPLACE   :  G = 1 / (4 pi r)                 (Sec. 5.2)
 *     dim 3, CFMM_HELMHOLTZ :  G = exp(i kappa r) / (4 pi r)    (Sec. 5.3)
 *
 * The method (Sec. 6): an adaptive level-restricted tree on the real parts of
 * the points (sources and targets together, a Morton sort), complexified box
 * centres, Lists 1-4, and the eight FMM steps (P2M, M2M, P2P, M2L, M2P, P2L,
 * L2L, L2P) with analytically continued expansions.  Everything on the hot
 * path runs as HIP kernels.
 *
 * Geometry: the imaginary parts must be a Lipschitz function of the real
 * parts with constant L < 1 (Sec. 4.1, Sec. 5.1); the configurations this
 * library is validated on have L <= 0.5.
 *
 * Memory: all arrays are owned by the caller.  Complex values are complex128
 * (interleaved re, im doubles, the numpy / torch layout).  A plan copies the
 * points, so the caller may free them once cfmm_plan returns.  cfmm_eval only
 * borrows density and potential until the work it enqueued completes
 * (call cfmm_sync or synchronise the stream).
 *
 * Errors: every function returns 0 on success or a negative CFMM_E* code;
 * nothing throws across this interface.  cfmm_last_error() returns a message
 * for the calling thread's last failure.
 *
 * Threading: one plan is used by one stream at a time; distinct plans may run
 * concurrently.  Given the same plan and density, cfmm_eval is bitwise
 * reproducible (no floating-point atomics).
 */
#ifndef CFMM_H
#define CFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFMM_OK 0
#define CFMM_EINVAL (-1)     /* bad dim / kernel / kappa / tol / precision / n / pointer */
#define CFMM_ENOTSUP (-2)    /* not supported: boxes so many wavelengths wide that the
                                expansion length exceeds the maximum */
#define CFMM_EGEOMETRY (-3)  /* non-finite coordinates, or Re r^2 <= 0 in a near pair */
#define CFMM_ENOMEM (-4)     /* device allocation failed */
#define CFMM_EHIP (-5)       /* a HIP runtime call failed (message has the HIP error) */
#define CFMM_ERANGE (-6)     /* an evaluation wrote a non-finite potential (inf or NaN) */

/* Smallest tol each kernel accepts: below it the FP64 rounding of the
 * translations, not the truncation, sets the error, and the requested
 * accuracy could not be met.  CFMM_MIXED needs tol >= CFMM_MIXED_TOL_MIN: its
 * FP32 stages round at about 1e-7 relative. */
#define CFMM_TOL_MIN_LAPLACE_2D 1e-12
#define CFMM_TOL_MIN_HELMHOLTZ_2D 1e-12
#define CFMM_TOL_MIN_LAPLACE_3D 1e-12
#define CFMM_TOL_MIN_HELMHOLTZ_3D 1e-10
#define CFMM_MIXED_TOL_MIN 1e-6

typedef struct cfmm_plan_s* cfmm_plan_t;

typedef enum { CFMM_LAPLACE = 0, CFMM_HELMHOLTZ = 1 } cfmm_kernel;
typedef enum { CFMM_FP64 = 0, CFMM_MIXED = 1 } cfmm_precision;

typedef struct {
    int dim;                   /* 2 or 3 */
    int kernel;                /* cfmm_kernel */
    double wavenumber;         /* kappa > 0 for Helmholtz; ignored for Laplace */
    double tol;                /* requested relative accuracy: CFMM_TOL_MIN_* <= tol < 1 */
    int64_t n_src;             /* number of sources, >= 1 */
    const void* src;           /* complex128[n_src][dim], row-major */
    int64_t n_trg;             /* number of targets (ignored when trg is NULL) */
    const void* trg;           /* complex128[n_trg][dim], row-major; NULL: the targets are
                                  the sources and the self term is left out.
                                  n_src + n_trg < 2^31 */
    int points_on_device;      /* src and trg are 1: device pointers, 0: host pointers */
    int precision;             /* cfmm_precision: FP64, or MIXED (tol >= CFMM_MIXED_TOL_MIN):
                                  FP32 3D near field (FP64-formed differences, compensated
                                  FP32 tile sums added in FP64) and an FP32 3D Laplace M2L
                                  when P <= 16 (FP64 row sums).  The 2D near field stays FP64
                                  (small-argument Hankel). */
    void* stream;              /* hipStream_t for all work; NULL: the null stream */
    int leaf_size;             /* N_s, max points per leaf (Sec. 6.1); 0: 64 in 2D, 256 in 3D */
    int separation;            /* k in {1, 2} (Sec. 6.2, Sec. 6.5); 0: 1 in 2D, 2 in 3D */
    int m2l_form;              /* 3D Laplace M2L (Sec. 5.2): 0 automatic, the point-and-shoot
                                  form (rotate, coaxial shift, rotate back) for every pair
                                  whose rotation phases are well conditioned when P <= 15 and
                                  tol >= 1e-10, the direct addition theorem for the rest;
                                  1: the direct form for every pair */
} cfmm_plan_desc;

/* Build a plan: sort, tree, lists, centres, expansion lengths (Sec. 6.1-6.3).
 * The tree is built on the sources and targets together (Sec. 6.1: a box's
 * complexified centre is the mean over all its points).  On success *out owns
 * device memory until cfmm_destroy.  Synchronises the stream (box and list
 * counts are read back to size allocations). */
int cfmm_plan(cfmm_plan_t* out, const cfmm_plan_desc* desc);

/* One evaluation (Sec. 6.4 steps 1-8) with densities sigma:
 *   density   : complex128[n_src];
 *   potential : complex128[n_trg] (n_src when the plan has no targets), overwritten.
 *   on_device : 1 if both pointers are device pointers (asynchronous on the
 *               plan's stream; a non-finite potential is reported by the next
 *               cfmm_sync), 0 if both are host pointers (synchronous; returns
 *               CFMM_ERANGE when a potential is not finite). */
int cfmm_eval(cfmm_plan_t plan, const void* density, void* potential, int on_device);

/* Layer potentials (Sec. 2.1: the single layer S[sigma], the double layer
 * D[tau] with the source normals nu, and their normal derivatives S', D' at
 * the targets, Sec. 2.2), for dim 3 Laplace (CFMM_ENOTSUP otherwise):
 *   u_i = sum_j G(x_i, y_j) sigma_j + v_j . grad_y G(x_i, y_j),   g_i = grad_x u_i
 * with dipole vectors v_j = tau_j nu_j (complex: bilinear dot products, no
 * conjugation).  S'[sigma], D'[tau] at a target with normal nu_i are
 * nu_i . g_i.  The self term j = i is left out when targets = sources.
 *   charge    : complex128[n_src] or NULL (no charges)
 *   dipole    : complex128[n_src][3] or NULL (no dipoles); not both NULL
 *   potential : complex128[n_trg] or NULL, overwritten
 *   gradient  : complex128[n_trg][3] or NULL, overwritten; not both NULL
 *   on_device : as cfmm_eval.  The first call allocates the dipole and
 *   gradient buffers (and the host staging for host pointers).
 * The expansions have the plan's length, so the gradients, one derivative
 * rougher, carry a somewhat larger relative error than tol.  FP64 near field
 * (owner computes per target leaf, no symmetric pairs). */
int cfmm_eval_layer(cfmm_plan_t plan, const void* charge, const void* dipole, void* potential, void* gradient,
                    int on_device);

/* Wait for all work enqueued on the plan's stream.  Returns CFMM_ERANGE if an
 * evaluation since the previous cfmm_sync (or since the plan was built) wrote
 * a non-finite potential (the potentials are written nevertheless). */
int cfmm_sync(cfmm_plan_t plan);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * evaluation of cfmm_eval with host pointers (on_device = 0), staged through
 * a static device buffer instead of staging the library allocates.
 *   density   : host complex128[n_src]; potential : host complex128[n_trg]
 *               (n_src without targets), overwritten.  Synchronous.
 * Requires n_src + n_trg <= CFMM_STATIC_MAX; larger plans get CFMM_EINVAL.
 * Calls no allocator.  The buffer (CFMM_STATIC_MAX complex values, 64 MiB)
 * is held by every GPU the library runs on until the process ends, and is
 * shared by all calls on that GPU: calls that overlap on one GPU (from
 * several threads or streams) race and must be serialised by the caller.
 * Errors as cfmm_eval with host pointers (CFMM_ERANGE for a non-finite
 * potential). */
#define CFMM_STATIC_MAX 4194304
int cfmm_eval_static(cfmm_plan_t plan, const void* density, void* potential);

/* Free a plan (NULL is accepted).  Synchronises its stream first.  Plans
 * allocate and free stream-ordered (hipMallocAsync / hipFreeAsync on the plan's
 * stream, from the device's default memory pool, which the library sets to keep
 * freed memory for reuse), so building or destroying a plan does not wait for
 * work on other streams. */
int cfmm_destroy(cfmm_plan_t plan);

/* Device bytes held by the plan (the resident footprint used for admission). */
int64_t cfmm_plan_bytes(cfmm_plan_t plan);

/* Message for the calling thread's last error ("" if none). */
const char* cfmm_last_error(void);

/* Plan description for tests and reporting.
 * info[0..19] = { nbox, nleaf, nlevels, top_level, n_list1, n_list2, n_list3,
 *                 n_list4, p2p_pairs (interactions per eval), m2l_pairs,
 *                 max_p, dim, kernel, separation, leaf_size, precision,
 *                 n_src, n_trg (potentials written), n_points (tree points:
 *                 n_src, or n_src + n_trg with distinct targets),
 *                 m2l_source_coefs (source coefficients contracted by M2L per
 *                 evaluation, summed over the List-2 pairs) }
 * The tree, lists and interaction counts are over the tree points. */
int cfmm_plan_info(cfmm_plan_t plan, int64_t* info20);

/* 3D Laplace M2L work of one evaluation by form (Sec. 5.2): work4 = {pairs
 * in the direct addition-theorem form, their algorithmic flops, pairs in
 * the point-and-shoot form, their algorithmic flops}.  Flops: direct
 * 8 (P+1)^2 (Ps+1)^2 per pair (Ps the pair's source length); point and
 * shoot 8 per entry of its four per-degree rotations (a real matrix times a
 * complex vector, two at length Ps and two at P), 4 per entry of the coaxial
 * shift and 6 per diagonal complex product.  Zeros for the other kernels. */
int cfmm_plan_m2l_work(cfmm_plan_t plan, int64_t* work4);

/* Wall-clock milliseconds of the plan's phases (Sec. 6.1, 6.2, 6.3), each
 * ended by a stream synchronisation: ms7[0] points to the device, bounding
 * box, Morton keys and sort; [1] tree topology (occupancy split and level
 * restriction, on the device); [2] complexified centres, top level and
 * expansion lengths; [3] Lists 1-4 (on the device); [4] operator tables,
 * work lists and near-field classes; [5] the geometry check of every near
 * point pair (on the device) and the plan's description; [6] the total. */
int cfmm_plan_timing(cfmm_plan_t plan, double* ms7);

/* Near-field work of one evaluation over the tree points: work2[0] = ordered
 * interactions G(x_i, x_j) sigma_j summed directly (j != i), work2[1] = kernel
 * evaluations that produce them.  G(x, y) = G(y, x), so a pair of near leaves
 * in the small-argument regime of the 2D Helmholtz kernel, and every pair of
 * near leaves in 3D, is evaluated once for both directions and
 * work2[1] < work2[0]. */
int cfmm_plan_near_work(cfmm_plan_t plan, int64_t* work2);

/* Expansion length of level l (0 if the level has no expansions). */
int cfmm_plan_nterms(cfmm_plan_t plan, int level);

/* Copy the integer tree to caller-owned host arrays (any may be NULL):
 *   perm[n]  (int64: sorted position -> input index: sources 0 .. n_src-1,
 *   then targets n_src ..), keys[n] (uint64), n = info[18] tree points,
 *   box_level, box_parent, box_child0, box_nchild, box_pbeg, box_pend [nbox]
 *   (int32), box_prefix[nbox] (uint64). */
int cfmm_plan_export_tree(cfmm_plan_t plan, int64_t* perm, uint64_t* keys,
                          int32_t* box_level, int32_t* box_parent, int32_t* box_child0,
                          int32_t* box_nchild, int32_t* box_pbeg, int32_t* box_pend,
                          uint64_t* box_prefix);

/* Copy list `which` (1..4) as CSR: offsets[nbox+1] and idx[offsets[nbox]]
 * (int32, rows sorted).  Either pointer may be NULL; *count receives the
 * number of entries. */
int cfmm_plan_export_list(cfmm_plan_t plan, int which, int32_t* offsets, int32_t* idx,
                          int64_t* count);

/* Complexified box centres, complex128[nbox][dim] (Sec. 6.1). */
int cfmm_plan_export_centers(cfmm_plan_t plan, void* centers);

/* Multipole and local expansion coefficients after the last evaluation
 * (complex128, box b's coefficients start at offsets[b], -1 for boxes without
 * expansions); *count receives the total.  Any pointer may be NULL.  For
 * checking the individual translation steps against a reference. */
int cfmm_plan_export_expansions(cfmm_plan_t plan, void* mpole, void* local, int64_t* offsets,
                                int64_t* count);

/* Per-stage timing with HIP events on the plan's stream.
 * mode 0: off.
 * mode 1: cfmm_eval records events around each stage; cfmm_stage_ms reads
 *   the last evaluation's times (after cfmm_sync).  Stages: 0 gather, 1 P2M,
 *   2 M2M, 3 M2L+P2L, 4 L2L, 5 L2P+M2P, 6 P2P (+ scatter), 7 whole eval.
 * mode 2: only the near field (stage 6) is bracketed, and mode 3 only the
 *   M2L translations (stage 3 without P2L), each evaluation into its own slot
 *   of a ring of 64 event pairs, so back-to-back evaluations need no host
 *   sync; setting mode 2 or 3 empties the ring.  cfmm_ring_ms (after
 *   cfmm_sync) writes the summed time of the last min(count, 64) evaluations
 *   recorded since, and their number to *count.
 * Any other mode: CFMM_EINVAL. */
int cfmm_set_profiling(cfmm_plan_t plan, int mode);
int cfmm_stage_ms(cfmm_plan_t plan, int stage, double* ms);
int cfmm_ring_ms(cfmm_plan_t plan, double* total_ms, int* count);

/* ---- host-side planning logic, callable without a GPU (for checking) ----
 * The integer tree and Lists 1-4 that cfmm_plan builds from the
 * Morton-sorted keys of the real parts (Sec. 6.1, Sec. 6.2), here from
 * caller-supplied sorted keys (uint64[n], non-decreasing).  top is the first
 * level that carries expansions (boxes coarser than top count as near to
 * everything).  Free the handle with cfmm_htree_free. */
typedef struct cfmm_htree_s* cfmm_htree_t;
int cfmm_htree_build(cfmm_htree_t* out, int dim, int64_t n, const uint64_t* sorted_keys,
                     int leaf_size, int separation, int top);
/* sizes[0] = nbox, sizes[1..4] = entries of Lists 1..4, sizes[5] = levels */
int cfmm_htree_sizes(cfmm_htree_t t, int64_t* sizes6);
int cfmm_htree_export(cfmm_htree_t t, int32_t* box_level, int32_t* box_parent,
                      int32_t* box_child0, int32_t* box_nchild, int32_t* box_pbeg,
                      int32_t* box_pend, uint64_t* box_prefix);
int cfmm_htree_export_list(cfmm_htree_t t, int which, int32_t* offsets, int32_t* idx);
int cfmm_htree_free(cfmm_htree_t t);

/* Expansion length the plan uses for boxes of width w (Sec. 6.3): the smallest
 * n >= 1 with |H_n(kappa R) J_n(kappa r)| <= eps (dim 2) or
 * |h_n(kappa R) j_n(kappa r)| <= eps (dim 3) at n and n+1, R = (0.5+k) w,
 * r = sqrt(dim)/2 w; pmax + 1 if none up to pmax qualifies.  Helmholtz only;
 * pmax <= 63 (dim 2) or 50 (dim 3). */
int cfmm_nterms(int dim, int kernel, double kappa, double w, int separation, double eps, int pmax);

#ifdef __cplusplus
}
#endif
#endif /* CFMM_H */
