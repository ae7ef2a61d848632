// C-ABI of the cfmm library: plan construction (Sec. 6.1-6.3) and one
// evaluation of the complex-coordinate FMM (the eight steps of Sec. 6.4).
#include "../../include/cfmm.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "h3d_host.hpp"
#include "kernels.hpp"
#include "l3d_layout.hpp"
#include "tree_host.hpp"
#include "tree_device.hpp"

#pragma clang fp contract(off)

using namespace cfmm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return fail(CFMM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

std::mutex g_init_mu;
std::set<int> g_inited;

int ensure_device_tables()
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_inited.count(dev)) return CFMM_OK;
    // plans allocate from the device's default memory pool; keep freed memory
    // in the pool for the next plan instead of returning it at every sync
    hipMemPool_t pool;
    HIPCHK(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t keep = UINT64_MAX;
    HIPCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    HIPCHK(static_scratch_init(dev));
    HIPCHK(h2d_init_tables(dev));
    HIPCHK(l2d_init_tables(dev));
    HIPCHK(h3d_init_tables(dev));
    HIPCHK(l3d_init_tables(dev));
    g_inited.insert(dev);
    return CFMM_OK;
}

}  // namespace

struct cfmm_plan_s {
    int dim = 0, kernel = 0, precision = 0, sep = 1, leaf_size = 64;
    double kappa = 0.0, tol = 0.0;
    int64_t n = 0;                // tree points: the sources, then the targets if distinct
    int64_t n_src = 0;            // densities per evaluation
    int64_t n_out = 0;            // potentials per evaluation
    int64_t obase = 0;            // tree point index of the first target (0: targets = sources)
    int device = 0;               // the GPU the plan lives on
    int* d_flag_nf = nullptr;     // set when an evaluation writes a non-finite potential
    hipStream_t stream = nullptr;
    HostTree tree;
    std::vector<uint64_t> keys_h;
    std::vector<int> P;          // per level (0 below the top level)
    std::vector<double> rs;      // per level
    int pmax = 0;
    double lo[3] = {0, 0, 0}, D = 1.0;
    std::vector<double> cen_h;   // complex centres after planning: [b][d] (re, im)

    std::vector<void*> allocs;
    std::vector<size_t> alloc_sz;
    int64_t bytes = 0;

    int* d_perm = nullptr;
    double *d_xre = nullptr, *d_xim = nullptr, *d_sre = nullptr, *d_sim = nullptr;
    int *d_pbeg = nullptr, *d_pend = nullptr, *d_level = nullptr, *d_parent = nullptr;
    int *d_child0 = nullptr, *d_nchild = nullptr, *d_eoff = nullptr, *d_P = nullptr;
    double *d_cre = nullptr, *d_cim = nullptr, *d_rs = nullptr;
    int* d_loff[4] = {nullptr, nullptr, nullptr, nullptr};
    int* d_lidx[4] = {nullptr, nullptr, nullptr, nullptr};
    int* d_work = nullptr;        // all work lists, concatenated
    int off_leaves = 0, nleaf = 0, off_p2m = 0, n_p2m = 0, off_m2l = 0, n_m2l = 0;
    std::vector<int> m2m_off, m2m_cnt, l2l_off, l2l_cnt;   // per level
    cplx *d_mpole = nullptr, *d_local = nullptr, *d_ufar = nullptr;
    int off_p2l = 0, n_p2l = 0;
    H2DNear near2{};              // 2D near-field work items and partial sums
    Near3Work near3{};            // 3D near-field work items and partial sums
    int64_t near_evals = -1;      // kernel evaluations per eval (-1: one per ordered pair)
    std::vector<int> p2l_h;       // host copy of the P2L work list (level order)
    std::vector<int> p2m_h;       // host copy of the P2M work list (level order)
    // plan-time translation operators (2D Helmholtz)
    int64_t *d_o_m2l = nullptr, *d_o_tr = nullptr;
    cplx *d_g_m2l = nullptr, *d_g_m2m = nullptr, *d_g_l2l = nullptr;
    int* d_m2l_src = nullptr;
    // 2D Helmholtz window M2L: groups (first, count) of consecutive M2L-list
    // boxes of one level, the boxes they cover and their LDS
    int2* d_m2lw_grp = nullptr;
    int m2lw_ngrp1 = 0, m2lw_ngrp = 0, m2lw_nbox = 0;   // one-wavefront groups first, then many-entry boxes
    int m2lw_lend = 0;            // levels [top, m2lw_lend) take the window kernel, their generators unscaled
    size_t m2lw_lds1 = 0, m2lw_ldsw = 0;
    double* d_pw = nullptr;
    double *d_io_in = nullptr, *d_io_out = nullptr;       // staging for host pointers
    // 3D Helmholtz: per-level kappa w and scale; translation stages and chunks
    struct H3Chunk {
        int pair_begin, np, grp_begin, ng, goff_off;
    };
    struct H3Stage {
        int kind, level, Ps, Pt, nq, src_h, trg_h;
        double ks, sc, rs_s, inv_w;
        int64_t o_nodes, o_W, o_T;
        int64_t sFG, sA, sR, sB, per_pair;
        std::vector<H3Chunk> chunks;
    };
    std::vector<H3Stage> h3;
    double *d_h3_kw = nullptr, *d_h3_sc = nullptr, *d_h3_tabd = nullptr, *d_h3_eq = nullptr;
    cplx *d_h3_tabc = nullptr, *d_h3_scr = nullptr;
    int *d_h3_src = nullptr, *d_h3_dst = nullptr, *d_h3_gdst = nullptr, *d_h3_goff = nullptr;
    int64_t h3_eq_half = 0;
    // 3D Laplace M2L: table row bases and lane slots (l3d_layout.hpp)
    int* d_l3map = nullptr;
    cplx* d_l3pc = nullptr;       // 3D Laplace M2L: table constants per List-2 entry (5 complex)
    int* d_l3ps = nullptr;        // and source expansion length per entry
    int* d_l3src = nullptr;       // and the source box's expansion offset
    unsigned *d_l3rows64 = nullptr, *d_l3rows32 = nullptr;   // rows per wavefront (l3d_m2l_rows)
    L3Pairs l3_pairs() const { return L3Pairs{d_l3pc, d_l3ps, d_l3src, d_l3rows64, d_l3rows32}; }
    int l3_ntab = 0, l3_R = 0;
    L3PairP l3_pp{};              // source expansion length per M2L pair distance
    // 3D M2P by List-3 entries: owner leaf, partial-sum offsets and storage
    int* d_m2p_owner = nullptr;
    int64_t* d_m2p_poff = nullptr;
    cplx* d_m2p_part = nullptr;
    int n_m2p3 = 0, m2p_pmax = 0;
    std::vector<int64_t> m2p_poff_h;   // host copy of the List-3 part offsets
    // layer potentials (3D Laplace, allocated on first use): dipoles in
    // sorted SoA, far-field gradients, gradient M2P parts, host staging
    double *d_dre = nullptr, *d_dim = nullptr;
    cplx *d_gfar = nullptr, *d_m2p_part4 = nullptr;
    int64_t* d_m2p_poff4 = nullptr;
    double *d_lio_q = nullptr, *d_lio_v = nullptr, *d_lio_u = nullptr, *d_lio_g = nullptr;
    M2PParts m2p_parts() const { return M2PParts{n_m2p3, d_m2p_owner, d_m2p_poff, d_m2p_part}; }
    int64_t ecount = 0;
    int64_t info[20];
    // 3D Laplace M2L forms: m2l_form 0 automatic, 1 direct only; the pairs
    // and algorithmic flops of each form; the boxes with direct-form pairs
    int m2l_form = 0;
    int64_t m2l_work[4] = {0, 0, 0, 0};
    int* d_m2l_dir = nullptr;
    int n_m2l_dir = 0;
    int* d_pns_off = nullptr;     // per box: its point-and-shoot pairs ent[off[b] .. off[b+1]-1]
    int4* d_pns_ent = nullptr;    // (List-2 entry, source expansion offset, Ps, 0)
    // plan phases, wall-clock ms: keys and sort, topology, centres and
    // expansion lengths, lists, operator tables and work lists, geometry
    // check and description; [6] the total
    std::chrono::steady_clock::time_point clk0;
    double tphase[7] = {0, 0, 0, 0, 0, 0, 0};
    double tlast = 0;
    void clock_start()
    {
        clk0 = std::chrono::steady_clock::now();
        tlast = 0;
    }
    void clock_mark(int k)
    {
        double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - clk0).count();
        tphase[k] = ms - tlast;
        tlast = ms;
        tphase[6] = ms;
    }

    int prof = 0;                       // 0 off, 1 every stage, 2 near-field ring
    hipEvent_t ev[8];
    bool ev_made = false;
    static constexpr int kRing = 64;    // evaluations whose near-field time is kept
    hipEvent_t rev[2 * kRing];
    bool rev_made = false;
    int64_t ring_n = 0;                 // evaluations recorded since mode 2 was set

    template <class T>
    int alloc(T** p, size_t count)
    {
        *p = nullptr;
        if (count == 0) count = 1;
        void* q = nullptr;
        // stream-ordered, from the device's memory pool: neither this nor the
        // matching hipFreeAsync waits for work on other streams, so plans
        // made and destroyed on one stream do not stall evaluations on others
        hipError_t e = hipMallocAsync(&q, count * sizeof(T), stream);
        if (e != hipSuccess)
            return fail(CFMM_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        allocs.push_back(q);
        alloc_sz.push_back(count * sizeof(T));
        bytes += (int64_t)(count * sizeof(T));
        *p = (T*)q;
        return CFMM_OK;
    }

    ~cfmm_plan_s()
    {
        hipStreamSynchronize(stream);
        for (void* q : allocs) hipFreeAsync(q, stream);
        hipStreamSynchronize(stream);
        if (ev_made)
            for (int i = 0; i < 8; ++i) hipEventDestroy(ev[i]);
        if (rev_made)
            for (int i = 0; i < 2 * kRing; ++i) hipEventDestroy(rev[i]);
    }

    TreeView view() const
    {
        TreeView tv;
        tv.nbox = tree.nbox();
        tv.pbeg = d_pbeg; tv.pend = d_pend; tv.level = d_level; tv.parent = d_parent;
        tv.child0 = d_child0; tv.nchild = d_nchild;
        tv.cre = d_cre; tv.cim = d_cim; tv.eoff = d_eoff; tv.P = d_P; tv.rs = d_rs;
        tv.l1off = d_loff[0]; tv.l1idx = d_lidx[0];
        tv.l2off = d_loff[1]; tv.l2idx = d_lidx[1];
        tv.l3off = d_loff[2]; tv.l3idx = d_lidx[2];
        tv.l4off = d_loff[3]; tv.l4idx = d_lidx[3];
        return tv;
    }
    H2DOps ops() const
    {
        H2DOps o;
        o.g_m2l = d_g_m2l; o.o_m2l = d_o_m2l; o.g_m2m = d_g_m2m; o.g_l2l = d_g_l2l;
        o.m2l_src = d_m2l_src;
        o.o_tr = d_o_tr; o.pw = d_pw;
        return o;
    }
    IoMap io() const { return IoMap{d_perm, n_src, obase, d_flag_nf}; }
    PointsView pview() const
    {
        PointsView pv;
        pv.n = n; pv.xre = d_xre; pv.xim = d_xim; pv.sre = d_sre; pv.sim = d_sim;
        return pv;
    }
};

namespace {

template <class T>
int upload(cfmm_plan_s* p, T** dst, const std::vector<T>& src)
{
    int rc = p->alloc(dst, src.size());
    if (rc) return rc;
    if (!src.empty())
        HIPCHK(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, p->stream));
    return CFMM_OK;
}

// expansion length of a level: smallest n with |f_n(R) g_n(r)| <= eps at n and
// n+1 (Sec. 6.3, prefactors dropped), R = (0.5 + k) w, r = sqrt(d)/2 w
int nterms_level(int dim, int sep, double kappa, double w, double eps, int pmax)
{
    double R = (0.5 + sep) * w, r = sqrt((double)dim) * 0.5 * w;
    double prev = 1e300;
    for (int m = 1; m <= pmax + 1; ++m) {
        double c = h2d_nterms_crit(kappa, R, r, m);
        if (prev <= eps && c <= eps) return m - 1 >= 1 ? m - 1 : 1;
        prev = c;
    }
    return pmax + 1;
}

// Laplace expansion length: (r/R)^n <= eps at n and n+1 with R = (0.5 + k) w,
// r = sqrt(d)/2 w (Sec. 6.3 with the prefactors dropped; scale free)
int nterms_laplace(int dim, int sep, double eps)
{
    double ratio = sqrt((double)dim) * 0.5 / (0.5 + sep);
    int n = 1;
    while (pow(ratio, n) > eps && n < 200) ++n;
    return n;
}

// 3D Helmholtz translation stages (Sec. 5.3, point-and-shoot with sampled
// rotations and coaxial translations): per stage (M2M, M2L or L2L at one
// level) the pairs grouped by target box, the Gauss-Legendre nodes, the
// projection weights W, the target radial constants and the chunking of the
// pairs over a bounded scratch region.
int plan_h3d(cfmm_plan_s* p, int nlev, int top)
{
    const HostTree& t = p->tree;
    int nb = t.nbox();
    double kappa = p->kappa;
    std::vector<double> kw(nlev, 0.0), sc(nlev, 1.0), wl(nlev);
    for (int l = 0; l < nlev; ++l) {
        wl[l] = p->D * ldexp(1.0, -l);
        kw[l] = kappa * wl[l];
        sc[l] = std::min(1.0, kw[l]);
    }
    std::vector<double> tabd;
    std::vector<cplx> tabc;
    std::vector<int> psrc, pdst, gdst, goff;
    const int64_t cap_bytes = (int64_t)512 << 20;
    int64_t scr = 0;
    auto add_stage = [&](int kind, int level, const std::vector<int>& groups,
                         const std::vector<std::vector<int>>& srcs) {
        cfmm_plan_s::H3Stage S;
        S.kind = kind;
        S.level = level;
        int ls = kind == 0 ? level + 1 : (kind == 1 ? level : level - 1);   // source level
        S.Ps = p->P[ls];
        S.Pt = p->P[level];
        int Pm = std::max(S.Ps, S.Pt);
        S.nq = std::max((int)(2.5 * Pm), Pm + 2);
        S.src_h = kind != 2;
        S.trg_h = kind == 0;
        S.ks = kw[ls];
        S.sc = sc[ls];
        S.inv_w = 1.0 / wl[ls];
        double rs = kind == 0 ? 1.5 * wl[level] : 0.5 * sqrt(3.0) * wl[level];   // physical radius
        S.rs_s = rs / wl[ls];
        // nodes and projection weights
        S.o_nodes = (int64_t)tabd.size();
        std::vector<double> gx(S.nq), gw(S.nq);
        gauss_legendre(S.nq, gx.data(), gw.data());
        for (int j = 0; j < S.nq; ++j) tabd.push_back(sqrt(std::max(0.0, 1.0 - gx[j] * gx[j])));
        for (int j = 0; j < S.nq; ++j) tabd.push_back(gx[j]);
        S.o_W = (int64_t)tabd.size();
        int ntri = (S.Pt + 1) * (S.Pt + 2) / 2;
        size_t w0 = tabd.size();
        tabd.resize(w0 + (size_t)ntri * S.nq);
        std::vector<double> col(ntri);
        for (int j = 0; j < S.nq; ++j) {
            schmidt_column_table(S.Pt, gx[j], sqrt(std::max(0.0, 1.0 - gx[j] * gx[j])), col.data());
            for (int n = 0; n <= S.Pt; ++n)
                for (int m = 0; m <= n; ++m) {
                    int k = n * (n + 1) / 2 + m;
                    tabd[w0 + (size_t)k * S.nq + j] = 0.5 * (2.0 * n + 1.0) * gw[j] * col[k];
                }
        }
        // target radial function T_n at rs and its derivative in source-scaled units
        S.o_T = (int64_t)tabc.size();
        std::vector<double> jj(S.Pt + 1), yy(S.Pt + 1), jd(S.Pt + 1), yd(S.Pt + 1);
        sph_bessel_real(S.Pt, kappa * rs, jj.data(), yy.data(), jd.data(), yd.data());
        std::vector<cplx> Tc(S.Pt + 1), Tdc(S.Pt + 1);
        double sct = sc[level], f = 1.0;
        for (int n = 0; n <= S.Pt; ++n) {
            cplx T, Td;
            if (S.trg_h) {
                T = mk(jj[n] * f, yy[n] * f);
                Td = mk(wl[ls] * kappa * jd[n] * f, wl[ls] * kappa * yd[n] * f);
            } else {
                T = mk(jj[n] / f, 0.0);
                Td = mk(wl[ls] * kappa * jd[n] / f, 0.0);
            }
            double den = cabs2(T) + cabs2(Td);
            Tc[n] = conj(T) * (1.0 / den);
            Tdc[n] = conj(Td) * (1.0 / den);
            f *= sct;
        }
        tabc.insert(tabc.end(), Tc.begin(), Tc.end());
        tabc.insert(tabc.end(), Tdc.begin(), Tdc.end());
        // per-pair scratch strides (complex units)
        int64_t J = 2 * Pm + 1;
        S.sFG = 2 * (int64_t)(Pm + 1) * J;
        S.sA = (int64_t)(Pm + 1) * (Pm + 1);
        S.sR = (int64_t)(S.Ps + 2) * S.nq;
        S.sB = (int64_t)(S.Pt + 1) * (S.Pt + 1);
        S.per_pair = 10 + S.sFG + S.sA + S.sR + S.sB;
        int64_t maxg = 1;
        for (auto& v : srcs) maxg = std::max<int64_t>(maxg, (int64_t)v.size());
        int64_t cap = std::max<int64_t>(maxg, cap_bytes / (S.per_pair * (int64_t)sizeof(cplx)));
        // chunks of whole groups
        size_t g = 0;
        while (g < groups.size()) {
            cfmm_plan_s::H3Chunk C;
            C.pair_begin = (int)psrc.size();
            C.grp_begin = (int)gdst.size();
            C.goff_off = (int)goff.size();
            int np = 0, ng = 0;
            goff.push_back(0);
            while (g < groups.size() && np + (int64_t)srcs[g].size() <= cap) {
                for (int a : srcs[g]) {
                    psrc.push_back(a);
                    pdst.push_back(groups[g]);
                }
                np += (int)srcs[g].size();
                gdst.push_back(groups[g]);
                goff.push_back(np);
                ++ng;
                ++g;
            }
            C.np = np;
            C.ng = ng;
            S.chunks.push_back(C);
            scr = std::max(scr, (int64_t)np * S.per_pair);
        }
        p->h3.push_back(S);
    };
    // M2M at parent level l (children at l + 1), l = nlev-2 .. top
    for (int l = nlev - 2; l >= top; --l) {
        std::vector<int> groups;
        std::vector<std::vector<int>> srcs;
        for (int b = t.lvl_beg[l]; b < t.lvl_beg[l + 1]; ++b)
            if (t.nchild[b] > 0) {
                groups.push_back(b);
                std::vector<int> c;
                for (int k = 0; k < t.nchild[b]; ++k) c.push_back(t.child0[b] + k);
                srcs.push_back(c);
            }
        if (!groups.empty()) add_stage(0, l, groups, srcs);
    }
    // M2L at level l
    for (int l = top; l < nlev; ++l) {
        std::vector<int> groups;
        std::vector<std::vector<int>> srcs;
        for (int b = t.lvl_beg[l]; b < t.lvl_beg[l + 1]; ++b)
            if (t.off[1][b + 1] > t.off[1][b]) {
                groups.push_back(b);
                srcs.emplace_back(t.idx[1].begin() + t.off[1][b], t.idx[1].begin() + t.off[1][b + 1]);
            }
        if (!groups.empty()) add_stage(1, l, groups, srcs);
    }
    // L2L into level l from its parents at l - 1
    for (int l = top + 1; l < nlev; ++l) {
        std::vector<int> groups;
        std::vector<std::vector<int>> srcs;
        for (int b = t.lvl_beg[l]; b < t.lvl_beg[l + 1]; ++b) {
            groups.push_back(b);
            srcs.push_back({t.parent[b]});
        }
        if (!groups.empty()) add_stage(2, l, groups, srcs);
    }
    int pm = 1;
    for (int l = 0; l < nlev; ++l) pm = std::max(pm, p->P[l]);
    int ntri = (pm + 1) * (pm + 2) / 2;
    std::vector<double> eq(2 * (size_t)ntri);
    equator_table(pm, eq.data(), eq.data() + ntri);
    p->h3_eq_half = ntri;
    int rc;
    if ((rc = upload(p, &p->d_h3_kw, kw)) || (rc = upload(p, &p->d_h3_sc, sc)) ||
        (rc = upload(p, &p->d_h3_tabd, tabd)) || (rc = upload(p, &p->d_h3_tabc, tabc)) ||
        (rc = upload(p, &p->d_h3_eq, eq)) || (rc = upload(p, &p->d_h3_src, psrc)) ||
        (rc = upload(p, &p->d_h3_dst, pdst)) || (rc = upload(p, &p->d_h3_gdst, gdst)) ||
        (rc = upload(p, &p->d_h3_goff, goff)) || (rc = p->alloc(&p->d_h3_scr, std::max<int64_t>(scr, 1))))
        return rc;
    (void)nb;
    return CFMM_OK;
}

int plan_impl(cfmm_plan_s* p, const cfmm_plan_desc* d)
{
    int rc;
    p->clock_start();
    int dim = d->dim;
    int64_t n = p->n;
    hipStream_t st = p->stream;
    // -------- points onto the device: the sources, then the distinct targets;
    // the tree holds both (a box's centre averages all its points, Sec. 6.1)
    double* d_pts = nullptr;
    if ((rc = p->alloc(&d_pts, (size_t)n * dim * 2))) return rc;
    hipMemcpyKind kind = d->points_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(d_pts, d->src, (size_t)d->n_src * dim * 2 * sizeof(double), kind, st));
    if (p->obase > 0)
        HIPCHK(hipMemcpyAsync(d_pts + (size_t)d->n_src * dim * 2, d->trg,
                              (size_t)d->n_trg * dim * 2 * sizeof(double), kind, st));
    // -------- real bounding box (a1)
    int nbb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    double *d_part = nullptr, *d_bb = nullptr;
    if ((rc = p->alloc(&d_part, (size_t)nbb * (2 * dim + 1)))) return rc;
    if ((rc = p->alloc(&d_bb, 2 * dim + 1))) return rc;
    HIPCHK(launch_bbox(d_pts, n, dim, d_part, nbb, d_bb, st));
    double bb[7];
    HIPCHK(hipMemcpyAsync(bb, d_bb, (2 * dim + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bb[2 * dim] != 0.0) return fail(CFMM_EGEOMETRY, "non-finite point coordinates");
    int B = (dim == 2) ? 31 : 21;
    double ext = 0.0, mid[3];
    for (int k = 0; k < dim; ++k) {
        mid[k] = (bb[k] + bb[dim + k]) * 0.5;
        ext = std::max(ext, bb[dim + k] - bb[k]);
    }
    p->D = ext > 0.0 ? ext * (1.0 + ldexp(1.0, -20)) : 1.0;
    KeyParams kp;
    for (int k = 0; k < 3; ++k) kp.lo[k] = 0.0;
    for (int k = 0; k < dim; ++k) {
        p->lo[k] = mid[k] - 0.5 * p->D;
        kp.lo[k] = p->lo[k];
    }
    kp.scale = ldexp(1.0, B) / p->D;
    kp.top = ldexp(1.0, B) - 1.0;
    // -------- Morton keys and sort (a1, a2)
    uint64_t *d_keys = nullptr, *d_keys2 = nullptr;
    int* d_idx2 = nullptr;
    unsigned char* d_scr = nullptr;
    if ((rc = p->alloc(&d_keys, n)) || (rc = p->alloc(&d_keys2, n)) || (rc = p->alloc(&p->d_perm, n)) ||
        (rc = p->alloc(&d_idx2, n)) || (rc = p->alloc(&d_scr, radix_sort_scratch_bytes(n))))
        return rc;
    HIPCHK(launch_morton(d_pts, n, dim, kp, d_keys, p->d_perm, st));
    HIPCHK(launch_radix_sort(d_keys, p->d_perm, d_keys2, d_idx2, n, dim * B, d_scr, st));
    p->keys_h.resize(n);
    HIPCHK(hipMemcpyAsync(p->keys_h.data(), d_keys, n * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    p->clock_mark(0);
    // -------- tree (a3) on the device; the host keeps a copy for planning
    DeviceTree dtree;
    HIPCHK(dtree.build(d_keys, n, dim, B, p->leaf_size, p->sep, st));
    HostTree& t = p->tree;
    int nb = dtree.nbox();
    if ((rc = p->alloc(&p->d_pbeg, nb)) || (rc = p->alloc(&p->d_pend, nb)) || (rc = p->alloc(&p->d_level, nb)) ||
        (rc = p->alloc(&p->d_parent, nb)) || (rc = p->alloc(&p->d_child0, nb)) || (rc = p->alloc(&p->d_nchild, nb)))
        return rc;
    HIPCHK(dtree.export_topology(p->d_level, p->d_parent, p->d_child0, p->d_nchild, p->d_pbeg, p->d_pend, t.level,
                                 t.parent, t.child0, t.nchild, t.pbeg, t.pend, t.prefix));
    t.dim = dim;
    t.nbits = B;
    t.sep = p->sep;
    t.n = n;
    {
        int maxl = 0;
        for (int b = 0; b < nb; ++b) maxl = std::max(maxl, t.level[b]);
        t.lvl_beg.assign(maxl + 2, 0);
        for (int b = 0; b < nb; ++b) t.lvl_beg[t.level[b] + 1]++;
        for (int l = 0; l <= maxl; ++l) t.lvl_beg[l + 1] += t.lvl_beg[l];
    }
    int nlev = t.nlevels();
    p->clock_mark(1);
    // -------- sorted SoA points
    if ((rc = p->alloc(&p->d_xre, (size_t)dim * n)) || (rc = p->alloc(&p->d_xim, (size_t)dim * n)))
        return rc;
    HIPCHK(launch_gather_points(d_pts, p->d_perm, n, dim, p->d_xre, p->d_xim, st));
    // -------- complexified centres (a4)
    std::vector<double> cre((size_t)dim * nb);
    for (int b = 0; b < nb; ++b) {
        int64_t c[3];
        box_coords(t, b, c);
        double h = p->D * ldexp(1.0, -(t.level[b] + 1));
        for (int k = 0; k < dim; ++k) cre[(size_t)k * nb + b] = p->lo[k] + (2.0 * (double)c[k] + 1.0) * h;
    }
    double* d_delta = nullptr;
    if ((rc = upload(p, &p->d_cre, cre)) || (rc = p->alloc(&p->d_cim, (size_t)dim * nb)) ||
        (rc = p->alloc(&d_delta, nb)))
        return rc;
    int *d_cbox = nullptr, *d_cbeg = nullptr, *d_cend = nullptr, *d_coff = nullptr;
    double *d_cpart = nullptr, *d_cpmax = nullptr;
    {
        std::vector<int> cbox, cbeg, cend, coff(nb + 1, 0);
        for (int b = 0; b < nb; ++b) {
            for (int i0 = t.pbeg[b]; i0 < t.pend[b]; i0 += kCentreChunk) {
                cbox.push_back(b);
                cbeg.push_back(i0);
                cend.push_back(std::min(t.pend[b], i0 + kCentreChunk));
            }
            coff[b + 1] = (int)cbox.size();
        }
        CentreChunks ch;
        if ((rc = upload(p, &d_cbox, cbox)) || (rc = upload(p, &d_cbeg, cbeg)) || (rc = upload(p, &d_cend, cend)) ||
            (rc = upload(p, &d_coff, coff)) || (rc = p->alloc(&d_cpart, 3 * cbox.size() + 3)) ||
            (rc = p->alloc(&d_cpmax, cbox.size() + 1)))
            return rc;
        ch.n = (int)cbox.size();
        ch.box = d_cbox; ch.beg = d_cbeg; ch.end = d_cend; ch.off = d_coff;
        ch.part = d_cpart; ch.pmax = d_cpmax;
        HIPCHK(launch_centres(ch, p->d_pbeg, p->d_pend, nb, n, dim, p->d_xim, p->d_cim, d_delta, st));
    }
    std::vector<double> delta(nb), cim((size_t)dim * nb);
    HIPCHK(hipMemcpyAsync(delta.data(), d_delta, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(cim.data(), p->d_cim, (size_t)dim * nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    p->cen_h.resize((size_t)nb * dim * 2);
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < dim; ++k) {
            p->cen_h[((size_t)b * dim + k) * 2] = cre[(size_t)k * nb + b];
            p->cen_h[((size_t)b * dim + k) * 2 + 1] = cim[(size_t)k * nb + b];
        }
    // -------- top level of the far field: the coarsest level (>= 2) whose boxes
    // keep the imaginary spread small enough that e^{2 kappa delta} times the
    // FP64 unit roundoff stays below tol/10 (the expansions of boxes with a
    // large imaginary spread cancel catastrophically)
    std::vector<double> dmax(nlev, 0.0);
    for (int b = 0; b < nb; ++b) dmax[t.level[b]] = std::max(dmax[t.level[b]], delta[b]);
    int top = 2;
    if (p->kernel == CFMM_HELMHOLTZ) {
        double tau = 0.5 * log(0.1 * p->tol / 2.2e-16);
        while (top < nlev && p->kappa * dmax[top] > tau) ++top;
    }
    if (top > nlev) top = nlev;
    // -------- expansion lengths (a6)
    bool h2d = dim == 2;
    bool lap2 = h2d && p->kernel == CFMM_LAPLACE;
    p->P.assign(nlev, 0);
    p->rs.assign(nlev, 1.0);
    int pmax = 0;
    if (lap2) {
        // 2D Laplace: (r/R)^n <= tol with R = (0.5 + k) w, r = sqrt(2)/2 w (Sec.
        // 6.3 with the prefactors dropped), the same on every level;
        // coordinates of level l are scaled by 1/w_l
        int m = nterms_laplace(dim, p->sep, p->tol);
        if (m > kPMax2D)
            return fail(CFMM_ENOTSUP, "expansion length " + std::to_string(m) + " above the supported maximum " +
                                          std::to_string(kPMax2D));
        for (int l = top; l < nlev; ++l) {
            p->rs[l] = 1.0 / (p->D * ldexp(1.0, -l));
            p->P[l] = m;
        }
        pmax = m;
    } else if (h2d) {
        double eps = 0.1 * p->tol;
        for (int l = top; l < nlev; ++l) {
            double w = p->D * ldexp(1.0, -l);
            p->rs[l] = std::min(1.0, p->kappa * w);
            int m = nterms_level(p->dim, p->sep, p->kappa, w, eps, kPMax2D);
            if (m > kPMax2D && l == top && top + 1 < nlev) {
                ++top;   // boxes this wide stay in the near field of the coarser lists
                continue;
            }
            if (m > kPMax2D)
                return fail(CFMM_ENOTSUP, "expansion length above the supported maximum (" +
                                             std::to_string(kPMax2D) + ") at level " + std::to_string(l) +
                                             "; the boxes are too many wavelengths wide");
            p->P[l] = m;
            pmax = std::max(pmax, m);
        }
    } else if (p->kernel == CFMM_HELMHOLTZ) {
        // 3D Helmholtz: |h_n(kR) j_n(kr)| <= eps_l at n and n+1 (Sec. 6.3) with
        // eps_l = (tol/10) e^{-kappa delta_l / 2}: in the oscillatory range the
        // continued expansion terms of a box whose points spread by delta_l in
        // the imaginary direction grow with e^{kappa delta_l}; half the exponent
        // is the empirical margin.  Coordinates of level l are scaled by 1/w_l.
        for (int l = top; l < nlev; ++l) {
            double w = p->D * ldexp(1.0, -l);
            p->rs[l] = 1.0 / w;
            double eps = 0.1 * p->tol * exp(-0.5 * p->kappa * dmax[l]);
            int m = h3d_nterms(p->kappa, w, p->sep, eps, kPMaxH3);
            if (m > kPMaxH3 && l == top && top + 1 < nlev) {
                ++top;   // boxes this wide stay in the near field of the coarser lists
                continue;
            }
            if (m > kPMaxH3)
                return fail(CFMM_ENOTSUP, "expansion length above the supported maximum (" +
                                             std::to_string(kPMaxH3) + ") at level " + std::to_string(l) +
                                             "; the boxes are too many wavelengths wide");
            p->P[l] = m;
            pmax = std::max(pmax, m);
        }
    } else {
        // 3D Laplace: (r/R)^n <= tol with R = (0.5 + k) w, r = sqrt(3)/2 w, the same
        // at every level; coordinates of level l are scaled by 1/w_l
        int m = nterms_laplace(dim, p->sep, p->tol);
        int lim = l3d_pmax_supported();
        if (m > lim)
            return fail(CFMM_ENOTSUP, "expansion length " + std::to_string(m) +
                                         " above the supported maximum " + std::to_string(lim));
        for (int l = top; l < nlev; ++l) {
            p->rs[l] = 1.0 / (p->D * ldexp(1.0, -l));
            p->P[l] = m;
        }
        pmax = m;
        // per M2L pair: the same rule with the pair's nearest target distance
        // (d - 1/2) w, d the max-norm centre distance in box widths
        for (int d = 0; d < 8; ++d) {
            double ratio = sqrt(3.0) * 0.5 / (d - 0.5);
            int md = m;
            if (d > p->sep) {
                md = 1;
                while (pow(ratio, md) > p->tol && md < m) ++md;
            }
            p->l3_pp.p[d] = md;
        }
        // point-and-shoot M2L where it applies: P within its lane layout,
        // tol >= 1e-10, and per pair the phases' powers bounded so that
        // K^(2P) stays below 1e10 tol (K the largest of |e^{+-ia}|,
        // |e^{+-ib}|; the FP64 error of the rotations grows like K^(2P))
        p->l3_pp.pns_P = (p->m2l_form == 0 && m <= l3d_pns_max_p() && p->tol >= 1e-10) ? m : 0;
        p->l3_pp.pns_logb = log(1e10 * p->tol);
        L3dM2LLayout lay = l3d_m2l_layout(m);
        std::vector<int> map(lay.base);
        map.insert(map.end(), lay.slot.begin(), lay.slot.end());
        if ((rc = upload(p, &p->d_l3map, map)) || (rc = upload(p, &p->d_l3rows64, l3d_m2l_rows(l3d_m2l_waves(0)))) ||
            (rc = upload(p, &p->d_l3rows32, l3d_m2l_rows(l3d_m2l_waves(1)))))
            return rc;
        p->l3_ntab = lay.entries;
        p->l3_R = lay.R;
    }
    p->pmax = pmax;
    p->clock_mark(2);
    // -------- lists (a5) on the device, from the final top level
    {
        int64_t cnt[4];
        HIPCHK(dtree.count_lists(top, t.lvl_beg, cnt));
        for (int q = 0; q < 4; ++q)
            if ((rc = p->alloc(&p->d_loff[q], (size_t)nb + 1)) || (rc = p->alloc(&p->d_lidx[q], (size_t)cnt[q])))
                return rc;
        HIPCHK(dtree.fill_lists(p->d_loff, p->d_lidx, t.off, t.idx));
        t.top = top;
        dtree.release();
    }
    p->clock_mark(3);
    auto ncoef = [&](int l) -> int64_t { return h2d ? 2 * p->P[l] + 1 : (int64_t)(p->P[l] + 1) * (p->P[l] + 1); };
    std::vector<int> eoff(nb, -1);
    int64_t ecount = 0;
    for (int b = 0; b < nb; ++b)
        if (t.level[b] >= top) {
            eoff[b] = (int)ecount;
            ecount += ncoef(t.level[b]);
        }
    if (ecount > (int64_t)0x7fffffff) return fail(CFMM_ENOTSUP, "expansion storage above 2^31 entries");
    p->ecount = ecount;
    if ((rc = upload(p, &p->d_eoff, eoff)) || (rc = upload(p, &p->d_P, p->P)) || (rc = upload(p, &p->d_rs, p->rs)))
        return rc;
    // -------- work lists
    std::vector<int> work;
    p->off_leaves = (int)work.size();
    for (int b = 0; b < nb; ++b)
        if (t.nchild[b] == 0) work.push_back(b);
    p->nleaf = (int)work.size() - p->off_leaves;
    p->off_p2m = (int)work.size();
    for (int b = 0; b < nb; ++b)
        if (t.nchild[b] == 0 && t.level[b] >= top) work.push_back(b);
    p->n_p2m = (int)work.size() - p->off_p2m;
    p->p2m_h.assign(work.begin() + p->off_p2m, work.end());
    p->m2m_off.assign(nlev, 0);
    p->m2m_cnt.assign(nlev, 0);
    p->l2l_off.assign(nlev, 0);
    p->l2l_cnt.assign(nlev, 0);
    for (int l = top; l < nlev; ++l) {
        p->m2m_off[l] = (int)work.size();
        for (int b = t.lvl_beg[l]; b < t.lvl_beg[l + 1]; ++b)
            if (t.nchild[b] > 0) work.push_back(b);
        p->m2m_cnt[l] = (int)work.size() - p->m2m_off[l];
    }
    p->off_m2l = (int)work.size();
    for (int b = 0; b < nb; ++b)
        if (t.level[b] >= top) work.push_back(b);
    p->n_m2l = (int)work.size() - p->off_m2l;
    for (int l = top + 1; l < nlev; ++l) {
        p->l2l_off[l] = (int)work.size();
        for (int b = t.lvl_beg[l]; b < t.lvl_beg[l + 1]; ++b) work.push_back(b);
        p->l2l_cnt[l] = (int)work.size() - p->l2l_off[l];
    }
    if (!t.idx[2].empty()) {
        int n3 = (int)t.idx[2].size();
        std::vector<int> owner(n3);
        std::vector<int64_t> poff(n3 + 1, 0);
        for (int b = 0; b < nb; ++b)
            for (int e = t.off[2][b]; e < t.off[2][b + 1]; ++e) {
                owner[e] = b;
                poff[e + 1] = t.pend[b] - t.pbeg[b];
                p->m2p_pmax = std::max(p->m2p_pmax, p->P[t.level[t.idx[2][e]]]);
            }
        for (int e = 0; e < n3; ++e) poff[e + 1] += poff[e];
        p->m2p_poff_h = poff;
        if ((rc = upload(p, &p->d_m2p_owner, owner)) || (rc = upload(p, &p->d_m2p_poff, poff)) ||
            (rc = p->alloc(&p->d_m2p_part, (size_t)std::max<int64_t>(1, poff[n3]))))
            return rc;
        p->n_m2p3 = n3;
    }
    p->off_p2l = (int)work.size();
    for (int b = 0; b < nb; ++b)
        if (t.level[b] >= top && t.off[3][b + 1] > t.off[3][b]) work.push_back(b);
    p->n_p2l = (int)work.size() - p->off_p2l;
    p->p2l_h.assign(work.begin() + p->off_p2l, work.end());
    int off_tr = (int)work.size();
    for (int b = 0; b < nb; ++b)
        if (t.level[b] >= top + 1) work.push_back(b);
    int n_tr = (int)work.size() - off_tr;
    int off_pairb = (int)work.size();
    for (int b = 0; b < nb; ++b)
        for (int e = t.off[1][b]; e < t.off[1][b + 1]; ++e) work.push_back(b);
    int npairs = (int)t.idx[1].size();
    // 2D Helmholtz near field by List-1 entries e = (target leaf b, source leaf
    // a).  A pair whose every point pair has |kappa r| < 3 (bound from the box
    // geometry: real half widths plus the imaginary spreads about the
    // complexified centres) takes the power series of H0 with a per-pair term
    // count; such pairs with a < b are evaluated once for both directions.
    // Diagonal entries and the remaining pairs are row items.
    if (h2d) {
        double k2 = 0.25 * p->kappa * p->kappa;
        int ne = (int)t.idx[0].size();
        std::vector<int> row_of(ne), partner(ne, -1), sym, sym_k, diag, diag_k, ser, ser_k, gen;
        std::vector<int64_t> coff(ne + 1, 0);
        for (int b = 0; b < nb; ++b)
            for (int e = t.off[0][b]; e < t.off[0][b + 1]; ++e) {
                row_of[e] = b;
                coff[e + 1] = coff[e] + (t.pend[b] - t.pbeg[b]);
            }
        for (int e = 0; e < ne; ++e) {
            int b = row_of[e], a = t.idx[0][e];
            const int* r0 = t.idx[0].data() + t.off[0][a];
            const int* r1 = t.idx[0].data() + t.off[0][a + 1];
            const int* f = std::lower_bound(r0, r1, b);
            if (f == r1 || *f != b) return fail(CFMM_EINVAL, "internal: List 1 is not symmetric");
            partner[e] = (int)(f - t.idx[0].data());
        }
        auto bound = [&](int b, int a) {
            double wb = p->D * ldexp(1.0, -t.level[b]), wa = p->D * ldexp(1.0, -t.level[a]);
            double sre = 0.0, sci = 0.0;
            for (int k = 0; k < dim; ++k) {
                double dr = fabs(cre[(size_t)k * nb + b] - cre[(size_t)k * nb + a]) + 0.5 * (wa + wb);
                double dc = cim[(size_t)k * nb + b] - cim[(size_t)k * nb + a];
                sre += dr * dr;
                sci += dc * dc;
            }
            double di = delta[a] + delta[b] + sqrt(sci);
            return k2 * (sre + di * di);
        };
        auto nterms_series = [](double qb) {
            int K = 1;
            double term = qb * qb / 4.0;      // q^(K+1) / ((K+1)!)^2 at K = 1
            while (term > 1e-17 && K < 39) {
                ++K;
                term *= qb / ((double)(K + 1) * (K + 1));
            }
            return K;
        };
        for (int e = 0; e < ne; ++e) {
            int b = row_of[e], a = t.idx[0][e];
            if (a > b) continue;                      // the pair is visited from a's row
            double qb = lap2 ? 0.0 : bound(b, a);
            bool series = lap2 || qb < 2.25;          // 2D Laplace: Log s for every pair
            if (a == b) {
                if (series && t.pend[b] - t.pbeg[b] <= 64) { diag.push_back(e); diag_k.push_back(nterms_series(qb)); }
                else if (series) { ser.push_back(e); ser_k.push_back(nterms_series(qb)); }
                else gen.push_back(e);
            } else if (series) {
                sym.push_back(e);
                sym_k.push_back(nterms_series(qb));
            } else {
                gen.push_back(e);
                gen.push_back(partner[e]);
            }
        }
        int64_t ev = 0;
        auto cnt = [&](int b) { return (int64_t)(t.pend[b] - t.pbeg[b]); };
        for (int e : sym) ev += cnt(row_of[e]) * cnt(t.idx[0][e]);
        for (int e : diag) ev += cnt(row_of[e]) * (cnt(row_of[e]) - 1) / 2;
        for (int e : ser) ev += cnt(row_of[e]) * (cnt(row_of[e]) - 1);
        for (int e : gen) {
            int b = row_of[e], a = t.idx[0][e];
            ev += a == b ? cnt(b) * (cnt(b) - 1) : cnt(b) * cnt(a);
        }
        p->near_evals = ev;
        p->near2.nsym = (int)sym.size();
        p->near2.ndiag = (int)diag.size();
        p->near2.nser = (int)ser.size();
        p->near2.ngen = (int)gen.size();
        int* dd[7] = {nullptr};
        if ((rc = upload(p, &dd[0], sym)) || (rc = upload(p, &dd[1], sym_k)) || (rc = upload(p, &dd[2], ser)) ||
            (rc = upload(p, &dd[3], ser_k)) || (rc = upload(p, &dd[4], gen)) || (rc = upload(p, &dd[5], row_of)) ||
            (rc = upload(p, &dd[6], partner)))
            return rc;
        int *dg = nullptr, *dgk = nullptr;
        if ((rc = upload(p, &dg, diag)) || (rc = upload(p, &dgk, diag_k))) return rc;
        p->near2.diag = dg;
        p->near2.diag_k = dgk;
        int64_t* dcoff = nullptr;
        cplx* dC = nullptr;
        if ((rc = upload(p, &dcoff, coff)) || (rc = p->alloc(&dC, std::max<int64_t>(coff[ne], 1)))) return rc;
        p->near2.sym = dd[0]; p->near2.sym_k = dd[1]; p->near2.ser = dd[2]; p->near2.ser_k = dd[3];
        p->near2.gen = dd[4]; p->near2.row_of = dd[5]; p->near2.partner = dd[6];
        p->near2.coff = dcoff; p->near2.C = dC;
    }
    // 3D near field by List-1 entries: each pair of near leaves once (a < b),
    // plus the diagonal entries.  In mixed Helmholtz, pairs whose near field
    // may reach kappa |r| > 8 (box bound as above) form the phase in FP64.
    if (dim == 3) {
        int ne = (int)t.idx[0].size();
        std::vector<int> row_of(ne), partner(ne, -1), it[4];
        std::vector<int64_t> coff(ne + 1, 0);
        for (int b = 0; b < nb; ++b)
            for (int e = t.off[0][b]; e < t.off[0][b + 1]; ++e) {
                row_of[e] = b;
                coff[e + 1] = coff[e] + (t.pend[b] - t.pbeg[b]);
            }
        for (int e = 0; e < ne; ++e) {
            int b = row_of[e], a = t.idx[0][e];
            const int* r0 = t.idx[0].data() + t.off[0][a];
            const int* r1 = t.idx[0].data() + t.off[0][a + 1];
            const int* f = std::lower_bound(r0, r1, b);
            if (f == r1 || *f != b) return fail(CFMM_EINVAL, "internal: List 1 is not symmetric");
            partner[e] = (int)(f - t.idx[0].data());
        }
        bool wide_split = p->kernel == CFMM_HELMHOLTZ && p->precision == CFMM_MIXED;
        auto rbound = [&](int b, int a) {
            double wb = p->D * ldexp(1.0, -t.level[b]), wa = p->D * ldexp(1.0, -t.level[a]);
            double sre = 0.0, sci = 0.0;
            for (int k = 0; k < dim; ++k) {
                double dr = fabs(cre[(size_t)k * nb + b] - cre[(size_t)k * nb + a]) + 0.5 * (wa + wb);
                double dc = cim[(size_t)k * nb + b] - cim[(size_t)k * nb + a];
                sre += dr * dr;
                sci += dc * dc;
            }
            double di = delta[a] + delta[b] + sqrt(sci);
            return sqrt(sre + di * di);
        };
        int64_t ev = 0;
        auto cnt = [&](int b) { return (int64_t)(t.pend[b] - t.pbeg[b]); };
        for (int e = 0; e < ne; ++e) {
            int b = row_of[e], a = t.idx[0][e];
            if (a > b) continue;
            int w = (wide_split && p->kappa * rbound(b, a) > 8.0) ? 2 : 0;
            it[w + (a == b ? 1 : 0)].push_back(e);
            ev += a == b ? cnt(b) * (cnt(b) - 1) / 2 : cnt(b) * cnt(a);
        }
        p->near_evals = ev;
        int* dd[6] = {nullptr};
        for (int q = 0; q < 4; ++q)
            if ((rc = upload(p, &dd[q], it[q]))) return rc;
        if ((rc = upload(p, &dd[4], row_of)) || (rc = upload(p, &dd[5], partner))) return rc;
        int64_t* dcoff = nullptr;
        cplx* dC = nullptr;
        if ((rc = upload(p, &dcoff, coff)) || (rc = p->alloc(&dC, std::max<int64_t>(coff[ne], 1)))) return rc;
        for (int q = 0; q < 4; ++q) {
            p->near3.items[q] = dd[q];
            p->near3.nitems[q] = (int)it[q].size();
        }
        p->near3.row_of = dd[4];
        p->near3.partner = dd[5];
        p->near3.coff = dcoff;
        p->near3.C = dC;
    }
    if ((rc = upload(p, &p->d_work, work))) return rc;
    int64_t gsz = 0, tsz = 0;
    if (h2d && !lap2) {
    // -------- translation operators (generators of M2L, M2M, L2L)
    std::vector<int64_t> o_m2l(npairs), o_tr(nb, -1);
    for (int b = 0; b < nb; ++b)
        for (int e = t.off[1][b]; e < t.off[1][b + 1]; ++e) {
            o_m2l[e] = gsz;
            gsz += 4 * p->P[t.level[b]] + 1;
        }
    for (int b = 0; b < nb; ++b)
        if (t.level[b] >= top + 1) {
            o_tr[b] = tsz;
            tsz += 2 * (p->P[t.level[b]] + p->P[t.level[b] - 1]) + 1;
        }
    std::vector<double> pw((size_t)nlev * kPwStride, 0.0);
    for (int l = 0; l < nlev; ++l)
        for (int e = 0; e < kPwStride; ++e) pw[(size_t)l * kPwStride + e] = pow(p->rs[l], (double)e);
    std::vector<int> msrc(t.idx[1].size());
    for (size_t e = 0; e < msrc.size(); ++e) msrc[e] = eoff[t.idx[1][e]];
    if ((rc = upload(p, &p->d_m2l_src, msrc))) return rc;
    {
        // window M2L for the levels whose operator fits FP64 unscaled: the
        // generator H_k e^{ik phi}, k <= 2P, is at most about (2P)! / r^(2P)
        // (r = min(1, kappa w), the centres at least 2w apart), kept below
        // 1e250; a prefix of the levels from top, r growing with the box.
        // Consecutive boxes of a level are grouped while their List-2 entries
        // fit one round, a box with more entries alone.
        std::vector<int2> grp, big;
        int k = 0, Wb = h2d_m2l_w_waves();
        p->m2lw_lend = top;
        for (int l = top; l < nlev; ++l) {
            int P = p->P[l];
            if (!(p->rs[l] > 0.0 && lgamma(2.0 * P + 1.0) / log(10.0) - 2.0 * P * log10(p->rs[l]) < 250.0)) break;
            p->m2lw_lend = l + 1;
            int E = h2d_m2l_w_slots(P);
            int b = t.lvl_beg[l], bend = t.lvl_beg[l + 1];
            while (b < bend) {
                int first = b, ne = t.off[1][b + 1] - t.off[1][b];
                ++b;
                if (ne > E) {
                    big.push_back(make_int2(k + (first - t.lvl_beg[l]), 1));
                    p->m2lw_ldsw = std::max(p->m2lw_ldsw, h2d_m2l_w_lds(P, Wb));
                    continue;
                }
                while (b < bend && t.off[1][b + 1] - t.off[1][b] <= E &&
                       ne + (t.off[1][b + 1] - t.off[1][b]) <= E) {
                    ne += t.off[1][b + 1] - t.off[1][b];
                    ++b;
                }
                grp.push_back(make_int2(k + (first - t.lvl_beg[l]), b - first));
                p->m2lw_lds1 = std::max(p->m2lw_lds1, h2d_m2l_w_lds(P, 1));
            }
            k += t.lvl_beg[l + 1] - t.lvl_beg[l];
        }
        p->m2lw_nbox = k;
        p->m2lw_ngrp1 = (int)grp.size();
        grp.insert(grp.end(), big.begin(), big.end());
        p->m2lw_ngrp = (int)grp.size();
        if ((rc = upload(p, &p->d_m2lw_grp, grp))) return rc;
    }
    if ((rc = upload(p, &p->d_o_m2l, o_m2l)) || (rc = upload(p, &p->d_o_tr, o_tr)) ||
        (rc = upload(p, &p->d_pw, pw)) || (rc = p->alloc(&p->d_g_m2l, gsz)) ||
        (rc = p->alloc(&p->d_g_m2m, tsz)) || (rc = p->alloc(&p->d_g_l2l, tsz)))
        return rc;
    {
        TreeView tv = p->view();
        HIPCHK(h2d_gen_ops(p->d_work + off_pairb, npairs, p->d_work + off_tr, n_tr, tv, p->kappa, p->m2lw_lend,
                           p->d_o_m2l, p->d_g_m2l, p->d_o_tr, p->d_g_m2m, p->d_g_l2l, st));
    }
    }  // h2d operator tables
    if (dim == 3 && p->kernel == CFMM_HELMHOLTZ)
        if ((rc = plan_h3d(p, nlev, top))) return rc;
    if (dim == 3 && p->kernel == CFMM_LAPLACE) {
        // M2L pair constants: fixed by the geometry, formed once per plan
        size_t nl2 = std::max<size_t>(t.idx[1].size(), 1);
        if ((rc = p->alloc(&p->d_l3pc, 5 * nl2)) || (rc = p->alloc(&p->d_l3ps, nl2)) ||
            (rc = p->alloc(&p->d_l3src, nl2)))
            return rc;
        TreeView tv = p->view();
        HIPCHK(l3d_m2l_pairs(p->d_work + p->off_m2l, p->n_m2l, tv, p->l3_pp, p->d_l3pc, p->d_l3ps, p->d_l3src, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    p->clock_mark(4);
    // -------- geometry check on the near pairs
    int* d_flag = nullptr;
    if ((rc = p->alloc(&d_flag, 1))) return rc;
    HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), st));
    HIPCHK(launch_check_near(p->d_work + p->off_leaves, p->nleaf, p->d_pbeg, p->d_pend, p->d_loff[0],
                             p->d_lidx[0], n, dim, p->d_xre, p->d_xim, d_flag, st));
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flag)
        return fail(CFMM_EGEOMETRY, "a near pair has Re(r^2) <= 0: the imaginary parts are not a "
                                    "Lipschitz function of the real parts with constant below 1");
    // -------- evaluation buffers
    if ((rc = p->alloc(&p->d_sre, n)) || (rc = p->alloc(&p->d_sim, n)) ||
        (rc = p->alloc(&p->d_mpole, ecount)) || (rc = p->alloc(&p->d_local, ecount)) ||
        (rc = p->alloc(&p->d_ufar, n)) || (rc = p->alloc(&p->d_flag_nf, 1)))
        return rc;
    HIPCHK(hipMemsetAsync(p->d_flag_nf, 0, sizeof(int), st));
    // -------- release planning scratch; the plan keeps the rest resident
    HIPCHK(hipStreamSynchronize(st));
    for (void* q : {(void*)d_pts, (void*)d_part, (void*)d_bb, (void*)d_keys, (void*)d_keys2,
                    (void*)d_idx2, (void*)d_scr, (void*)d_delta, (void*)d_flag, (void*)d_cbox, (void*)d_cbeg,
                    (void*)d_cend, (void*)d_coff, (void*)d_cpart, (void*)d_cpmax}) {
        auto it = std::find(p->allocs.begin(), p->allocs.end(), q);
        if (it != p->allocs.end()) {
            size_t k = it - p->allocs.begin();
            p->bytes -= (int64_t)p->alloc_sz[k];
            p->allocs.erase(it);
            p->alloc_sz.erase(p->alloc_sz.begin() + k);
            HIPCHK(hipFreeAsync(q, st));
        }
    }
    // -------- description
    int64_t p2p = 0, m2l = (int64_t)t.idx[1].size();
    for (int b = 0; b < nb; ++b) {
        if (t.nchild[b]) continue;
        int64_t nt = t.pend[b] - t.pbeg[b], ns = 0;
        for (int e = t.off[0][b]; e < t.off[0][b + 1]; ++e) {
            int a = t.idx[0][e];
            ns += t.pend[a] - t.pbeg[a];
        }
        p2p += nt * ns - nt;   // the self pairs are skipped
    }
    int64_t* I = p->info;
    I[0] = nb; I[1] = p->nleaf; I[2] = nlev; I[3] = top;
    for (int q = 0; q < 4; ++q) I[4 + q] = (int64_t)t.idx[q].size();
    I[8] = p2p; I[9] = m2l; I[10] = pmax; I[11] = dim; I[12] = p->kernel; I[13] = p->sep;
    I[14] = p->leaf_size; I[15] = p->precision;
    // M2L work: the source coefficients contracted over all List-2 pairs (3D
    // Laplace: (Ps+1)^2 with the pair's own Ps; otherwise the level's count)
    int64_t m2l_src = 0;
    if (dim == 3 && p->kernel == CFMM_LAPLACE) {
        // the pairs' own lengths, formed on the device with the pair constants
        std::vector<int> ps(t.idx[1].size());
        if (!ps.empty()) {
            HIPCHK(hipMemcpyAsync(ps.data(), p->d_l3ps, ps.size() * sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        // a negative entry marks a point-and-shoot pair (~Ps); algorithmic
        // flops: direct 8 (P+1)^2 (Ps+1)^2; point and shoot 8 per entry of
        // the four rotations (real matrix, complex vector: 4 flops per entry,
        // two rotations at each length), 4 per coaxial entry and 6 per
        // diagonal complex product (three at each length)
        auto rot = [](int64_t q) { return (q + 1) * (2 * q + 1) * (2 * q + 3) / 3; };
        int64_t P1 = pmax + 1;
        for (int v : ps) {
            int64_t q = v < 0 ? ~v : v;
            m2l_src += (q + 1) * (q + 1);
            if (v >= 0) {
                p->m2l_work[0] += 1;
                p->m2l_work[1] += 8 * P1 * P1 * (q + 1) * (q + 1);
            } else {
                int64_t cx = 0;
                for (int64_t k = -q; k <= q; ++k) {
                    int64_t ak = k < 0 ? -k : k;
                    cx += (P1 - ak) * (q + 1 - ak);
                }
                p->m2l_work[2] += 1;
                p->m2l_work[3] += 8 * (rot(q) + rot(pmax)) + 4 * cx + 18 * ((q + 1) * (q + 1) + P1 * P1);
            }
        }
        if (p->m2l_work[2] > 0) {
            // the boxes with direct-form pairs, in the M2L work order, and
            // every box's point-and-shoot pairs in list order
            std::vector<int> dir, poff(nb + 1, 0);
            std::vector<int4> pent;
            pent.reserve((size_t)p->m2l_work[2]);
            for (int b = 0; b < nb; ++b) {
                poff[b] = (int)pent.size();
                for (int e = t.off[1][b]; e < t.off[1][b + 1]; ++e)
                    if (ps[e] < 0) pent.push_back(make_int4(e, eoff[t.idx[1][e]], ~ps[e], 0));
            }
            poff[nb] = (int)pent.size();
            const int* mb = work.data() + p->off_m2l;
            for (int i = 0; i < p->n_m2l; ++i) {
                int b = mb[i];
                for (int e = t.off[1][b]; e < t.off[1][b + 1]; ++e)
                    if (ps[e] >= 0) {
                        dir.push_back(b);
                        break;
                    }
            }
            p->n_m2l_dir = (int)dir.size();
            if (!dir.empty() && (rc = upload(p, &p->d_m2l_dir, dir))) return rc;
            if ((rc = upload(p, &p->d_pns_off, poff)) || (rc = upload(p, &p->d_pns_ent, pent))) return rc;
        }
    } else {
        for (int b = 0; b < nb; ++b) {
            int Ps = p->P[t.level[b]];
            m2l_src += (int64_t)(t.off[1][b + 1] - t.off[1][b]) * (h2d ? 2 * Ps + 1 : (int64_t)(Ps + 1) * (Ps + 1));
        }
    }
    I[16] = p->n_src; I[17] = p->n_out; I[18] = p->n; I[19] = m2l_src;
    HIPCHK(hipStreamSynchronize(st));
    p->clock_mark(5);
    return CFMM_OK;
}

// 3D Laplace M2L: the point-and-shoot kernel writes every box's local from
// its pairs of that form, then the direct kernel adds the other pairs on the
// boxes that have any; with no point-and-shoot pair the direct kernel writes.
static hipError_t run_l3d_m2l(cfmm_plan_s* p, const TreeView& tv, int P, int mixed, hipStream_t st)
{
    const int* W = p->d_work;
    if (p->m2l_work[2] > 0) {
        hipError_t e = l3d_m2l_pns(W + p->off_m2l, p->n_m2l, P, tv, p->d_l3pc, p->d_pns_off, p->d_pns_ent,
                                   p->d_mpole, p->d_local, st);
        if (e != hipSuccess) return e;
        return l3d_m2l(p->d_m2l_dir, p->n_m2l_dir, P, tv, p->d_l3map, p->l3_ntab, p->l3_R, p->l3_pairs(), mixed, 1,
                       p->d_mpole, p->d_local, st);
    }
    return l3d_m2l(W + p->off_m2l, p->n_m2l, P, tv, p->d_l3map, p->l3_ntab, p->l3_R, p->l3_pairs(), mixed, 0,
                   p->d_mpole, p->d_local, st);
}

int check_finite(cfmm_plan_s* p);
int eval_on_device(cfmm_plan_s* p, const double* sig, double* out);

}  // namespace

extern "C" {

int cfmm_plan(cfmm_plan_t* out, const cfmm_plan_desc* d)
{
    if (!out) return fail(CFMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(CFMM_EINVAL, "desc is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(CFMM_EINVAL, "dim must be 2 or 3");
    if (d->kernel != CFMM_LAPLACE && d->kernel != CFMM_HELMHOLTZ) return fail(CFMM_EINVAL, "unknown kernel");
    if (d->kernel == CFMM_HELMHOLTZ && !(d->wavenumber > 0.0 && isfinite(d->wavenumber)))
        return fail(CFMM_EINVAL, "Helmholtz needs a finite wavenumber > 0");
    double tmin = d->dim == 2 ? (d->kernel == CFMM_LAPLACE ? CFMM_TOL_MIN_LAPLACE_2D : CFMM_TOL_MIN_HELMHOLTZ_2D)
                              : (d->kernel == CFMM_LAPLACE ? CFMM_TOL_MIN_LAPLACE_3D : CFMM_TOL_MIN_HELMHOLTZ_3D);
    if (!(d->tol >= tmin && d->tol < 1.0))
        return fail(CFMM_EINVAL, "tol must lie in [" + std::to_string(tmin) + ", 1) for this kernel: below it "
                                 "the FP64 rounding of the translations sets the error");
    if (d->precision != CFMM_FP64 && d->precision != CFMM_MIXED) return fail(CFMM_EINVAL, "unknown precision");
    if (d->precision == CFMM_MIXED && !(d->tol >= CFMM_MIXED_TOL_MIN))
        return fail(CFMM_EINVAL, "CFMM_MIXED needs tol >= 1e-6 (its FP32 stages round at about 1e-7); "
                                 "use CFMM_FP64 below that");
    if (d->n_src < 1) return fail(CFMM_EINVAL, "n_src must be >= 1");
    if (!d->src) return fail(CFMM_EINVAL, "src is NULL");
    if (d->trg && d->n_trg < 1) return fail(CFMM_EINVAL, "n_trg must be >= 1 when trg is given");
    int64_t ntot = d->n_src + (d->trg ? d->n_trg : 0);
    if (ntot > 0x7fffffffLL) return fail(CFMM_EINVAL, "n_src + n_trg must be below 2^31");
    if (d->leaf_size < 0 || d->leaf_size > 4096) return fail(CFMM_EINVAL, "leaf_size must lie in [0, 4096]");
    if (d->separation < 0 || d->separation > 2) return fail(CFMM_EINVAL, "separation must be 0, 1 or 2");
    if (d->m2l_form < 0 || d->m2l_form > 1) return fail(CFMM_EINVAL, "m2l_form must be 0 or 1");
    int rc = ensure_device_tables();
    if (rc) return rc;
    cfmm_plan_s* p = new cfmm_plan_s();
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(CFMM_EHIP, "hipGetDevice failed");
    }
    p->dim = d->dim;
    p->kernel = d->kernel;
    p->kappa = d->kernel == CFMM_HELMHOLTZ ? d->wavenumber : 0.0;
    p->tol = d->tol;
    p->n_src = d->n_src;
    p->obase = d->trg ? d->n_src : 0;
    p->n_out = d->trg ? d->n_trg : d->n_src;
    p->n = d->n_src + (d->trg ? d->n_trg : 0);
    p->precision = d->precision;
    // default separation: k = 1 in 2D; k = 2 in 3D, where the convergence of the
    // continued expansions degrades fastest with the Lipschitz constant (Sec. 5.1, 6.5)
    p->sep = d->separation ? d->separation : (d->dim == 3 ? 2 : 1);
    p->leaf_size = d->leaf_size ? d->leaf_size : (d->dim == 2 ? 64 : 256);
    p->m2l_form = d->m2l_form;
    p->stream = (hipStream_t)d->stream;
    rc = plan_impl(p, d);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    g_err.clear();
    return CFMM_OK;
}

int cfmm_eval(cfmm_plan_t p, const void* density, void* potential, int on_device)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    if (!density || !potential) return fail(CFMM_EINVAL, "density or potential is NULL");
    hipStream_t st = p->stream;
    const double* sig = (const double*)density;
    double* out = (double*)potential;
    if (!on_device) {
        if (!p->d_io_in) {
            int rc;
            if ((rc = p->alloc(&p->d_io_in, 2 * p->n_src)) || (rc = p->alloc(&p->d_io_out, 2 * p->n_out)))
                return rc;
        }
        HIPCHK(hipMemcpyAsync(p->d_io_in, density, 2 * p->n_src * sizeof(double), hipMemcpyHostToDevice, st));
        sig = p->d_io_in;
        out = p->d_io_out;
    }
    int rc = eval_on_device(p, sig, out);
    if (rc) return rc;
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(potential, p->d_io_out, 2 * p->n_out * sizeof(double), hipMemcpyDeviceToHost, st));
        return check_finite(p);
    }
    return CFMM_OK;
}

int cfmm_plan_timing(cfmm_plan_t p, double* ms)
{
    if (!p || !ms) return fail(CFMM_EINVAL, "plan or ms is NULL");
    for (int k = 0; k < 7; ++k) ms[k] = p->tphase[k];
    return CFMM_OK;
}

int cfmm_sync(cfmm_plan_t p)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    return check_finite(p);
}

int cfmm_eval_layer(cfmm_plan_t p, const void* charge, const void* dipole, void* potential, void* gradient,
                    int on_device)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    if (!charge && !dipole) return fail(CFMM_EINVAL, "charge and dipole are both NULL");
    if (!potential && !gradient) return fail(CFMM_EINVAL, "potential and gradient are both NULL");
    if (!(p->dim == 3 && p->kernel == CFMM_LAPLACE))
        return fail(CFMM_ENOTSUP, "layer potentials (dipoles, gradients) are implemented for dim 3 Laplace");
    hipStream_t st = p->stream;
    int64_t n = p->n;
    int rc;
    if (!p->d_dre) {
        if ((rc = p->alloc(&p->d_dre, 3 * n)) || (rc = p->alloc(&p->d_dim, 3 * n)) ||
            (rc = p->alloc(&p->d_gfar, 3 * n)))
            return rc;
        if (p->n_m2p3 > 0) {
            std::vector<int64_t> p4(p->m2p_poff_h.size());
            for (size_t k = 0; k < p4.size(); ++k) p4[k] = 4 * p->m2p_poff_h[k];
            if ((rc = upload(p, &p->d_m2p_poff4, p4)) || (rc = p->alloc(&p->d_m2p_part4, std::max<int64_t>(1, p4.back()))))
                return rc;
        }
    }
    const double* q = (const double*)charge;
    const double* v = (const double*)dipole;
    double* u = (double*)potential;
    double* g = (double*)gradient;
    if (!on_device) {
        if (!p->d_lio_q) {
            if ((rc = p->alloc(&p->d_lio_q, 2 * p->n_src)) || (rc = p->alloc(&p->d_lio_v, 6 * p->n_src)) ||
                (rc = p->alloc(&p->d_lio_u, 2 * p->n_out)) || (rc = p->alloc(&p->d_lio_g, 6 * p->n_out)))
                return rc;
        }
        if (q) HIPCHK(hipMemcpyAsync(p->d_lio_q, q, 2 * p->n_src * sizeof(double), hipMemcpyHostToDevice, st));
        if (v) HIPCHK(hipMemcpyAsync(p->d_lio_v, v, 6 * p->n_src * sizeof(double), hipMemcpyHostToDevice, st));
        q = q ? p->d_lio_q : nullptr;
        v = v ? p->d_lio_v : nullptr;
        u = u ? p->d_lio_u : nullptr;
        g = g ? p->d_lio_g : nullptr;
    }
    TreeView tv = p->view();
    PointsView pv = p->pview();
    const HostTree& t = p->tree;
    int top = t.top, nlev = t.nlevels(), P = p->pmax;
    const int* W = p->d_work;
    if (q) HIPCHK(launch_gather_density(q, p->io(), n, p->d_sre, p->d_sim, st));
    else {
        HIPCHK(hipMemsetAsync(p->d_sre, 0, n * sizeof(double), st));
        HIPCHK(hipMemsetAsync(p->d_sim, 0, n * sizeof(double), st));
    }
    if (v) HIPCHK(launch_gather_dipole(v, p->io(), n, p->d_dre, p->d_dim, st));
    if (v) HIPCHK(l3d_p2x_dip(W + p->off_p2m, p->n_p2m, P, 0, tv, pv, p->d_dre, p->d_dim, p->d_mpole, st));
    else HIPCHK(l3d_p2m(W + p->off_p2m, p->n_p2m, P, tv, pv, p->d_mpole, st));
    for (int l = nlev - 2; l >= top; --l) HIPCHK(l3d_m2m(W + p->m2m_off[l], p->m2m_cnt[l], P, tv, p->d_mpole, st));
    HIPCHK(run_l3d_m2l(p, tv, P, 0, st));
    if (v) HIPCHK(l3d_p2x_dip(W + p->off_p2l, p->n_p2l, P, 1, tv, pv, p->d_dre, p->d_dim, p->d_local, st));
    else HIPCHK(l3d_p2l(W + p->off_p2l, p->n_p2l, P, tv, pv, p->d_local, st));
    for (int l = top; l + 1 < nlev; ++l) HIPCHK(l3d_l2l(W + p->m2m_off[l], p->m2m_cnt[l], P, tv, p->d_local, st));
    if (g) {
        M2PParts m4{p->n_m2p3, p->d_m2p_owner, p->d_m2p_poff4, p->d_m2p_part4};
        HIPCHK(l3d_leaf_far_grad(W + p->off_leaves, p->nleaf, top, tv, pv, p->d_mpole, p->d_local, m4, p->d_ufar,
                                 p->d_gfar, st));
    } else {
        HIPCHK(l3d_leaf_far(W + p->off_leaves, p->nleaf, top, tv, pv, p->d_mpole, p->d_local, p->m2p_parts(),
                            p->d_ufar, st));
    }
    HIPCHK(l3d_near_layer(W + p->off_leaves, p->nleaf, tv, pv, p->d_dre, p->d_dim, v != nullptr, p->d_ufar,
                          p->d_gfar, p->io(), u, g, st));
    if (!on_device) {
        if (potential)
            HIPCHK(hipMemcpyAsync(potential, p->d_lio_u, 2 * p->n_out * sizeof(double), hipMemcpyDeviceToHost, st));
        if (gradient)
            HIPCHK(hipMemcpyAsync(gradient, p->d_lio_g, 6 * p->n_out * sizeof(double), hipMemcpyDeviceToHost, st));
        return check_finite(p);
    }
    return CFMM_OK;
}

int cfmm_eval_static(cfmm_plan_t p, const void* density, void* potential)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    if (!density || !potential) return fail(CFMM_EINVAL, "density or potential is NULL");
    if (p->n_src + p->n_out > kStaticScratch)
        return fail(CFMM_EINVAL, "n_src + n_trg = " + std::to_string(p->n_src + p->n_out) +
                                     " exceeds the static staging of CFMM_STATIC_MAX = " +
                                     std::to_string(kStaticScratch) + " complex values; use cfmm_eval");
    cplx* scr = static_scratch(p->device);
    if (!scr) return fail(CFMM_EINVAL, "the library was not initialised on the plan's device");
    hipStream_t st = p->stream;
    double* sig = reinterpret_cast<double*>(scr);
    double* out = reinterpret_cast<double*>(scr + p->n_src);
    HIPCHK(hipMemcpyAsync(sig, density, 2 * p->n_src * sizeof(double), hipMemcpyHostToDevice, st));
    int rc = eval_on_device(p, sig, out);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(potential, out, 2 * p->n_out * sizeof(double), hipMemcpyDeviceToHost, st));
    return check_finite(p);
}

}  // extern "C"

namespace {

// Waits for the plan's stream, then reads and clears the non-finite flag.
int check_finite(cfmm_plan_s* p)
{
    hipStream_t st = p->stream;
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, p->d_flag_nf, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!flag) return CFMM_OK;
    int zero = 0;
    HIPCHK(hipMemcpyAsync(p->d_flag_nf, &zero, sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return fail(CFMM_ERANGE, "an evaluation wrote a non-finite potential (inf or NaN): the densities are "
                             "not finite, or the growth e^{kappa |Im r|} of the complexified kernel "
                             "exceeds the FP64 range");
}

// Steps 1-8 of Sec. 6.4 on the plan's stream, densities sig[n_src] and
// potentials out[n_out] in device memory.
int eval_on_device(cfmm_plan_s* p, const double* sig, double* out)
{
    hipStream_t st = p->stream;
    int64_t n = p->n;
    // mode 1 brackets every stage (marks 0..7); mode 2 only the near field
    // (marks 6, 7) and mode 3 only the M2L translations (marks 8, 9), into the
    // next ring slot, so that back-to-back evaluations need no host sync
    int slot = (int)(p->ring_n % cfmm_plan_s::kRing);
    int ring_lo = p->prof == 2 ? 6 : 8;
    auto mark = [&](int i) -> hipError_t {
        if (p->prof == 1 && i < 8) return hipEventRecord(p->ev[i], st);
        if (p->prof >= 2 && (i == ring_lo || i == ring_lo + 1))
            return hipEventRecord(p->rev[2 * slot + (i - ring_lo)], st);
        return hipSuccess;
    };
    TreeView tv = p->view();
    PointsView pv = p->pview();
    const HostTree& t = p->tree;
    int top = t.top, nlev = t.nlevels();
    const int* W = p->d_work;
    HIPCHK(mark(0));
    HIPCHK(launch_gather_density(sig, p->io(), n, p->d_sre, p->d_sim, st));
    HIPCHK(mark(1));
    if (p->dim == 2 && p->kernel == CFMM_LAPLACE) {
        HIPCHK(l2d_p2m(W + p->off_p2m, p->n_p2m, tv, pv, p->d_mpole, st));
        HIPCHK(mark(2));
        for (int l = nlev - 2; l >= top; --l) HIPCHK(l2d_m2m(W + p->m2m_off[l], p->m2m_cnt[l], tv, p->d_mpole, st));
        HIPCHK(mark(3));
        HIPCHK(mark(8));
        HIPCHK(l2d_m2l(W + p->off_m2l, p->n_m2l, tv, p->d_mpole, p->d_local, st));
        HIPCHK(mark(9));
        HIPCHK(l2d_p2l(W + p->off_p2l, p->n_p2l, tv, pv, p->d_local, st));
        HIPCHK(mark(4));
        for (int l = top + 1; l < nlev; ++l) HIPCHK(l2d_l2l(W + p->l2l_off[l], p->l2l_cnt[l], tv, p->d_local, st));
        HIPCHK(mark(5));
        HIPCHK(l2d_leaf_far(W + p->off_leaves, p->nleaf, p->m2p_parts(), top, tv, pv, p->d_mpole, p->d_local,
                            p->d_ufar, st));
        HIPCHK(mark(6));
        HIPCHK(h2d_p2p(p->near2, W + p->off_leaves, p->nleaf, tv, pv, 0.0, p->d_ufar, p->io(), out, 1, st));
    } else if (p->dim == 2) {
        {
            // the P2M list is in level order; one launch per level sizes its LDS by that level's P
            int k0 = 0;
            while (k0 < p->n_p2m) {
                int l = t.level[p->p2m_h[k0]], k1 = k0;
                while (k1 < p->n_p2m && t.level[p->p2m_h[k1]] == l) ++k1;
                HIPCHK(h2d_p2m(W + p->off_p2m + k0, k1 - k0, p->P[l], tv, pv, p->kappa, p->d_mpole, st));
                k0 = k1;
            }
        }
        HIPCHK(mark(2));
        for (int l = nlev - 2; l >= top; --l)
            HIPCHK(h2d_m2m(W + p->m2m_off[l], p->m2m_cnt[l], 2 * p->P[l] + 1, tv, p->ops(), p->d_mpole, st));
        HIPCHK(mark(3));
        HIPCHK(mark(8));
        HIPCHK(h2d_m2l(W + p->off_m2l, p->d_m2lw_grp, p->m2lw_ngrp1, p->m2lw_ngrp, p->m2lw_lds1, p->m2lw_ldsw,
                       p->m2lw_nbox, p->n_m2l, tv, p->ops(), p->d_mpole, p->d_local, st));
        HIPCHK(mark(9));
        {
            // the P2L list is in level order; one launch per level sizes its LDS by that level's P
            int k0 = 0;
            while (k0 < p->n_p2l) {
                int l = t.level[p->p2l_h[k0]], k1 = k0;
                while (k1 < p->n_p2l && t.level[p->p2l_h[k1]] == l) ++k1;
                HIPCHK(h2d_p2l(W + p->off_p2l + k0, k1 - k0, p->P[l], tv, pv, p->kappa, p->d_local, st));
                k0 = k1;
            }
        }
        HIPCHK(mark(4));
        for (int l = top + 1; l < nlev; ++l)
            HIPCHK(h2d_l2l(W + p->l2l_off[l], p->l2l_cnt[l], 2 * p->P[l] + 1, tv, p->ops(), p->d_local, st));
        HIPCHK(mark(5));
        HIPCHK(h2d_leaf_far(W + p->off_leaves, p->nleaf, p->m2p_parts(), p->m2p_pmax, top, tv, pv, p->kappa,
                            p->d_mpole, p->d_local, p->d_ufar, st));
        HIPCHK(mark(6));
        HIPCHK(h2d_p2p(p->near2, W + p->off_leaves, p->nleaf, tv, pv, p->kappa, p->d_ufar, p->io(), out, 0, st));
    } else if (p->kernel == CFMM_HELMHOLTZ) {
        H3DLevels hl{p->d_h3_kw, p->d_h3_sc, nullptr};
        HIPCHK(hipMemsetAsync(p->d_mpole, 0, p->ecount * sizeof(cplx), st));
        HIPCHK(hipMemsetAsync(p->d_local, 0, p->ecount * sizeof(cplx), st));
        // the P2M and P2L lists are in level order; one launch per level sizes
        // its threads and LDS by that level's P
        auto per_level = [&](const std::vector<int>& h, int off, int cnt, bool p2l) -> int {
            int k0 = 0;
            while (k0 < cnt) {
                int l = t.level[h[k0]], k1 = k0;
                while (k1 < cnt && t.level[h[k1]] == l) ++k1;
                if (p2l) HIPCHK(h3d_p2l(W + off + k0, k1 - k0, p->P[l], tv, pv, hl, p->d_local, st));
                else HIPCHK(h3d_p2m(W + off + k0, k1 - k0, p->P[l], tv, pv, hl, p->d_mpole, st));
                k0 = k1;
            }
            return CFMM_OK;
        };
        int rc0;
        if ((rc0 = per_level(p->p2m_h, p->off_p2m, p->n_p2m, false))) return rc0;
        HIPCHK(mark(2));
        auto run = [&](int kind, const cplx* src, cplx* dst) -> int {
            for (const auto& S : p->h3) {
                if (S.kind != kind) continue;
                for (const auto& C : S.chunks) {
                    H3DTr tr;
                    tr.np = C.np;
                    tr.src = p->d_h3_src + C.pair_begin;
                    tr.dst = p->d_h3_dst + C.pair_begin;
                    tr.Ps = S.Ps; tr.Pt = S.Pt; tr.nq = S.nq;
                    tr.src_h = S.src_h; tr.trg_h = S.trg_h;
                    // mixed precision samples the M2L rotations in FP32 (angular
                    // values only; M2M and L2L stay FP64)
                    tr.f32 = kind == 1 && p->precision == CFMM_MIXED && p->tol >= 1e-6;
                    tr.ks = S.ks; tr.sc = S.sc; tr.rs = S.rs_s; tr.inv_w = S.inv_w;
                    tr.sth = p->d_h3_tabd + S.o_nodes;
                    tr.cth = tr.sth + S.nq;
                    tr.W = p->d_h3_tabd + S.o_W;
                    tr.Tc = p->d_h3_tabc + S.o_T;
                    tr.Tdc = tr.Tc + S.Pt + 1;
                    int64_t np = C.np;
                    tr.geo = p->d_h3_scr;
                    tr.FG = tr.geo + 10 * np; tr.sFG = S.sFG;
                    tr.A = tr.FG + S.sFG * np; tr.sA = S.sA;
                    tr.R = tr.A + S.sA * np; tr.sR = S.sR;
                    tr.B = tr.R + S.sR * np; tr.sB = S.sB;
                    HIPCHK(h3d_translate(tr, tv, p->d_eoff, src, p->d_h3_gdst + C.grp_begin,
                                         p->d_h3_goff + C.goff_off, C.ng, p->d_eoff, dst, p->d_h3_eq,
                                         p->d_h3_eq + p->h3_eq_half, st));
                }
            }
            return CFMM_OK;
        };
        int rc;
        if ((rc = run(0, p->d_mpole, p->d_mpole))) return rc;
        HIPCHK(mark(3));
        HIPCHK(mark(8));
        if ((rc = run(1, p->d_mpole, p->d_local))) return rc;
        HIPCHK(mark(9));
        if ((rc0 = per_level(p->p2l_h, p->off_p2l, p->n_p2l, true))) return rc0;
        HIPCHK(mark(4));
        if ((rc = run(2, p->d_local, p->d_local))) return rc;
        HIPCHK(mark(5));
        HIPCHK(h3d_leaf_far(W + p->off_leaves, p->nleaf, top, std::max(1, p->pmax), tv, pv, hl,
                            p->d_mpole, p->d_local, p->m2p_parts(), p->d_ufar, st));
        HIPCHK(mark(6));
        HIPCHK(near3_p2p(p->near3, 1, p->precision, W + p->off_leaves, p->nleaf, tv, pv, p->kappa, p->d_ufar,
                         p->io(), out, st));
    } else {
        int P = p->pmax;
        HIPCHK(l3d_p2m(W + p->off_p2m, p->n_p2m, P, tv, pv, p->d_mpole, st));
        HIPCHK(mark(2));
        for (int l = nlev - 2; l >= top; --l)
            HIPCHK(l3d_m2m(W + p->m2m_off[l], p->m2m_cnt[l], P, tv, p->d_mpole, st));
        HIPCHK(mark(3));
        // FP32 M2L in mixed precision only where its ~1e-7 rounding floor sits
        // below the requested accuracy
        int m2l32 = p->precision == CFMM_MIXED && p->tol >= 1e-6;
        HIPCHK(mark(8));
        HIPCHK(run_l3d_m2l(p, tv, P, m2l32, st));
        HIPCHK(mark(9));
        HIPCHK(l3d_p2l(W + p->off_p2l, p->n_p2l, P, tv, pv, p->d_local, st));
        HIPCHK(mark(4));
        for (int l = top; l + 1 < nlev; ++l)
            HIPCHK(l3d_l2l(W + p->m2m_off[l], p->m2m_cnt[l], P, tv, p->d_local, st));
        HIPCHK(mark(5));
        HIPCHK(l3d_leaf_far(W + p->off_leaves, p->nleaf, top, tv, pv, p->d_mpole, p->d_local,
                            p->m2p_parts(), p->d_ufar, st));
        HIPCHK(mark(6));
        HIPCHK(near3_p2p(p->near3, 0, p->precision, W + p->off_leaves, p->nleaf, tv, pv, 0.0, p->d_ufar,
                         p->io(), out, st));
    }
    HIPCHK(mark(7));
    if (p->prof >= 2) ++p->ring_n;
    return CFMM_OK;
}

}  // namespace

extern "C" {

int cfmm_destroy(cfmm_plan_t p)
{
    delete p;
    return CFMM_OK;
}

int64_t cfmm_plan_bytes(cfmm_plan_t p) { return p ? p->bytes : 0; }

const char* cfmm_last_error(void) { return g_err.c_str(); }

int cfmm_plan_m2l_work(cfmm_plan_t p, int64_t* work4)
{
    if (!p || !work4) return fail(CFMM_EINVAL, "null argument");
    for (int i = 0; i < 4; ++i) work4[i] = p->m2l_work[i];
    return CFMM_OK;
}

int cfmm_plan_info(cfmm_plan_t p, int64_t* info20)
{
    if (!p || !info20) return fail(CFMM_EINVAL, "NULL argument");
    memcpy(info20, p->info, sizeof(p->info));
    return CFMM_OK;
}

int cfmm_plan_near_work(cfmm_plan_t p, int64_t* work2)
{
    if (!p || !work2) return fail(CFMM_EINVAL, "NULL argument");
    work2[0] = p->info[8];
    work2[1] = p->near_evals >= 0 ? p->near_evals : p->info[8];
    return CFMM_OK;
}

int cfmm_plan_nterms(cfmm_plan_t p, int level)
{
    if (!p || level < 0 || level >= (int)p->P.size()) return 0;
    return p->P[level];
}

int cfmm_plan_export_tree(cfmm_plan_t p, int64_t* perm, uint64_t* keys, int32_t* box_level,
                          int32_t* box_parent, int32_t* box_child0, int32_t* box_nchild,
                          int32_t* box_pbeg, int32_t* box_pend, uint64_t* box_prefix)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    const HostTree& t = p->tree;
    size_t nb = t.level.size();
    if (perm) {
        std::vector<int> tmp(p->n);
        HIPCHK(hipMemcpyAsync(tmp.data(), p->d_perm, p->n * sizeof(int), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        for (int64_t i = 0; i < p->n; ++i) perm[i] = tmp[i];
    }
    if (keys) memcpy(keys, p->keys_h.data(), p->n * sizeof(uint64_t));
    if (box_level) memcpy(box_level, t.level.data(), nb * 4);
    if (box_parent) memcpy(box_parent, t.parent.data(), nb * 4);
    if (box_child0) memcpy(box_child0, t.child0.data(), nb * 4);
    if (box_nchild) memcpy(box_nchild, t.nchild.data(), nb * 4);
    if (box_pbeg) memcpy(box_pbeg, t.pbeg.data(), nb * 4);
    if (box_pend) memcpy(box_pend, t.pend.data(), nb * 4);
    if (box_prefix) memcpy(box_prefix, t.prefix.data(), nb * 8);
    return CFMM_OK;
}

int cfmm_plan_export_list(cfmm_plan_t p, int which, int32_t* offsets, int32_t* idx, int64_t* count)
{
    if (!p || which < 1 || which > 4) return fail(CFMM_EINVAL, "bad plan or list number");
    const HostTree& t = p->tree;
    if (count) *count = (int64_t)t.idx[which - 1].size();
    if (offsets) memcpy(offsets, t.off[which - 1].data(), t.off[which - 1].size() * 4);
    if (idx) memcpy(idx, t.idx[which - 1].data(), t.idx[which - 1].size() * 4);
    return CFMM_OK;
}

int cfmm_plan_export_centers(cfmm_plan_t p, void* centers)
{
    if (!p || !centers) return fail(CFMM_EINVAL, "NULL argument");
    memcpy(centers, p->cen_h.data(), p->cen_h.size() * sizeof(double));
    return CFMM_OK;
}

}  // extern "C"

struct cfmm_htree_s {
    HostTree t;
};

extern "C" {

int cfmm_htree_build(cfmm_htree_t* out, int dim, int64_t n, const uint64_t* keys, int leaf_size,
                     int separation, int top)
{
    if (!out || !keys || (dim != 2 && dim != 3) || n < 1 || leaf_size < 1 || separation < 1 ||
        separation > 2 || top < 0)
        return fail(CFMM_EINVAL, "bad argument");
    for (int64_t i = 1; i < n; ++i)
        if (keys[i] < keys[i - 1]) return fail(CFMM_EINVAL, "keys are not sorted");
    cfmm_htree_s* h = new cfmm_htree_s();
    build_topology(keys, n, dim, leaf_size, separation, h->t);
    build_lists(h->t, top);
    *out = h;
    return CFMM_OK;
}

int cfmm_htree_sizes(cfmm_htree_t h, int64_t* s)
{
    if (!h || !s) return fail(CFMM_EINVAL, "NULL argument");
    s[0] = h->t.nbox();
    for (int q = 0; q < 4; ++q) s[1 + q] = (int64_t)h->t.idx[q].size();
    s[5] = h->t.nlevels();
    return CFMM_OK;
}

int cfmm_htree_export(cfmm_htree_t h, int32_t* box_level, int32_t* box_parent, int32_t* box_child0,
                      int32_t* box_nchild, int32_t* box_pbeg, int32_t* box_pend, uint64_t* box_prefix)
{
    if (!h) return fail(CFMM_EINVAL, "NULL argument");
    const HostTree& t = h->t;
    size_t nb = t.level.size();
    if (box_level) memcpy(box_level, t.level.data(), nb * 4);
    if (box_parent) memcpy(box_parent, t.parent.data(), nb * 4);
    if (box_child0) memcpy(box_child0, t.child0.data(), nb * 4);
    if (box_nchild) memcpy(box_nchild, t.nchild.data(), nb * 4);
    if (box_pbeg) memcpy(box_pbeg, t.pbeg.data(), nb * 4);
    if (box_pend) memcpy(box_pend, t.pend.data(), nb * 4);
    if (box_prefix) memcpy(box_prefix, t.prefix.data(), nb * 8);
    return CFMM_OK;
}

int cfmm_htree_export_list(cfmm_htree_t h, int which, int32_t* offsets, int32_t* idx)
{
    if (!h || which < 1 || which > 4) return fail(CFMM_EINVAL, "bad argument");
    const HostTree& t = h->t;
    if (offsets) memcpy(offsets, t.off[which - 1].data(), t.off[which - 1].size() * 4);
    if (idx) memcpy(idx, t.idx[which - 1].data(), t.idx[which - 1].size() * 4);
    return CFMM_OK;
}

int cfmm_htree_free(cfmm_htree_t h)
{
    delete h;
    return CFMM_OK;
}

int cfmm_nterms(int dim, int kernel, double kappa, double w, int separation, double eps, int pmax)
{
    if ((dim != 2 && dim != 3) || kernel != CFMM_HELMHOLTZ || !(kappa > 0) || !(w > 0) ||
        separation < 1 || separation > 2 || !(eps > 0) || pmax < 1 ||
        pmax > (dim == 2 ? kPMax2D : kPMaxH3))
        return fail(CFMM_EINVAL, "bad argument");
    if (dim == 3) return h3d_nterms(kappa, w, separation, eps, pmax);
    return nterms_level(dim, separation, kappa, w, eps, pmax);
}

int cfmm_plan_export_expansions(cfmm_plan_t p, void* mpole, void* local, int64_t* offsets,
                                int64_t* count)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    const HostTree& t = p->tree;
    int nb = t.nbox();
    int64_t tot = 0;
    for (int b = 0; b < nb; ++b) {
        int64_t nc = 0;
        if (t.level[b] >= t.top) {
            int P = p->P[t.level[b]];
            nc = p->dim == 2 ? 2 * P + 1 : (int64_t)(P + 1) * (P + 1);
        }
        if (offsets) offsets[b] = nc ? tot : -1;
        tot += nc;
    }
    if (count) *count = tot;
    HIPCHK(hipStreamSynchronize(p->stream));
    if (mpole && tot) HIPCHK(hipMemcpy(mpole, p->d_mpole, tot * sizeof(cplx), hipMemcpyDeviceToHost));
    if (local && tot) HIPCHK(hipMemcpy(local, p->d_local, tot * sizeof(cplx), hipMemcpyDeviceToHost));
    return CFMM_OK;
}

int cfmm_set_profiling(cfmm_plan_t p, int mode)
{
    if (!p) return fail(CFMM_EINVAL, "plan is NULL");
    if (mode < 0 || mode > 3) return fail(CFMM_EINVAL, "profiling mode must be 0, 1, 2 or 3");
    // the events are made here, so that an evaluation creates nothing
    if (mode == 1 && !p->ev_made) {
        for (int i = 0; i < 8; ++i) HIPCHK(hipEventCreate(&p->ev[i]));
        p->ev_made = true;
    }
    if (mode >= 2 && !p->rev_made) {
        for (int i = 0; i < 2 * cfmm_plan_s::kRing; ++i) HIPCHK(hipEventCreate(&p->rev[i]));
        p->rev_made = true;
    }
    p->prof = mode;
    if (mode >= 2) p->ring_n = 0;
    return CFMM_OK;
}

int cfmm_ring_ms(cfmm_plan_t p, double* total_ms, int* count)
{
    if (!p || !total_ms || !count) return fail(CFMM_EINVAL, "bad argument");
    int n = (int)(p->ring_n < cfmm_plan_s::kRing ? p->ring_n : cfmm_plan_s::kRing);
    double tot = 0.0;
    for (int s = 0; s < n; ++s) {
        float f = 0.0f;
        HIPCHK(hipEventElapsedTime(&f, p->rev[2 * s], p->rev[2 * s + 1]));
        tot += f;
    }
    *total_ms = tot;
    *count = n;
    return CFMM_OK;
}

int cfmm_stage_ms(cfmm_plan_t p, int stage, double* ms)
{
    if (!p || !ms || stage < 0 || stage > 7) return fail(CFMM_EINVAL, "bad argument");
    if (!p->ev_made) return fail(CFMM_EINVAL, "profiling was not enabled before the evaluation");
    float f = 0.0f;
    if (stage == 7) {
        HIPCHK(hipEventElapsedTime(&f, p->ev[0], p->ev[7]));
    } else {
        HIPCHK(hipEventElapsedTime(&f, p->ev[stage], p->ev[stage + 1]));
    }
    *ms = f;
    return CFMM_OK;
}

}  // extern "C"
