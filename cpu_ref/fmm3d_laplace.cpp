// CPU FMM reference for the 3D Laplace single layer at complex points: the
// baseline the GPU path is timed against on the host's cores (not an oracle:
// the oracle is the direct sum).  The same method as the library (Sec. 5.2,
// 6.1-6.4): the adaptive tree and Lists 1-4 from the library's host planning
// logic (cfmm_htree_*, the C-ABI), complexified centres, P from (r/R)^n <= tol
// with R = (k + 1/2) w (per M2L pair from its own nearest target distance),
// and P2M, M2M, M2L, L2L, L2P, M2P, P2L, P2P with the solid-harmonic addition
// theorems at complex offsets, in plain C++ with OpenMP over boxes.
//
//   R_n^m(x) = rho^n P_n^m e^{i m phi} / (n+m)!,   I_n^m(x) = (n-m)! P_n^m e^{i m phi} / rho^{n+1}
//   1/|X - Y| = sum (-1)^m R_n^{-m}(Y) I_n^m(X)            (|Y| < |X|)
//   R_n^m(X + Y) = sum_{j,k} R_j^k(X) R_{n-j}^{m-k}(Y)
// Coordinates of level l are scaled by 1/w_l: M = sum sigma (-1)^m R_n^{-m}(Y/w),
// u = (1/w) sum M I(X/w); L = sum sigma (-1)^m I_n^{-m}(Y/w), u = (1/w) sum L R(X/w).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "../include/cfmm.h"

namespace {

typedef std::complex<double> cd;

inline int idx(int n, int m) { return n * n + n + m; }

// all R_n^m (or I_n^m), n <= P, by the Cartesian recurrences; out[(P+1)^2]
void solid_R(cd x, cd y, cd z, int P, cd* out)
{
    cd r2 = x * x + y * y + z * z;
    for (int s = 0; s < 2; ++s) {
        cd w = s == 0 ? x + cd(0, 1) * y : x - cd(0, 1) * y;
        cd d = 1.0;
        for (int m = 0; m <= P; ++m) {
            if (m > 0) d = d * w / (2.0 * m);
            double sg = (s == 1 && (m & 1)) ? -1.0 : 1.0;
            if (s == 1 && m == 0) continue;
            int mm = s == 0 ? m : -m;
            cd a = d * sg;
            out[idx(m, mm)] = a;
            if (m + 1 > P) continue;
            cd b = z * a;
            out[idx(m + 1, mm)] = b;
            for (int n = m + 2; n <= P; ++n) {
                cd c = ((2.0 * n - 1.0) * z * b - r2 * a) / ((double)(n + m) * (double)(n - m));
                out[idx(n, mm)] = c;
                a = b;
                b = c;
            }
        }
    }
}

void solid_I(cd x, cd y, cd z, int P, cd* out)
{
    cd r2 = x * x + y * y + z * z;
    cd rho = std::sqrt(r2);          // principal
    for (int s = 0; s < 2; ++s) {
        cd w = s == 0 ? x + cd(0, 1) * y : x - cd(0, 1) * y;
        cd d = 1.0 / rho;
        for (int m = 0; m <= P; ++m) {
            if (m > 0) d = d * (2.0 * m - 1.0) * w / r2;
            double sg = (s == 1 && (m & 1)) ? -1.0 : 1.0;
            if (s == 1 && m == 0) continue;
            int mm = s == 0 ? m : -m;
            cd a = d * sg;
            out[idx(m, mm)] = a;
            if (m + 1 > P) continue;
            cd b = (2.0 * m + 1.0) * z * a / r2;
            out[idx(m + 1, mm)] = b;
            for (int n = m + 2; n <= P; ++n) {
                cd c = ((2.0 * n - 1.0) * z * b - (double)(n + m - 1) * (double)(n - m - 1) * a) / r2;
                out[idx(n, mm)] = c;
                a = b;
                b = c;
            }
        }
    }
}

struct Tree {
    int nb = 0, nlev = 0, top = 2;
    std::vector<int32_t> level, parent, child0, nchild, pbeg, pend, loff[4], lidx[4];
    std::vector<uint64_t> prefix;
};

}  // namespace

extern "C" {

// u[i] = sum_{j != i} sigma_j / (4 pi r_ij) at the n points (complex128[n][3]);
// sigma, u complex128[n].  times[0] = plan seconds (keys, sort, tree,
// lists, centres), times[1] = evaluation seconds.  Returns 0, or a negative
// value (a cfmm_htree error or bad arguments).
int cpu_fmm3d_laplace(int64_t n, const double* pts, const double* sigma, double tol, int leaf_size, int sep,
                      double* u, int nthreads, double* times)
{
    if (n < 2 || !(tol > 0 && tol < 1) || leaf_size < 1 || sep < 1 || sep > 2) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    auto t0 = std::chrono::steady_clock::now();
    const cd* X = reinterpret_cast<const cd*>(pts);
    const cd* S = reinterpret_cast<const cd*>(sigma);
    // root cube and Morton keys of the real parts (21 bits per coordinate)
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = 1e300; hi[d] = -1e300; }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], X[i * 3 + d].real());
            hi[d] = std::max(hi[d], X[i * 3 + d].real());
        }
    double ext = 0.0, mid[3];
    for (int d = 0; d < 3; ++d) { mid[d] = 0.5 * (lo[d] + hi[d]); ext = std::max(ext, hi[d] - lo[d]); }
    double D = ext > 0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
    double scale = std::ldexp(1.0, 21) / D, qtop = std::ldexp(1.0, 21) - 1.0;
    std::vector<std::pair<uint64_t, int64_t>> kv(n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t key = 0;
        for (int d = 0; d < 3; ++d) {
            double q = std::floor((X[i * 3 + d].real() - (mid[d] - 0.5 * D)) * scale);
            q = std::min(std::max(q, 0.0), qtop);
            uint64_t qi = (uint64_t)q;
            for (int b = 0; b < 21; ++b) key |= ((qi >> b) & 1ull) << (3 * b + d);
        }
        kv[i] = {key, i};
    }
    std::stable_sort(kv.begin(), kv.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    std::vector<uint64_t> keys(n);
    std::vector<int64_t> perm(n);
    for (int64_t i = 0; i < n; ++i) { keys[i] = kv[i].first; perm[i] = kv[i].second; }
    cfmm_htree_t h = nullptr;
    int top = 2;
    int rc = cfmm_htree_build(&h, 3, n, keys.data(), leaf_size, sep, top);
    if (rc) return rc;
    int64_t sz[6];
    cfmm_htree_sizes(h, sz);
    Tree t;
    t.nb = (int)sz[0];
    t.nlev = (int)sz[5];
    for (auto* v : {&t.level, &t.parent, &t.child0, &t.nchild, &t.pbeg, &t.pend}) v->resize(t.nb);
    t.prefix.resize(t.nb);
    cfmm_htree_export(h, t.level.data(), t.parent.data(), t.child0.data(), t.nchild.data(), t.pbeg.data(),
                      t.pend.data(), t.prefix.data());
    for (int q = 0; q < 4; ++q) {
        t.loff[q].resize(t.nb + 1);
        t.lidx[q].resize(std::max<int64_t>(1, sz[1 + q]));
        cfmm_htree_export_list(h, q + 1, t.loff[q].data(), t.lidx[q].data());
    }
    cfmm_htree_free(h);
    // sorted points, densities, complexified centres
    std::vector<cd> Y(3 * n), sg(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) Y[3 * i + d] = X[3 * perm[i] + d];
        sg[i] = S[perm[i]];
    }
    std::vector<cd> cen(3 * (size_t)t.nb);
    std::vector<double> w(t.nb);
    for (int b = 0; b < t.nb; ++b) {
        int l = t.level[b];
        w[b] = D * std::ldexp(1.0, -l);
        int64_t c[3] = {0, 0, 0};
        for (int bit = 0; bit < l; ++bit)
            for (int d = 0; d < 3; ++d) c[d] |= (int64_t)((t.prefix[b] >> (3 * bit + d)) & 1ull) << bit;
        double ims[3] = {0, 0, 0};
        for (int i = t.pbeg[b]; i < t.pend[b]; ++i)
            for (int d = 0; d < 3; ++d) ims[d] += Y[3 * i + d].imag();
        int cnt = t.pend[b] - t.pbeg[b];
        for (int d = 0; d < 3; ++d)
            cen[3 * b + d] = cd(mid[d] - 0.5 * D + (c[d] + 0.5) * w[b], ims[d] / std::max(1, cnt));
    }
    int P = 1;
    double ratio = std::sqrt(3.0) * 0.5 / (0.5 + sep);
    while (std::pow(ratio, P) > tol && P < 60) ++P;
    int pd[8];
    for (int d = 0; d < 8; ++d) {
        pd[d] = P;
        if (d > sep) {
            double rr = std::sqrt(3.0) * 0.5 / (d - 0.5);
            int m = 1;
            while (std::pow(rr, m) > tol && m < P) ++m;
            pd[d] = m;
        }
    }
    int nc = (P + 1) * (P + 1);
    auto t1 = std::chrono::steady_clock::now();
    // ----------------------------------------------------------------- eval
    std::vector<cd> M((size_t)t.nb * nc, 0.0), L((size_t)t.nb * nc, 0.0), uf(n, 0.0);
    auto rel = [&](int64_t i, int b, double s, cd* o) {
        for (int d = 0; d < 3; ++d) o[d] = (Y[3 * i + d] - cen[3 * b + d]) * s;
    };
    // P2M
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < t.nb; ++b) {
        if (t.nchild[b] || t.level[b] < top) continue;
        std::vector<cd> Rv(nc);
        cd* Mb = &M[(size_t)b * nc];
        for (int i = t.pbeg[b]; i < t.pend[b]; ++i) {
            cd y[3];
            rel(i, b, 1.0 / w[b], y);
            solid_R(y[0], y[1], y[2], P, Rv.data());
            for (int nn = 0; nn <= P; ++nn)
                for (int m = -nn; m <= nn; ++m)
                    Mb[idx(nn, m)] += sg[i] * ((m & 1) ? -1.0 : 1.0) * Rv[idx(nn, -m)];
        }
    }
    // M2M, level by level upward
    for (int l = t.nlev - 2; l >= top; --l) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int b = 0; b < t.nb; ++b) {
            if (t.level[b] != l || !t.nchild[b]) continue;
            std::vector<cd> Rv(nc);
            cd* Mb = &M[(size_t)b * nc];
            for (int c = t.child0[b]; c < t.child0[b] + t.nchild[b]; ++c) {
                cd d[3];
                for (int k = 0; k < 3; ++k) d[k] = (cen[3 * c + k] - cen[3 * b + k]) / w[b];
                solid_R(d[0], d[1], d[2], P, Rv.data());
                const cd* Mc = &M[(size_t)c * nc];
                for (int nn = 0; nn <= P; ++nn)
                    for (int m = -nn; m <= nn; ++m) {
                        cd a = 0.0;
                        double hh = 1.0;
                        for (int j = 0; j <= nn; ++j, hh *= 0.5)
                            for (int k = -j; k <= j; ++k) {
                                int q = m - k, lm = nn - j;
                                if (q > lm || q < -lm) continue;
                                a += hh * Mc[idx(j, k)] * ((q & 1) ? -1.0 : 1.0) * Rv[idx(lm, -q)];
                            }
                        Mb[idx(nn, m)] += a;
                    }
            }
        }
    }
    // M2L (per pair, the source contracted to its own length) and P2L
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < t.nb; ++b) {
        if (t.level[b] < top) continue;
        std::vector<cd> Iv((2 * P + 1) * (2 * P + 1));
        cd* Lb = &L[(size_t)b * nc];
        for (int e = t.loff[1][b]; e < t.loff[1][b + 1]; ++e) {
            int a = t.lidx[1][e];
            cd D3[3];
            double dm = 0.0;
            for (int k = 0; k < 3; ++k) {
                D3[k] = (cen[3 * b + k] - cen[3 * a + k]) / w[b];
                dm = std::max(dm, std::fabs(D3[k].real()));
            }
            int dd = (int)(dm + 0.5);
            int Ps = pd[dd < 7 ? dd : 7];
            solid_I(D3[0], D3[1], D3[2], P + Ps, Iv.data());
            const cd* Ma = &M[(size_t)a * nc];
            for (int j = 0; j <= P; ++j)
                for (int k = -j; k <= j; ++k) {
                    cd acc = 0.0;
                    for (int nn = 0; nn <= Ps; ++nn)
                        for (int m = -nn; m <= nn; ++m) acc += Ma[idx(nn, m)] * Iv[idx(j + nn, m - k)];
                    Lb[idx(j, k)] += ((j + k) & 1) ? -acc : acc;
                }
        }
        std::vector<cd> Jv(nc);
        for (int e = t.loff[3][b]; e < t.loff[3][b + 1]; ++e) {
            int a = t.lidx[3][e];
            for (int i = t.pbeg[a]; i < t.pend[a]; ++i) {
                cd y[3];
                rel(i, b, 1.0 / w[b], y);
                solid_I(y[0], y[1], y[2], P, Jv.data());
                for (int nn = 0; nn <= P; ++nn)
                    for (int m = -nn; m <= nn; ++m)
                        Lb[idx(nn, m)] += sg[i] * ((m & 1) ? -1.0 : 1.0) * Jv[idx(nn, -m)];
            }
        }
    }
    // L2L, level by level downward
    for (int l = top + 1; l < t.nlev; ++l) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int c = 0; c < t.nb; ++c) {
            if (t.level[c] != l) continue;
            int p = t.parent[c];
            std::vector<cd> Rv(nc);
            cd d[3];
            for (int k = 0; k < 3; ++k) d[k] = (cen[3 * c + k] - cen[3 * p + k]) / w[p];
            solid_R(d[0], d[1], d[2], P, Rv.data());
            const cd* Lp = &L[(size_t)p * nc];
            cd* Lc = &L[(size_t)c * nc];
            for (int j = 0; j <= P; ++j) {
                double f = std::ldexp(1.0, -(j + 1));
                for (int k = -j; k <= j; ++k) {
                    cd a = 0.0;
                    for (int nn = j; nn <= P; ++nn)
                        for (int m = -nn; m <= nn; ++m) {
                            int q = m - k, lm = nn - j;
                            if (q > lm || q < -lm) continue;
                            a += Lp[idx(nn, m)] * Rv[idx(lm, q)];
                        }
                    Lc[idx(j, k)] += f * a;
                }
            }
        }
    }
    // L2P, M2P (List 3) and P2P (List 1), by target leaf
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < t.nb; ++b) {
        if (t.nchild[b]) continue;
        std::vector<cd> Rv(nc);
        for (int i = t.pbeg[b]; i < t.pend[b]; ++i) {
            cd acc = 0.0;
            if (t.level[b] >= top) {
                cd x[3];
                rel(i, b, 1.0 / w[b], x);
                solid_R(x[0], x[1], x[2], P, Rv.data());
                const cd* Lb = &L[(size_t)b * nc];
                cd s = 0.0;
                for (int k = 0; k < nc; ++k) s += Lb[k] * Rv[k];
                acc += s / w[b];
                for (int e = t.loff[2][b]; e < t.loff[2][b + 1]; ++e) {
                    int a = t.lidx[2][e];
                    rel(i, a, 1.0 / w[a], x);
                    solid_I(x[0], x[1], x[2], P, Rv.data());
                    const cd* Ma = &M[(size_t)a * nc];
                    cd s2 = 0.0;
                    for (int k = 0; k < nc; ++k) s2 += Ma[k] * Rv[k];
                    acc += s2 / w[a];
                }
            }
            for (int e = t.loff[0][b]; e < t.loff[0][b + 1]; ++e) {
                int a = t.lidx[0][e];
                for (int j = t.pbeg[a]; j < t.pend[a]; ++j) {
                    if (j == i) continue;
                    cd s2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        cd dd = Y[3 * i + d] - Y[3 * j + d];
                        s2 += dd * dd;
                    }
                    if (s2 == cd(0.0, 0.0)) continue;
                    acc += sg[j] / std::sqrt(s2);
                }
            }
            uf[i] = acc;
        }
    }
    cd* U = reinterpret_cast<cd*>(u);
    for (int64_t i = 0; i < n; ++i) U[perm[i]] = uf[i] / (4.0 * M_PI);
    auto t2 = std::chrono::steady_clock::now();
    if (times) {
        times[0] = std::chrono::duration<double>(t1 - t0).count();
        times[1] = std::chrono::duration<double>(t2 - t1).count();
    }
    return 0;
}

}  // extern "C"
