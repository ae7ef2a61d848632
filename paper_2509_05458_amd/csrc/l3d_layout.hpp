// LDS layout of the 3D Laplace M2L translation table and the assignment of
// output groups to lanes (host side, computed once per expansion length P).
//
// The kernel's lane owning outputs (j, k0..k0+3), k0 = -j + 4g, reads at one
// step the table entry (l, q) = (j + n, m - k0 - c): in a row whose q = 0
// entry sits at a multiple of 16 entries (16-byte entries, so 256 bytes), its
// 16-byte bank slot is (m - c + j - 4g) mod 16.  Lanes are therefore grouped
// in sixteens by the class (j - 4g) mod 16, one group of each class per
// sixteen where the classes allow it, so that the sixteen reads of a step fall
// in distinct slots; a slot left without a group repeats the address of the
// first group of its sixteen (a broadcast) and writes nothing.
//
// Rows: entry (l, q) is stored at base[l] + q for q in [-l-3, l] (the three
// extra entries below -l are the zero guards that discarded orders read);
// rows are packed in order of l with base[l] = 0 mod 16.
#pragma once
#include <cstddef>
#include <vector>

namespace cfmm {

struct L3dM2LLayout {
    int P = 0;
    int R = 0;                 // groups per lane
    int entries = 0;           // table entries (16 bytes each)
    std::vector<int> base;     // 2P+1 row bases (index of q = 0)
    std::vector<int> slot;     // 64 R lane slots: j | g << 8 | active << 16
};

// Rows n <= Ps of an M2L pair's contraction dealt to W wavefronts: each row
// (2n + 1 steps) runs as chunks of six steps, the last one zero-padded, plus a
// window start of about three steps; rows go to the least loaded wavefront,
// longest first.  mask[Ps * W + w] has bit n set when wavefront w takes row n.
inline std::vector<unsigned> l3d_m2l_rows(int W)
{
    std::vector<unsigned> mask(32 * (size_t)W, 0u);
    for (int Ps = 0; Ps < 32; ++Ps) {
        std::vector<int> rows(Ps + 1), load(W, 0);
        auto cost = [](int n) { return 6 * ((2 * n + 1 + 5) / 6) + 3; };
        for (int n = 0; n <= Ps; ++n) rows[n] = Ps - n;          // longest first
        for (int n : rows) {
            int best = 0;
            for (int w = 1; w < W; ++w)
                if (load[w] < load[best]) best = w;
            load[best] += cost(n);
            mask[(size_t)Ps * W + best] |= 1u << n;
        }
    }
    return mask;
}

inline L3dM2LLayout l3d_m2l_layout(int P)
{
    L3dM2LLayout L;
    L.P = P;
    std::vector<std::vector<int>> cls(16);   // groups by class, in (j, g) order
    int G = 0;
    for (int j = 0; j <= P; ++j)
        for (int g = 0; g <= j / 2; ++g, ++G) cls[((j - 4 * g) % 16 + 16) % 16].push_back(j | g << 8);
    L.R = (G + 63) / 64;
    int npass = 4 * L.R;
    std::vector<int> s(64 * L.R, -1);
    std::vector<std::size_t> next(16, 0);
    for (int p = 0; p < npass; ++p)
        for (int c = 0; c < 16; ++c)
            if (next[c] < cls[c].size()) s[16 * p + c] = cls[c][next[c]++];
    // groups beyond one per sixteen go to the sixteen holding the fewest of
    // their class (first such sixteen with a free slot)
    for (int c = 0; c < 16; ++c)
        for (; next[c] < cls[c].size(); ++next[c]) {
            int v = cls[c][next[c]], bestp = -1, bestn = 1 << 30;
            for (int p = 0; p < npass; ++p) {
                bool hole = false;
                int same = 0;
                for (int i = 0; i < 16; ++i) {
                    int u = s[16 * p + i];
                    if (u < 0) hole = true;
                    else if ((((u & 255) - 4 * (u >> 8)) % 16 + 16) % 16 == c) ++same;
                }
                if (hole && same < bestn) { bestn = same; bestp = p; }
            }
            for (int i = 0; i < 16; ++i)
                if (s[16 * bestp + i] < 0) { s[16 * bestp + i] = v; break; }
        }
    L.slot.assign(64 * L.R, 0);
    for (int p = 0; p < npass; ++p) {
        int first = 0;
        for (int i = 0; i < 16; ++i)
            if (s[16 * p + i] >= 0) { first = s[16 * p + i]; break; }
        for (int i = 0; i < 16; ++i) {
            int u = s[16 * p + i];
            L.slot[16 * p + i] = u >= 0 ? (u | 1 << 16) : first;
        }
    }
    L.base.assign(2 * P + 1, 0);
    int a = 3;
    for (int l = 0; l <= 2 * P; ++l) {
        int lo = a + l + 3;
        lo = (lo + 15) & ~15;
        L.base[l] = lo;
        a = lo + l + 1;
    }
    L.entries = a + 4;
    return L;
}

}  // namespace cfmm
