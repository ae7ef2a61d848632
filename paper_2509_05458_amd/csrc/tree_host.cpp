// Host-side tree topology and interaction lists (Sec. 6.1, Sec. 6.2).
//
// Readings of the paper fixed here:
//  * a box with more than N_s points splits into its non-empty children;
//  * near zone: boxes a, b are near iff ||x_a - x_b||_inf <= (k/2)(w_a + w_b)
//    (real centres and widths), tested exactly in integer units of the finest
//    grid; colleagues are same-level near boxes;
//  * level restriction: two leaves whose levels differ by two or more are never
//    near; the coarser leaf is split until that holds (coarsest such tree);
//  * List 1 (leaf b): leaves near b, b included; List 2: same-level boxes not
//    near b whose parent is near b's parent; List 3 (leaf b): finer boxes not
//    near b whose parent is near b; List 4: transpose of List 3.
#include "tree_host.hpp"

#include <algorithm>
#include <unordered_map>

namespace cfmm {

namespace {

struct Node {
    int level;
    uint64_t prefix;
    int pbeg, pend;
    int first = -1, nchild = 0, parent = -1;
};

uint64_t coords_to_prefix(const int64_t* c, int level, int dim)
{
    uint64_t p = 0;
    for (int b = 0; b < level; ++b)
        for (int d = 0; d < dim; ++d) p |= (uint64_t)((c[d] >> b) & 1) << (b * dim + d);
    return p;
}

void prefix_to_coords(uint64_t p, int level, int dim, int64_t* c)
{
    for (int d = 0; d < dim; ++d) c[d] = 0;
    for (int b = 0; b < level; ++b)
        for (int d = 0; d < dim; ++d) c[d] |= (int64_t)((p >> (b * dim + d)) & 1) << b;
}

struct Builder {
    const uint64_t* keys;
    int64_t n;
    int dim, B, ns, sep;
    std::vector<Node> nodes;
    std::vector<std::unordered_map<uint64_t, int>> lookup;

    int add(int level, uint64_t prefix, int b0, int b1, int parent)
    {
        Node nd;
        nd.level = level;
        nd.prefix = prefix;
        nd.pbeg = b0;
        nd.pend = b1;
        nd.parent = parent;
        nodes.push_back(nd);
        if ((int)lookup.size() <= level) lookup.resize(level + 1);
        lookup[level][prefix] = (int)nodes.size() - 1;
        return (int)nodes.size() - 1;
    }

    void split(int i)
    {
        int level = nodes[i].level;
        int shift = dim * (B - level - 1);
        int b0 = nodes[i].pbeg, b1 = nodes[i].pend;
        int start = b0;
        uint64_t cur = keys[b0] >> shift;
        int first = -1, cnt = 0;
        for (int j = b0 + 1; j <= b1; ++j) {
            uint64_t v = (j < b1) ? (keys[j] >> shift) : ~0ull;
            if (j == b1 || v != cur) {
                int c = add(level + 1, cur, start, j, i);
                if (first < 0) first = c;
                ++cnt;
                start = j;
                cur = v;
            }
        }
        nodes[i].first = first;
        nodes[i].nchild = cnt;
    }

    void centre_units(int i, int64_t* c, int64_t* w) const
    {
        int64_t q[3];
        prefix_to_coords(nodes[i].prefix, nodes[i].level, dim, q);
        int sh = B - nodes[i].level;
        for (int d = 0; d < dim; ++d) c[d] = (2 * q[d] + 1) << sh;
        *w = (int64_t)1 << (B + 1 - nodes[i].level);
    }

    bool near(int a, int b) const
    {
        int64_t ca[3], cb[3], wa, wb;
        centre_units(a, ca, &wa);
        centre_units(b, cb, &wb);
        for (int d = 0; d < dim; ++d) {
            int64_t dd = ca[d] - cb[d];
            if (dd < 0) dd = -dd;
            if (2 * dd > (int64_t)sep * (wa + wb)) return false;
        }
        return true;
    }
};

}  // namespace

void box_coords(const HostTree& t, int b, int64_t* c)
{
    prefix_to_coords(t.prefix[b], t.level[b], t.dim, c);
}

void build_topology(const uint64_t* keys, int64_t n, int dim, int leaf_size, int sep, HostTree& t)
{
    Builder bl;
    bl.keys = keys;
    bl.n = n;
    bl.dim = dim;
    bl.B = (dim == 2) ? 31 : 21;
    bl.ns = leaf_size;
    bl.sep = sep;
    bl.nodes.reserve((size_t)(4 * n / (leaf_size > 0 ? leaf_size : 1)) + 64);
    bl.add(0, 0, 0, (int)n, -1);
    // refinement by occupancy, level by level
    std::vector<int> frontier{0}, next;
    while (!frontier.empty()) {
        next.clear();
        for (int i : frontier) {
            if (bl.nodes[i].pend - bl.nodes[i].pbeg > leaf_size && bl.nodes[i].level < bl.B) {
                bl.split(i);
                for (int c = 0; c < bl.nodes[i].nchild; ++c) next.push_back(bl.nodes[i].first + c);
            }
        }
        frontier.swap(next);
    }
    // level restriction
    std::vector<char> has_leaf;
    for (;;) {
        int maxl = 0;
        for (auto& nd : bl.nodes) maxl = std::max(maxl, nd.level);
        has_leaf.assign(maxl + 1, 0);
        for (auto& nd : bl.nodes)
            if (nd.nchild == 0) has_leaf[nd.level] = 1;
        std::vector<int> marks;
        std::vector<char> marked(bl.nodes.size(), 0);
        int64_t span = sep;
        for (int b = 0; b < (int)bl.nodes.size(); ++b) {
            const Node& nb = bl.nodes[b];
            if (nb.nchild != 0 || nb.level < 2) continue;
            int64_t cb[3];
            prefix_to_coords(nb.prefix, nb.level, dim, cb);
            for (int lp = nb.level - 2; lp >= 0; --lp) {
                if (!has_leaf[lp]) continue;
                int64_t A[3];
                for (int d = 0; d < dim; ++d) A[d] = cb[d] >> (nb.level - lp);
                int64_t lim = ((int64_t)1 << lp) - 1;
                int64_t o[3] = {0, 0, 0};
                int cnt = 1;
                for (int d = 0; d < dim; ++d) cnt *= (int)(2 * span + 1);
                for (int q = 0; q < cnt; ++q) {
                    int rem = q;
                    int64_t cc[3];
                    bool ok = true;
                    for (int d = 0; d < dim; ++d) {
                        o[d] = (rem % (2 * span + 1)) - span;
                        rem /= (int)(2 * span + 1);
                        cc[d] = A[d] + o[d];
                        if (cc[d] < 0 || cc[d] > lim) ok = false;
                    }
                    if (!ok) continue;
                    auto it = bl.lookup[lp].find(coords_to_prefix(cc, lp, dim));
                    if (it == bl.lookup[lp].end()) continue;
                    int a = it->second;
                    if (bl.nodes[a].nchild == 0 && !marked[a] && bl.near(a, b)) {
                        marked[a] = 1;
                        marks.push_back(a);
                    }
                }
            }
        }
        if (marks.empty()) break;
        for (int a : marks) bl.split(a);
    }
    // number boxes in (level, prefix) order
    int nb = (int)bl.nodes.size();
    std::vector<int> order(nb);
    for (int i = 0; i < nb; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (bl.nodes[a].level != bl.nodes[b].level) return bl.nodes[a].level < bl.nodes[b].level;
        return bl.nodes[a].prefix < bl.nodes[b].prefix;
    });
    std::vector<int> rank(nb);
    for (int i = 0; i < nb; ++i) rank[order[i]] = i;
    t.dim = dim;
    t.nbits = bl.B;
    t.sep = sep;
    t.n = n;
    t.level.resize(nb);
    t.parent.resize(nb);
    t.child0.resize(nb);
    t.nchild.resize(nb);
    t.pbeg.resize(nb);
    t.pend.resize(nb);
    t.prefix.resize(nb);
    int maxl = 0;
    for (int i = 0; i < nb; ++i) {
        const Node& nd = bl.nodes[order[i]];
        t.level[i] = nd.level;
        t.prefix[i] = nd.prefix;
        t.pbeg[i] = nd.pbeg;
        t.pend[i] = nd.pend;
        t.parent[i] = nd.parent >= 0 ? rank[nd.parent] : -1;
        t.nchild[i] = nd.nchild;
        t.child0[i] = -1;
        maxl = std::max(maxl, nd.level);
    }
    for (int i = 0; i < nb; ++i) {
        int p = t.parent[i];
        if (p >= 0 && (t.child0[p] < 0 || i < t.child0[p])) t.child0[p] = i;
    }
    t.lvl_beg.assign(maxl + 2, 0);
    for (int i = 0; i < nb; ++i) t.lvl_beg[t.level[i] + 1]++;
    for (int l = 0; l <= maxl; ++l) t.lvl_beg[l + 1] += t.lvl_beg[l];
}

void build_lists(HostTree& t, int top)
{
    int nb = t.nbox(), dim = t.dim, B = t.nbits;
    t.top = top;
    std::vector<int64_t> cen((size_t)nb * 3), wid(nb);
    for (int b = 0; b < nb; ++b) {
        int64_t q[3];
        prefix_to_coords(t.prefix[b], t.level[b], dim, q);
        int sh = B - t.level[b];
        for (int d = 0; d < dim; ++d) cen[(size_t)b * 3 + d] = (2 * q[d] + 1) << sh;
        wid[b] = (int64_t)1 << (B + 1 - t.level[b]);
    }
    int64_t k = t.sep;
    auto near = [&](int a, int b) {
        if (t.level[a] < top || t.level[b] < top) return true;
        for (int d = 0; d < dim; ++d) {
            int64_t dd = cen[(size_t)a * 3 + d] - cen[(size_t)b * 3 + d];
            if (dd < 0) dd = -dd;
            if (2 * dd > k * (wid[a] + wid[b])) return false;
        }
        return true;
    };
    std::vector<std::vector<int>> L[4];
    for (int q = 0; q < 4; ++q) L[q].assign(nb, {});
    std::vector<int> stack, nbrs, pcol;
    int last_parent = -2;
    for (int b = 0; b < nb; ++b) {
        bool leaf = t.nchild[b] == 0;
        if (leaf) {
            // every box near b, by descent from the root (a box that is not near b
            // has no descendant near b)
            nbrs.clear();
            stack.assign(1, 0);
            while (!stack.empty()) {
                int a = stack.back();
                stack.pop_back();
                if (!near(a, b)) continue;
                nbrs.push_back(a);
                for (int c = 0; c < t.nchild[a]; ++c) stack.push_back(t.child0[a] + c);
            }
            for (int a : nbrs) {
                if (t.nchild[a] == 0) L[0][b].push_back(a);
                if (t.level[a] >= t.level[b])
                    for (int c = 0; c < t.nchild[a]; ++c)
                        if (!near(t.child0[a] + c, b)) L[2][b].push_back(t.child0[a] + c);
            }
            std::sort(L[0][b].begin(), L[0][b].end());
            std::sort(L[2][b].begin(), L[2][b].end());
        }
        int p = t.parent[b];
        if (p >= 0) {
            if (p != last_parent) {
                // same-level boxes near p (its colleagues), by descent
                pcol.clear();
                stack.assign(1, 0);
                while (!stack.empty()) {
                    int a = stack.back();
                    stack.pop_back();
                    if (!near(a, p)) continue;
                    if (t.level[a] == t.level[p]) { pcol.push_back(a); continue; }
                    for (int c = 0; c < t.nchild[a]; ++c) stack.push_back(t.child0[a] + c);
                }
                last_parent = p;
            }
            for (int a : pcol)
                for (int c = 0; c < t.nchild[a]; ++c)
                    if (!near(t.child0[a] + c, b)) L[1][b].push_back(t.child0[a] + c);
            std::sort(L[1][b].begin(), L[1][b].end());
        }
    }
    for (int b = 0; b < nb; ++b)
        for (int c : L[2][b]) L[3][c].push_back(b);
    for (int q = 0; q < 4; ++q) {
        t.off[q].assign(nb + 1, 0);
        for (int b = 0; b < nb; ++b) t.off[q][b + 1] = t.off[q][b] + (int)L[q][b].size();
        t.idx[q].resize(t.off[q][nb]);
        for (int b = 0; b < nb; ++b)
            std::copy(L[q][b].begin(), L[q][b].end(), t.idx[q].begin() + t.off[q][b]);
    }
}

}  // namespace cfmm
