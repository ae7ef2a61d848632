// Host-side tree topology and interaction lists (Sec. 6.1, Sec. 6.2), built
// from the Morton-sorted keys the device produced.
#pragma once
#include <stdint.h>
#include <vector>

namespace cfmm {

struct HostTree {
    int dim = 0, nbits = 0, sep = 1, top = 0;
    int64_t n = 0;
    std::vector<int32_t> level, parent, child0, nchild, pbeg, pend;
    std::vector<uint64_t> prefix;
    std::vector<int32_t> lvl_beg;         // boxes of level l: [lvl_beg[l], lvl_beg[l+1])
    std::vector<int32_t> off[4], idx[4];  // Lists 1..4 as CSR
    int nbox() const { return (int)level.size(); }
    int nlevels() const { return (int)lvl_beg.size() - 1; }
};

// Adaptive split by occupancy (> leaf_size points) and the level restriction
// (leaves two or more levels apart are never near).  keys are sorted.
void build_topology(const uint64_t* keys, int64_t n, int dim, int leaf_size, int sep,
                    HostTree& t);

// Lists 1-4 for far-field work starting at level `top` (boxes coarser than
// top carry no expansions: any pair involving one counts as near).
void build_lists(HostTree& t, int top);

// integer box coordinates at the box's level
void box_coords(const HostTree& t, int b, int64_t* c);

}  // namespace cfmm
