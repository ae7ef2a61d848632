// Tree topology (Sec. 6.1) and Lists 1-4 (Sec. 6.2) built on the device from
// the Morton-sorted keys, with the readings of the host builder (tree_host.hpp):
// the same boxes in the same (level, prefix) numbering and the same lists, each
// sorted by box index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace cfmm {

class DeviceTree {
public:
    // Occupancy split and level restriction, then the final numbering.  keys
    // are the sorted Morton keys (B bits per coordinate).  Owns its device
    // scratch until release().
    hipError_t build(const uint64_t* keys, int64_t n, int dim, int B, int leaf_size, int sep, hipStream_t st);
    int nbox() const { return nbox_; }

    // The topology in the final numbering: device arrays of nbox() entries
    // (any pointer may be null) and host copies of everything.
    hipError_t export_topology(int* level, int* parent, int* child0, int* nchild, int* pbeg, int* pend,
                               std::vector<int32_t>& h_level, std::vector<int32_t>& h_parent,
                               std::vector<int32_t>& h_child0, std::vector<int32_t>& h_nchild,
                               std::vector<int32_t>& h_pbeg, std::vector<int32_t>& h_pend,
                               std::vector<uint64_t>& h_prefix);

    // Lists 1-4 for far-field work from level `top`: count() gives the entries
    // of each list, fill() writes the CSR (off[nbox + 1], idx[count]) to the
    // device arrays and the host copies.  lvl_beg is the host's level table.
    hipError_t count_lists(int top, const std::vector<int32_t>& lvl_beg, int64_t cnt[4]);
    hipError_t fill_lists(int* const off[4], int* const idx[4], std::vector<int32_t> h_off[4],
                          std::vector<int32_t> h_idx[4]);

    void release();
    ~DeviceTree() { release(); }

private:
    template <class T>
    hipError_t grab(T** p, size_t count);
    hipError_t grow_boxes(int need);
    hipError_t split_pass(int mode, int level_for_mode0, int* added);
    hipError_t sort_pairs(uint64_t* keys, int64_t m, int key_bits);

    hipStream_t st_ = nullptr;
    int64_t n_ = 0;
    int dim_ = 0, B_ = 0, ns_ = 0, sep_ = 1, top_ = 0;
    int nbox_ = 0, cap_ = 0;
    const uint64_t* keys_ = nullptr;
    std::vector<void*> mem_;
    // creation-order boxes (capacity cap_)
    int *lev_ = nullptr, *pb_ = nullptr, *pe_ = nullptr, *par_ = nullptr, *first_ = nullptr, *nch_ = nullptr;
    uint64_t* pre_ = nullptr;
    unsigned char* mark_ = nullptr;
    // per point
    int* pbox_ = nullptr;
    unsigned *flag_ = nullptr, *pos_ = nullptr, *scan_tmp_ = nullptr;
    // hash of (level, prefix) -> box
    uint64_t* hk_ = nullptr;
    int* hv_ = nullptr;
    unsigned hmask_ = 0;
    // final numbering
    int *f_level_ = nullptr, *f_parent_ = nullptr, *f_child0_ = nullptr, *f_nchild_ = nullptr;
    int *f_pbeg_ = nullptr, *f_pend_ = nullptr;
    uint64_t* f_prefix_ = nullptr;
    int* counter_ = nullptr;
    // lists
    int* lvl_beg_d_ = nullptr;
    int* leaves_ = nullptr;
    int nleaf_ = 0;
    int* coarse_ = nullptr;
    int ncoarse_ = 0;
    unsigned* lcnt_[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t lsize_[4] = {0, 0, 0, 0};
};

}  // namespace cfmm
