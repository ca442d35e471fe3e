// Transposition of the group-major interaction lists (entries (cluster, lane mask) per
// 64-target group) into cluster-major order, and work items over cluster-major ranges.
#pragma once

#include "stk_internal.hpp"

namespace stk {
namespace {

__global__ void k_entry_group(const int32_t *__restrict__ off, int32_t ng, int32_t *__restrict__ eg) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    for (int32_t e = off[g]; e < off[g + 1]; ++e) eg[e] = g;
}

__global__ void k_node_keys(const int32_t *__restrict__ node, int64_t ne, uint64_t *__restrict__ keys,
                            int32_t *__restrict__ vals) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    keys[e] = uint64_t(node[e]);
    vals[e] = int32_t(e);
}

// node_off[c] = first position of node c in the sorted keys (lower bound), c in [0, nn]
__global__ void k_node_off(const uint64_t *__restrict__ keys, int64_t ne, int32_t nn, int32_t *__restrict__ off) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nn) return;
    int64_t lo = 0, hi = ne;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < uint64_t(c))
            lo = mid + 1;
        else
            hi = mid;
    }
    off[c] = int32_t(lo);
}

// work items: per node, ceil(count / per) items of up to `per` consecutive units
__global__ void k_item_count(const int32_t *__restrict__ off, int32_t nn, int32_t per, int32_t *__restrict__ cnt) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nn) return;
    cnt[c] = (off[c + 1] - off[c] + per - 1) / per;
}

// one thread per item: its node is the last c with ioff[c] <= item (nodes without items
// have ioff[c] == ioff[c + 1]); a node's items cover its range in runs of `per`
__global__ void k_item_fill(const int32_t *__restrict__ off, const int32_t *__restrict__ ioff, int32_t nn, int32_t per,
                            int32_t nitems, int32_t *__restrict__ inode, int32_t *__restrict__ i0,
                            int32_t *__restrict__ i1) {
    const int32_t it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= nitems) return;
    int32_t lo = 0, hi = nn;  // ioff[lo] <= it < ioff[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (ioff[mid] <= it)
            lo = mid;
        else
            hi = mid;
    }
    const int32_t b = off[lo] + (it - ioff[lo]) * per;
    inode[it] = lo;
    i0[it] = b;
    i1[it] = min(b + per, off[lo + 1]);
}

}  // namespace
}  // namespace stk
