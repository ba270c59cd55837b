// Storage layout of the per-sub-circuit inverses, shared by the setup kernels
// (writers) and the sweep kernels (readers).
//
// An n x n inverse Kinv is stored in "column groups" of G = 16 / sizeof(T)
// columns: for every group g the n rows follow one another, each row holding
// its G consecutive entries, so one 16-byte load gives lane r the entries
// (r, gG .. gG+G-1) and a wavefront's loads are contiguous.  Columns beyond the
// last full group are stored column-major after the groups.  Each sub-circuit's
// block starts at a multiple of 4 elements (16-byte aligned for FP32 and FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vtm {

template <typename T>
struct Group {
    static constexpr int G = 16 / int(sizeof(T));
};

// element offset of Kinv(r, c) inside a sub-circuit's block
template <typename T>
__host__ __device__ inline int64_t inv_offset(int n, int r, int c) {
    constexpr int G = Group<T>::G;
    const int full = (n / G) * G;
    if (c < full) return (int64_t(c / G) * n + r) * G + (c % G);
    return int64_t(full) * n + int64_t(c - full) * n + r;
}

// (r, c) of the d-th stored element of an n x n block (inverse of inv_offset)
template <typename T>
__host__ __device__ inline void inv_rc(int n, int64_t d, int& r, int& c) {
    constexpr int G = Group<T>::G;
    const int full = (n / G) * G;
    const int64_t head = int64_t(full) * n;
    if (d < head) {
        const int64_t g = d / (int64_t(n) * G), rem = d - g * int64_t(n) * G;
        r = int(rem / G);
        c = int(g) * G + int(rem % G);
    } else {
        const int64_t e = d - head;
        c = full + int(e / n);
        r = int(e % n);
    }
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2): block
// b of a grid of n runs on XCD b % 8.  xcd_block renumbers them so that each XCD
// takes one contiguous range of logical blocks, and sub-circuits that exchange
// waves (neighbours in the block order) share an L2.  A bijection on [0, n).
__device__ inline int xcd_block(int b, int n) {
    const int x = b & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// The same ranges, each walked backwards: every XCD keeps its logical blocks
// (and what its L2 holds of them), in the opposite order.
__device__ inline int xcd_block_reversed(int b, int n) {
    const int x = b & 7, q = n >> 3, r = n & 7;
    const int count = q + (x < r ? 1 : 0);  // blocks of XCD x
    return x * q + (x < r ? x : r) + (count - 1 - (b >> 3));
}

// Items of m consecutive logical blocks each (a sub-circuit's column blocks),
// dealt to the XCDs in turn: item i runs on XCD i % 8, its m blocks one after
// another there, so that items of uneven cost spread over the chip while an
// item's blocks share an L2.  The grid holds 8 m ceil(n_items / 8) blocks; a
// block past the last item of its XCD gets -1.  reversed walks each XCD's items
// backwards.
__device__ inline int xcd_item_block(int b, int n_items, int m, bool reversed) {
    const int x = b & 7, j = b >> 3;
    const int k = j / m, r = j - k * m;      // block r of the k-th item of XCD x
    const int count = (n_items - x + 7) >> 3;  // items x, x + 8, ... below n_items
    if (k >= count) return -1;
    return ((reversed ? count - 1 - k : k) * 8 + x) * m + r;
}

// elements reserved for an n x n block (rounded up to a multiple of 4)
__host__ __device__ inline int64_t inv_block_elems(int n) { return (int64_t(n) * n + 3) & ~int64_t(3); }

}  // namespace vtm
