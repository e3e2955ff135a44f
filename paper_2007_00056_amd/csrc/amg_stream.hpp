// CSR-stream building block shared by the level and Krylov kernels.
//
// A block of RB threads (256 by default) owns RB consecutive rows.  It reads their contiguous
// entry range with coalesced, independent loads (values, columns and the
// gathered vector), stages the products in LDS, and then each thread adds
// its own row's products in entry order.  Entries are processed in LDS chunks,
// so rows of any length are handled.
#pragma once

#include "amg_device.hpp"

namespace amg {

constexpr int kStreamBS = 256;
constexpr int kStreamChunk = 2048;  // products per LDS chunk

template <class T>
struct EntAx {  // a_ij x_j
    const T* __restrict__ v;
    const int* __restrict__ ci;
    const T* __restrict__ x;
    __device__ __forceinline__ T operator()(int e) const { return v[e] * x[ci[e]]; }
};

// RB rows per block (the block has RB threads); a row's sum does not depend
// on RB.
template <class T, int RB = kStreamBS, class Ent>
__device__ __forceinline__ T stream_rows(int r0, int n, const int* __restrict__ rp, const Ent& ent, T* prod) {
    constexpr int BS = RB;
    const int r1 = min(r0 + BS, n);
    const int e0 = rp[r0], e1 = rp[r1];
    const int row = r0 + threadIdx.x;
    const int rb = row < r1 ? rp[row] : 0, re = row < r1 ? rp[row + 1] : 0;
    T acc = T(0);
    for (int c0 = e0; c0 < e1; c0 += kStreamChunk) {
        const int c1 = min(c0 + kStreamChunk, e1);
#pragma unroll 4
        for (int e = c0 + threadIdx.x; e < c1; e += BS) prod[e - c0] = ent(e);
        __syncthreads();
        const int lo = max(rb, c0), hi = min(re, c1);
        for (int e = lo; e < hi; ++e) acc += prod[e - c0];
        __syncthreads();
    }
    return acc;
}

inline int stream_blocks(int n, int cap) {
    const int b = (n + kStreamBS - 1) / kStreamBS;
    return b < cap ? (b < 1 ? 1 : b) : cap;
}

}  // namespace amg
