// Device-side helpers shared by the gfx950 kernels: wavefront reductions,
// XCD-aware block mapping, coherent loads and a register-resident sorted
// accumulator.  Wavefronts are 64 lanes wide on CDNA4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amg {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Remapping gives each XCD one contiguous range of logical blocks, so
// rows that share x-vector cache lines share one XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int g) {
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    const int per = g / kNumXcd, rem = g % kNumXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Butterfly sum over groups of W consecutive lanes (W a power of two <= 64);
// every lane of the group ends with the group total, in a fixed order.
template <int W>
__device__ __forceinline__ double group_sum(double s) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, W);
    return s;
}

template <int W>
__device__ __forceinline__ float group_sum(float s) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, W);
    return s;
}

// Deterministic block reduction of NV sums: block b writes its totals to
// part[k * gridDim.x + b].  A separate single-block kernel adds the partials
// in a fixed order (same-address device-scope atomics serialise across the
// XCDs, so no "last block" ticket is used).
template <int NV, int BS>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* part) {
    static_assert(BS % kWave == 0, "block size must be whole waves");
    constexpr int NW = BS / kWave;
    __shared__ double sh[NV][NW];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = group_sum<kWave>(v[k]);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = sh[k][0];
            for (int w = 1; w < NW; ++w) s += sh[k][w];
            part[k * gridDim.x + blockIdx.x] = s;
        }
    }
}

// Sum of np block partials in a fixed order, formed by a whole block of BS
// threads and returned to every thread: lane sums over a stride of BS, the
// wave butterfly, then the waves in order.  Every block that calls it gets
// the same value, so a consumer kernel can finish a reduction itself.
template <int BS>
__device__ __forceinline__ double block_sum_partials(const double* __restrict__ part, int np) {
    static_assert(BS % kWave == 0, "block size must be whole waves");
    constexpr int NW = BS / kWave;
    __shared__ double sh[NW];
    __shared__ double tot;
    double s = 0.0;
    for (int b = threadIdx.x; b < np; b += BS) s += part[b];
    s = group_sum<kWave>(s);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < NW; ++w) t += sh[w];
        tot = t;
    }
    __syncthreads();
    return tot;
}

// Sorted list of up to CAP (key, sum) pairs kept in registers (all indexing
// resolves at compile time after unrolling).  The first value added for a key
// initialises its sum; later values are added in call order.
template <int CAP>
struct SortedAcc {
    int key[CAP];
    double val[CAP];
    int len;

    __device__ __forceinline__ void clear() { len = 0; }

    // Returns false (and leaves the list unchanged) when a new key does not fit.
    template <bool WITH_VAL>
    __device__ __forceinline__ bool add(int k, double x) {
        int pos = 0;
        bool found = false;
#pragma unroll
        for (int t = 0; t < CAP; ++t) {
            if (t < len) {
                if (key[t] < k) pos = t + 1;
                if (key[t] == k) {
                    found = true;
                    if (WITH_VAL) val[t] += x;
                }
            }
        }
        if (found) return true;
        if (len == CAP) return false;
#pragma unroll
        for (int t = CAP - 1; t > 0; --t) {
            if (t > pos && t <= len) {
                key[t] = key[t - 1];
                if (WITH_VAL) val[t] = val[t - 1];
            }
        }
#pragma unroll
        for (int t = 0; t < CAP; ++t) {
            if (t == pos) {
                key[t] = k;
                if (WITH_VAL) val[t] = x;
            }
        }
        ++len;
        return true;
    }
};

}  // namespace amg
