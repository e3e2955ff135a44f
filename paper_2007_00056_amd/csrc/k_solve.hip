// Solve-phase kernels: CSR SpMV, the V-cycle level kernels of Algorithm 1
// (damped Jacobi, residual, piecewise-constant restriction and prolongation),
// the coarsest dense solve, and the vector kernels of Algorithm 4 (PCG) and
// Algorithm 5 (BiCGStab).
//
// Large levels use a block-level CSR-stream schedule: a 256-thread block owns
// 256 consecutive rows, reads their contiguous entry range with coalesced,
// independent loads (val, col and the gathered vector), stages the products
// in LDS, and then each thread adds its own row's products.  Small levels,
// where launch latency dominates, use lane groups per row and the fused
// coarse-row restriction.  Blocks are mapped XCD-contiguously so rows that
// share vector cache lines share one XCD's L2.
#include <cstdlib>

#include "amg_device.hpp"
#include "amg_internal.hpp"

namespace amg {

namespace {
constexpr int BS = 256;

inline int level_blocks(int64_t rows, int lpr) {
    int64_t b = (rows * lpr + BS - 1) / BS;
    return (int)(b < 1 ? 1 : b);
}

inline int vec_blocks(int64_t n) {
    int64_t b = (n + BS - 1) / BS;
    if (b < 1) b = 1;
    return (int)(b < kRedBlocks ? b : kRedBlocks);
}

template <int LPR>
__device__ __forceinline__ double row_ax(int row, int lane, const int* __restrict__ rp, const int* __restrict__ ci,
                                         const double* __restrict__ v, const double* __restrict__ x) {
    double s = 0.0;
    const int b = rp[row], e = rp[row + 1];
    for (int k = b + lane; k < e; k += LPR) s += v[k] * x[ci[k]];
    return s;
}
}  // namespace

int pick_lanes_per_row(double avg) {
    // HEMAMG_LPR=1|2|4|8|16 fixes the schedule (tuning sweeps)
    if (const char* e = getenv("HEMAMG_LPR")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16) return v;
    }
    if (avg <= 2.0) return 2;
    return 4;
}

#define AMG_DISPATCH_LPR(lpr, CALL) \
    switch (lpr) {                  \
        case 1: CALL(1); break;     \
        case 2: CALL(2); break;     \
        case 4: CALL(4); break;     \
        case 8: CALL(8); break;     \
        default: CALL(16); break;   \
    }

// ---------------------------------------------------------------------------
// CSR-stream building block.  Rows [r0, min(r0 + 256, n)); entries are
// processed in LDS chunks so rows of any length are handled.  The sum of a
// row's products runs in entry order.
// ---------------------------------------------------------------------------
constexpr int kStreamChunk = 2048;  // doubles of LDS (16 KB)

template <class Ent>
__device__ __forceinline__ double stream_rows(int r0, int n, const int* __restrict__ rp, const Ent& ent,
                                              double* prod) {
    const int r1 = min(r0 + BS, n);
    const int e0 = rp[r0], e1 = rp[r1];
    const int row = r0 + threadIdx.x;
    const int rb = row < r1 ? rp[row] : 0, re = row < r1 ? rp[row + 1] : 0;
    double acc = 0.0;
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

struct EntAx {  // a_ij x_j
    const double* __restrict__ v;
    const int* __restrict__ ci;
    const double* __restrict__ x;
    __device__ __forceinline__ double operator()(int e) const { return v[e] * x[ci[e]]; }
};

constexpr int FIN_BS = 1024;

__global__ __launch_bounds__(FIN_BS) void k_finish(int nparts, int nv, const double* __restrict__ part,
                                                   double* __restrict__ S, int slot0, int slot1) {
    __shared__ double sh[2][FIN_BS / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nparts; b += FIN_BS) s += part[k * nparts + b];
        s = group_sum<kWave>(s);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < nv; ++k) {
            double s = sh[k][0];
            for (int w = 1; w < FIN_BS / kWave; ++w) s += sh[k][w];
            S[k == 0 ? slot0 : slot1] = s;
        }
    }
}

// y = A x
__global__ __launch_bounds__(BS) void k_stream_spmv(int n, const int* __restrict__ rp, EntAx ent,
                                                    double* __restrict__ y) {
    __shared__ double prod[kStreamChunk];
    for (int b = xcd_block(blockIdx.x, gridDim.x); b * BS < n; b += gridDim.x) {
        const double s = stream_rows(b * BS, n, rp, ent, prod);
        const int row = b * BS + threadIdx.x;
        if (row < n) y[row] = s;
    }
}

// r = f - w A g, g = D^{-1} f : residual after the zero-guess presmoothing sweep
__global__ __launch_bounds__(BS) void k_stream_resid(int n, const int* __restrict__ rp, EntAx ent,
                                                     const double* __restrict__ f, double w,
                                                     double* __restrict__ r) {
    __shared__ double prod[kStreamChunk];
    for (int b = xcd_block(blockIdx.x, gridDim.x); b * BS < n; b += gridDim.x) {
        const double s = stream_rows(b * BS, n, rp, ent, prod);
        const int row = b * BS + threadIdx.x;
        if (row < n) r[row] = f[row] - w * s;
    }
}

// Postsmoothing on the prolongated iterate xp = w g + P e (written by the
// coarser level): z = xp + w D^{-1} (f - A xp) = xp + w (g - D^{-1} A xp).
// MODE 1 also forms block partials of (f, z); MODE 2 scatters z to the finer
// level's prolongated iterate.
template <int MODE>
__global__ __launch_bounds__(BS) void k_stream_post(int n, const int* __restrict__ rp, EntAx ent,
                                                    const double* __restrict__ g, const double* __restrict__ dinv,
                                                    double w, double* __restrict__ z, const double* __restrict__ f,
                                                    double* part, Scatter sc) {
    __shared__ double prod[kStreamChunk];
    double acc[1] = {0.0};
    for (int b = xcd_block(blockIdx.x, gridDim.x); b * BS < n; b += gridDim.x) {
        const double s = stream_rows(b * BS, n, rp, ent, prod);
        const int row = b * BS + threadIdx.x;
        if (row < n) {
            const double zi = ent.x[row] + w * (g[row] - dinv[row] * s);
            z[row] = zi;
            if (MODE == 1) acc[0] += f[row] * zi;
            if (MODE == 2) sc(row, zi);
        }
    }
    if (MODE == 1) block_partials<1, BS>(acc, part);
}

// f_c = P^T r (members added in ascending order) and g_c = D_c^{-1} f_c
__global__ __launch_bounds__(BS) void k_restrict(int nc, const int4* __restrict__ mem, const double* __restrict__ r,
                                                 const double* __restrict__ dinv_c, double* __restrict__ fc,
                                                 double* __restrict__ gc) {
    const int J = blockIdx.x * BS + threadIdx.x;
    if (J >= nc) return;
    const int4 m = mem[J];
    double s = r[m.x];
    if (m.y >= 0) s += r[m.y];
    if (m.z >= 0) s += r[m.z];
    if (m.w >= 0) s += r[m.w];
    fc[J] = s;
    gc[J] = dinv_c[J] * s;
}

inline int stream_blocks(int n) {
    const int b = (n + BS - 1) / BS;
    return b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks;
}

void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_stream_spmv, dim3(stream_blocks(L.n)), dim3(BS), 0, s, L.n, L.rp, EntAx{L.v, L.ci, x}, y);
}

void launch_stream_resid(const LevelView& L, const double* f, const double* g, double w, double* r,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_stream_resid, dim3(stream_blocks(L.n)), dim3(BS), 0, s, L.n, L.rp, EntAx{L.v, L.ci, g}, f, w,
                       r);
}

void launch_restrict(int nc, const int4* mem, const double* r, const double* dinv_c, double* fc, double* gc,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_restrict, dim3(level_blocks(nc, 1)), dim3(BS), 0, s, nc, mem, r, dinv_c, fc, gc);
}

void launch_stream_post(const LevelView& L, const double* xp, const double* g, double w, double* z, const double* f,
                        const Reducer* R, int slot, const Scatter* sc, hipStream_t s) {
    const int gsz = stream_blocks(L.n);
    const EntAx ent{L.v, L.ci, xp};
    const Scatter none{nullptr, nullptr, nullptr, 0.0};
    if (R) {
        hipLaunchKernelGGL(k_stream_post<1>, dim3(gsz), dim3(BS), 0, s, L.n, L.rp, ent, g, L.dinv, w, z, f, R->part,
                           none);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(FIN_BS), 0, s, gsz, 1, R->part, R->S, slot, slot);
    } else if (sc) {
        hipLaunchKernelGGL(k_stream_post<2>, dim3(gsz), dim3(BS), 0, s, L.n, L.rp, ent, g, L.dinv, w, z, f, nullptr,
                           *sc);
    } else {
        hipLaunchKernelGGL(k_stream_post<0>, dim3(gsz), dim3(BS), 0, s, L.n, L.rp, ent, g, L.dinv, w, z, f, nullptr,
                           none);
    }
}

// ---------------------------------------------------------------------------
// Small levels: down-sweep fused in one kernel.  A group of 4*LPR lanes owns
// one coarse row; sub-group q handles member q (members ascending) and the
// member residuals are added in that order.
// ---------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(BS) void k_resid_restrict(int nc, const int4* __restrict__ mem,
                                                       const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v, const double* __restrict__ g,
                                                       const double* __restrict__ f, double w,
                                                       const double* __restrict__ dinv_c, double* __restrict__ fc,
                                                       double* __restrict__ gc) {
    constexpr int G = 4 * LPR;
    const int t = blockIdx.x * BS + threadIdx.x;
    const int J = t / G, sub = (t % G) / LPR, lane = t % LPR;
    int i = -1;
    if (J < nc) {
        const int4 m = mem[J];
        i = sub == 0 ? m.x : sub == 1 ? m.y : sub == 2 ? m.z : m.w;
    }
    double s = 0.0;
    if (i >= 0) s = row_ax<LPR>(i, lane, rp, ci, v, g);
    s = group_sum<LPR>(s);
    const double ri = i >= 0 ? f[i] - w * s : 0.0;
    const int base = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const double r0 = __shfl(ri, base, kWave);
    const double r1 = __shfl(ri, base + LPR, kWave);
    const double r2 = __shfl(ri, base + 2 * LPR, kWave);
    const double r3 = __shfl(ri, base + 3 * LPR, kWave);
    if (J < nc && (t % G) == 0) {
        const double fj = ((r0 + r1) + r2) + r3;
        fc[J] = fj;
        gc[J] = dinv_c[J] * fj;
    }
}

void launch_resid_restrict(const LevelView& L, int nc, const double* f, const double* g, double w,
                           const double* dinv_c, double* fc, double* gc, hipStream_t s) {
#define CALL(W)                                                                                                 \
    hipLaunchKernelGGL(k_resid_restrict<W>, dim3(level_blocks((int64_t)nc * 4, W)), dim3(BS), 0, s, nc, L.mem, \
                       L.rp, L.ci, L.v, g, f, w, dinv_c, fc, gc)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

template <int LPR, bool SCAT>
__global__ __launch_bounds__(BS) void k_prolong_post(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ g, const double* __restrict__ xp,
                                                     double w, double* __restrict__ z, Scatter sc) {
    const int t = blockIdx.x * BS + threadIdx.x;
    const int row = t / LPR, lane = t % LPR;
    double s = row < n ? row_ax<LPR>(row, lane, rp, ci, v, xp) : 0.0;
    s = group_sum<LPR>(s);
    if (row < n && lane == 0) {
        const double zi = xp[row] + w * (g[row] - dinv[row] * s);
        z[row] = zi;
        if (SCAT) sc(row, zi);
    }
}

void launch_prolong_post(const LevelView& L, const double* xp, const double* g, double w, double* z,
                         const Scatter* sc, hipStream_t s) {
    const Scatter none{nullptr, nullptr, nullptr, 0.0};
#define CALL(W)                                                                                                     \
    if (sc)                                                                                                        \
        hipLaunchKernelGGL((k_prolong_post<W, true>), dim3(level_blocks(L.n, W)), dim3(BS), 0, s, L.n, L.rp, L.ci, \
                           L.v, L.dinv, g, xp, w, z, *sc);                                                         \
    else                                                                                                           \
        hipLaunchKernelGGL((k_prolong_post<W, false>), dim3(level_blocks(L.n, W)), dim3(BS), 0, s, L.n, L.rp,     \
                           L.ci, L.v, L.dinv, g, xp, w, z, none)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

// g = D^{-1} f
__global__ __launch_bounds__(BS) void k_scale_dinv(int n, const double* __restrict__ dinv,
                                                   const double* __restrict__ f, double* __restrict__ g) {
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) g[i] = dinv[i] * f[i];
}

void launch_scale_dinv(int n, const double* dinv, const double* f, double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_dinv, dim3(vec_blocks(n)), dim3(BS), 0, s, n, dinv, f, g);
}

// ---------------------------------------------------------------------------
// General smoothing path (any number of sweeps).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_jacobi_zero(int n, const double* __restrict__ dinv,
                                                    const double* __restrict__ f, double w, double* __restrict__ x) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) x[i] = w * (dinv[i] * f[i]);
}

void launch_jacobi_zero(int n, const double* dinv, const double* f, double w, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_zero, dim3(level_blocks(n, 1)), dim3(BS), 0, s, n, dinv, f, w, x);
}

template <int LPR>
__global__ __launch_bounds__(BS) void k_jacobi(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                               const double* __restrict__ v, const double* __restrict__ dinv,
                                               const double* __restrict__ f, const double* __restrict__ x, double w,
                                               double* __restrict__ xo) {
    const int t = xcd_block(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    const int row = t / LPR, lane = t % LPR;
    double s = row < n ? row_ax<LPR>(row, lane, rp, ci, v, x) : 0.0;
    s = group_sum<LPR>(s);
    if (row < n && lane == 0) xo[row] = x[row] + w * (dinv[row] * (f[row] - s));
}

void launch_jacobi(const LevelView& L, const double* f, const double* x, double w, double* xo, hipStream_t s) {
#define CALL(W)                                                                                                  \
    hipLaunchKernelGGL(k_jacobi<W>, dim3(level_blocks(L.n, W)), dim3(BS), 0, s, L.n, L.rp, L.ci, L.v, L.dinv, f, \
                       x, w, xo)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

// f_c = P^T (f - A x) for a stored x (x == nullptr means x = 0).
template <int LPR>
__global__ __launch_bounds__(BS) void k_resid_restrict_x(int nc, const int4* __restrict__ mem,
                                                         const int* __restrict__ rp, const int* __restrict__ ci,
                                                         const double* __restrict__ v, const double* __restrict__ f,
                                                         const double* __restrict__ x, double* __restrict__ fc) {
    constexpr int G = 4 * LPR;
    const int t = blockIdx.x * BS + threadIdx.x;
    const int J = t / G, sub = (t % G) / LPR, lane = t % LPR;
    int i = -1;
    if (J < nc) {
        const int4 m = mem[J];
        i = sub == 0 ? m.x : sub == 1 ? m.y : sub == 2 ? m.z : m.w;
    }
    double s = 0.0;
    if (i >= 0 && x != nullptr) s = row_ax<LPR>(i, lane, rp, ci, v, x);
    s = group_sum<LPR>(s);
    const double ri = i >= 0 ? f[i] - s : 0.0;
    const int base = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const double r0 = __shfl(ri, base, kWave);
    const double r1 = __shfl(ri, base + LPR, kWave);
    const double r2 = __shfl(ri, base + 2 * LPR, kWave);
    const double r3 = __shfl(ri, base + 3 * LPR, kWave);
    if (J < nc && (t % G) == 0) fc[J] = ((r0 + r1) + r2) + r3;
}

void launch_resid_restrict_x(const LevelView& L, int nc, const double* f, const double* x, double* fc,
                             hipStream_t s) {
#define CALL(W)                                                                                                   \
    hipLaunchKernelGGL(k_resid_restrict_x<W>, dim3(level_blocks((int64_t)nc * 4, W)), dim3(BS), 0, s, nc, L.mem, \
                       L.rp, L.ci, L.v, f, x, fc)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

__global__ __launch_bounds__(BS) void k_prolong_add(int n, const int* __restrict__ agg, const double* __restrict__ e,
                                                    double* __restrict__ x) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) x[i] += e[agg[i]];
}

void launch_prolong_add(int n, const int* agg, const double* e, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_prolong_add, dim3(level_blocks(n, 1)), dim3(BS), 0, s, n, agg, e, x);
}

// Coarsest level: x = A_L^{-1} f with the inverse stored column-major.  One
// block stages f in LDS; each thread forms one row with independent loads.
// With a scatter, x also becomes the finer level's prolongated iterate.
__global__ __launch_bounds__(BS) void k_dense_apply(int n, const double* __restrict__ ainv_t,
                                                   const double* __restrict__ f, double* __restrict__ x, Scatter sc) {
    __shared__ double fs[1024];
    for (int j = threadIdx.x; j < n; j += BS) fs[j] = f[j];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += BS) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int j = 0;
        for (; j + 4 <= n; j += 4) {
            s0 += ainv_t[(size_t)j * n + i] * fs[j];
            s1 += ainv_t[(size_t)(j + 1) * n + i] * fs[j + 1];
            s2 += ainv_t[(size_t)(j + 2) * n + i] * fs[j + 2];
            s3 += ainv_t[(size_t)(j + 3) * n + i] * fs[j + 3];
        }
        for (; j < n; ++j) s0 += ainv_t[(size_t)j * n + i] * fs[j];
        const double xi = (s0 + s1) + (s2 + s3);
        x[i] = xi;
        if (sc.mem) sc(i, xi);
    }
}

void launch_dense_apply(int n, const double* ainv_t, const double* f, double* x, const Scatter* sc, hipStream_t s) {
    const Scatter none{nullptr, nullptr, nullptr, 0.0};
    hipLaunchKernelGGL(k_dense_apply, dim3(1), dim3(BS), 0, s, n, ainv_t, f, x, sc ? *sc : none);
}

// ---------------------------------------------------------------------------
// Krylov kernels.  A reduction kernel writes one partial per block; k_finish
// (one block) adds them in a fixed order into the scalar slots, so results are
// reproducible run to run.  The scalars of the recurrences stay in device
// slots, so no host round trip sits between the kernels of one iteration.
// Update kernels skip the update when a denominator they depend on is zero or
// not finite; the host reports the breakdown after reading the slots.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool usable(double d) { return isfinite(d) && d != 0.0; }

inline void finish(int nparts, int nv, const Reducer& R, int slot0, int slot1, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(FIN_BS), 0, s, nparts, nv, R.part, R.S, slot0, slot1);
}

// r = b - A x, partial (r, r)
__global__ __launch_bounds__(BS) void k_stream_residual(int n, const int* __restrict__ rp, EntAx ent,
                                                        const double* __restrict__ b, double* __restrict__ r,
                                                        const double* __restrict__ dinv, double* __restrict__ g,
                                                        double* part) {
    __shared__ double prod[kStreamChunk];
    double acc[1] = {0.0};
    for (int blk = xcd_block(blockIdx.x, gridDim.x); blk * BS < n; blk += gridDim.x) {
        const double s = stream_rows(blk * BS, n, rp, ent, prod);
        const int row = blk * BS + threadIdx.x;
        if (row < n) {
            const double ri = b[row] - s;
            r[row] = ri;
            if (g) g[row] = dinv[row] * ri;
            acc[0] += ri * ri;
        }
    }
    block_partials<1, BS>(acc, part);
}

void launch_residual(const LevelView& A, const double* b, const double* x, double* r, double* gout, const Reducer& R,
                     int slot, hipStream_t s) {
    const int g = stream_blocks(A.n);
    hipLaunchKernelGGL(k_stream_residual, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAx{A.v, A.ci, x}, b, r, A.dinv, gout,
                       R.part);
    finish(g, 1, R, slot, slot, s);
}

// q = A p, partial (d, q)
__global__ __launch_bounds__(BS) void k_stream_spmv_dot(int n, const int* __restrict__ rp, EntAx ent,
                                                        double* __restrict__ q, const double* __restrict__ d,
                                                        double* part) {
    __shared__ double prod[kStreamChunk];
    double acc[1] = {0.0};
    for (int blk = xcd_block(blockIdx.x, gridDim.x); blk * BS < n; blk += gridDim.x) {
        const double s = stream_rows(blk * BS, n, rp, ent, prod);
        const int row = blk * BS + threadIdx.x;
        if (row < n) {
            q[row] = s;
            acc[0] += d[row] * s;
        }
    }
    block_partials<1, BS>(acc, part);
}

void launch_spmv_dot(const LevelView& A, const double* p, double* q, const double* d, const Reducer& R, int slot,
                     hipStream_t s) {
    const int g = stream_blocks(A.n);
    hipLaunchKernelGGL(k_stream_spmv_dot, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAx{A.v, A.ci, p}, q, d, R.part);
    finish(g, 1, R, slot, slot, s);
}

// t = A p, partials (t, t) and (t, sv)
__global__ __launch_bounds__(BS) void k_stream_spmv_dot2(int n, const int* __restrict__ rp, EntAx ent,
                                                         double* __restrict__ t, const double* __restrict__ sv,
                                                         double* part) {
    __shared__ double prod[kStreamChunk];
    double acc[2] = {0.0, 0.0};
    for (int blk = xcd_block(blockIdx.x, gridDim.x); blk * BS < n; blk += gridDim.x) {
        const double s = stream_rows(blk * BS, n, rp, ent, prod);
        const int row = blk * BS + threadIdx.x;
        if (row < n) {
            t[row] = s;
            acc[0] += s * s;
            acc[1] += s * sv[row];
        }
    }
    block_partials<2, BS>(acc, part);
}

void launch_spmv_dot2(const LevelView& A, const double* p, double* t, const double* sv, const Reducer& R, int slot_tt,
                      int slot_ts, hipStream_t s) {
    const int g = stream_blocks(A.n);
    hipLaunchKernelGGL(k_stream_spmv_dot2, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAx{A.v, A.ci, p}, t, sv, R.part);
    finish(g, 2, R, slot_tt, slot_ts, s);
}

__global__ __launch_bounds__(BS) void k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                            double* part) {
    double acc[1] = {0.0};
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) acc[0] += a[i] * b[i];
    block_partials<1, BS>(acc, part);
}

void launch_dot(int n, const double* a, const double* b, const Reducer& R, int slot, hipStream_t s) {
    const int g = vec_blocks(n);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(BS), 0, s, n, a, b, R.part);
    finish(g, 1, R, slot, slot, s);
}

// Algorithm 4: alpha = (r,z)/(Ap,p); x += alpha p; r -= alpha Ap; partial (r,r).
__global__ __launch_bounds__(BS) void k_cg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ dinv, double* __restrict__ g,
                                                  double* part, const double* __restrict__ S, int slot_rho,
                                                  int slot_pq) {
    const double rho = S[slot_rho], pq = S[slot_pq];
    const bool ok = usable(pq) && isfinite(rho);
    const double alpha = ok ? rho / pq : 0.0;
    double acc[1] = {0.0};
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
        double ri = r[i];
        if (ok) {
            x[i] += alpha * p[i];
            ri -= alpha * q[i];
            r[i] = ri;
        }
        if (g) g[i] = dinv[i] * ri;
        acc[0] += ri * ri;
    }
    block_partials<1, BS>(acc, part);
}

void launch_cg_update(int n, double* x, double* r, const double* p, const double* q, const double* dinv, double* gout,
                      const Reducer& R, int slot_rho, int slot_pq, int slot_rr, hipStream_t s) {
    const int g = vec_blocks(n);
    hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(BS), 0, s, n, x, r, p, q, dinv, gout, R.part, R.S, slot_rho,
                       slot_pq);
    finish(g, 1, R, slot_rr, slot_rr, s);
}

// p_new = z + beta p, beta = rho_new / rho
__global__ __launch_bounds__(BS) void k_cg_dir(int n, const double* __restrict__ z, const double* __restrict__ p,
                                               double* __restrict__ pn, const double* __restrict__ S, int slot_new,
                                               int slot_old) {
    const double beta = S[slot_new] / S[slot_old];
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) pn[i] = z[i] + beta * p[i];
}

void launch_cg_dir(int n, const double* z, const double* p, double* pn, const double* S, int slot_new, int slot_old,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir, dim3(vec_blocks(n)), dim3(BS), 0, s, n, z, p, pn, S, slot_new, slot_old);
}

// Algorithm 5: s = r - alpha v, alpha = rho / (rbar, v)
__global__ __launch_bounds__(BS) void k_bicg_s(int n, const double* __restrict__ r, const double* __restrict__ v,
                                               double* __restrict__ sv, const double* __restrict__ S, int slot_rho,
                                               int slot_rv) {
    const double alpha = S[slot_rho] / S[slot_rv];
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) sv[i] = r[i] - alpha * v[i];
}

void launch_bicg_s(int n, const double* r, const double* v, double* sv, const double* S, int slot_rho, int slot_rv,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_s, dim3(vec_blocks(n)), dim3(BS), 0, s, n, r, v, sv, S, slot_rho, slot_rv);
}

// x += alpha pt + omega st; r = s - omega t; partials (r,r) and (r, rbar)
__global__ __launch_bounds__(BS) void k_bicg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ pt, const double* __restrict__ st,
                                                    const double* __restrict__ sv, const double* __restrict__ t,
                                                    const double* __restrict__ rb, double* part,
                                                    const double* __restrict__ S, int slot_rho, int slot_rv,
                                                    int slot_tt, int slot_ts) {
    const double rho = S[slot_rho], rv = S[slot_rv], tt = S[slot_tt], ts = S[slot_ts];
    const bool ok = usable(rho) && usable(rv) && usable(tt) && isfinite(ts);
    const double alpha = ok ? rho / rv : 0.0, omega = ok ? ts / tt : 0.0;
    double acc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
        double ri = r[i];
        if (ok) {
            x[i] = x[i] + alpha * pt[i] + omega * st[i];
            ri = sv[i] - omega * t[i];
            r[i] = ri;
        }
        acc[0] += ri * ri;
        acc[1] += ri * rb[i];
    }
    block_partials<2, BS>(acc, part);
}

void launch_bicg_update(int n, double* x, double* r, const double* pt, const double* st, const double* sv,
                        const double* t, const double* rb, const Reducer& R, int slot_rho, int slot_rv, int slot_tt,
                        int slot_ts, int slot_rr, int slot_rhonew, hipStream_t s) {
    const int g = vec_blocks(n);
    hipLaunchKernelGGL(k_bicg_update, dim3(g), dim3(BS), 0, s, n, x, r, pt, st, sv, t, rb, R.part, R.S, slot_rho,
                       slot_rv, slot_tt, slot_ts);
    finish(g, 2, R, slot_rr, slot_rhonew, s);
}

// p_new = r + beta (p - omega v), beta = (rho_new / rho) (alpha / omega)
__global__ __launch_bounds__(BS) void k_bicg_dir(int n, const double* __restrict__ r, const double* __restrict__ p,
                                                 const double* __restrict__ v, double* __restrict__ pn,
                                                 const double* __restrict__ S, int slot_rho, int slot_rv, int slot_tt,
                                                 int slot_ts, int slot_rhonew) {
    const double alpha = S[slot_rho] / S[slot_rv], omega = S[slot_ts] / S[slot_tt];
    const double beta = (S[slot_rhonew] / S[slot_rho]) * (alpha / omega);
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) pn[i] = r[i] + beta * (p[i] - omega * v[i]);
}

void launch_bicg_dir(int n, const double* r, const double* p, const double* v, double* pn, const double* S,
                     int slot_rho, int slot_rv, int slot_tt, int slot_ts, int slot_rhonew, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_dir, dim3(vec_blocks(n)), dim3(BS), 0, s, n, r, p, v, pn, S, slot_rho, slot_rv,
                       slot_tt, slot_ts, slot_rhonew);
}

__global__ __launch_bounds__(BS) void k_zero(int n, double* __restrict__ x) {
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) x[i] = 0.0;
}

void launch_scale_zero(int n, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(vec_blocks(n)), dim3(BS), 0, s, n, x);
}

__global__ __launch_bounds__(BS) void k_check_finite(int n, const double* __restrict__ a,
                                                     const double* __restrict__ b, int* err) {
    bool bad = false;
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) bad |= !isfinite(a[i]) || !isfinite(b[i]);
    if (bad) atomicOr(err, ERR_NONFINITE);
}

void launch_check_finite(int n, const double* a, const double* b, int* err, hipStream_t s) {
    const int g = vec_blocks(n) < 2048 ? vec_blocks(n) : 2048;
    hipLaunchKernelGGL(k_check_finite, dim3(g), dim3(BS), 0, s, n, a, b, err);
}

}  // namespace amg
