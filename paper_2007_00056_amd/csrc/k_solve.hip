// Solve-phase kernels: the outer CSR SpMV and the vector kernels of
// Algorithm 4 (PCG) and Algorithm 5 (BiCGStab), the general-sweep smoothing
// path of Algorithm 1, and the fixed-order reduction finish.  The default
// V-cycle kernels (one pre- and one post-sweep) are in k_vcycle.hip.
#include <cstdlib>

#include "amg_internal.hpp"
#include "amg_stream.hpp"

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
    return avg <= 10.0 ? 4 : 8;  // coarse levels of variable coefficients carry 15-30 entries per row
}

#define AMG_DISPATCH_LPR(lpr, CALL) \
    switch (lpr) {                  \
        case 1: CALL(1); break;     \
        case 2: CALL(2); break;     \
        case 4: CALL(4); break;     \
        case 8: CALL(8); break;     \
        default: CALL(16); break;   \
    }

using EntAxD = EntAx<double>;

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
__global__ __launch_bounds__(BS) void k_stream_spmv(int n, const int* __restrict__ rp, EntAxD ent,
                                                    double* __restrict__ y) {
    __shared__ double prod[kStreamChunk];
    for (int b = xcd_block(blockIdx.x, gridDim.x); b * BS < n; b += gridDim.x) {
        const double s = stream_rows<double>(b * BS, n, rp, ent, prod);
        const int row = b * BS + threadIdx.x;
        if (row < n) y[row] = s;
    }
}

inline int stream_blocks(int n) { return amg::stream_blocks(n, kRedBlocks); }

void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_stream_spmv, dim3(stream_blocks(L.n)), dim3(BS), 0, s, L.n, L.rp, EntAxD{L.v, L.ci, x}, y);
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

// ---------------------------------------------------------------------------
// Krylov kernels.  A reduction kernel writes one partial per block; k_finish
// (one block) adds them in a fixed order into the scalar slots, so results are
// reproducible run to run.  The scalars of the recurrences stay in device
// slots, so no host round trip sits between the kernels of one iteration.
// Update kernels skip the update when a denominator they depend on is zero or
// not finite; the host reports the breakdown after reading the slots.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool usable(double d) { return isfinite(d) && d != 0.0; }

void launch_finish(int nparts, int nv, const Reducer& R, int slot0, int slot1, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(FIN_BS), 0, s, nparts, nv, R.part, R.S, slot0, slot1);
}

inline void finish(int nparts, int nv, const Reducer& R, int slot0, int slot1, hipStream_t s) {
    launch_finish(nparts, nv, R, slot0, slot1, s);
}

// r = b - A x, partial (r, r)
template <class TG>
__global__ __launch_bounds__(BS) void k_stream_residual(int n, const int* __restrict__ rp, EntAxD ent,
                                                        const double* __restrict__ b, double* __restrict__ r,
                                                        const double* __restrict__ dinv, TG* __restrict__ g,
                                                        double* part) {
    __shared__ double prod[kStreamChunk];
    double acc[1] = {0.0};
    for (int blk = xcd_block(blockIdx.x, gridDim.x); blk * BS < n; blk += gridDim.x) {
        const double s = stream_rows<double>(blk * BS, n, rp, ent, prod);
        const int row = blk * BS + threadIdx.x;
        if (row < n) {
            const double ri = b[row] - s;
            r[row] = ri;
            if (g) g[row] = TG(dinv[row] * ri);
            acc[0] += ri * ri;
        }
    }
    block_partials<1, BS>(acc, part);
}

void launch_residual(const LevelView& A, const double* b, const double* x, double* r, void* gout, bool g32,
                     const Reducer& R, int slot, hipStream_t s) {
    const int g = stream_blocks(A.n);
    if (g32)
        hipLaunchKernelGGL(k_stream_residual<float>, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAxD{A.v, A.ci, x}, b, r,
                           A.dinv, static_cast<float*>(gout), R.part);
    else
        hipLaunchKernelGGL(k_stream_residual<double>, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAxD{A.v, A.ci, x}, b, r,
                           A.dinv, static_cast<double*>(gout), R.part);
    finish(g, 1, R, slot, slot, s);
}

// q = A p, partial (d, q)
__global__ __launch_bounds__(BS) void k_stream_spmv_dot(int n, const int* __restrict__ rp, EntAxD ent,
                                                        double* __restrict__ q, const double* __restrict__ d,
                                                        double* part) {
    __shared__ double prod[kStreamChunk];
    double acc[1] = {0.0};
    for (int blk = xcd_block(blockIdx.x, gridDim.x); blk * BS < n; blk += gridDim.x) {
        const double s = stream_rows<double>(blk * BS, n, rp, ent, prod);
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
    hipLaunchKernelGGL(k_stream_spmv_dot, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAxD{A.v, A.ci, p}, q, d, R.part);
    finish(g, 1, R, slot, slot, s);
}

int launch_spmv_dot_parts(const LevelView& A, const double* p, double* q, const double* d, double* part,
                          hipStream_t s) {
    const int g = amg::stream_blocks(A.n, kFusedParts);
    hipLaunchKernelGGL(k_stream_spmv_dot, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAxD{A.v, A.ci, p}, q, d, part);
    return g;
}

// t = A p, partials (t, t) and (t, sv)
__global__ __launch_bounds__(BS) void k_stream_spmv_dot2(int n, const int* __restrict__ rp, EntAxD ent,
                                                         double* __restrict__ t, const double* __restrict__ sv,
                                                         double* part) {
    __shared__ double prod[kStreamChunk];
    double acc[2] = {0.0, 0.0};
    for (int blk = xcd_block(blockIdx.x, gridDim.x); blk * BS < n; blk += gridDim.x) {
        const double s = stream_rows<double>(blk * BS, n, rp, ent, prod);
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
    hipLaunchKernelGGL(k_stream_spmv_dot2, dim3(g), dim3(BS), 0, s, A.n, A.rp, EntAxD{A.v, A.ci, p}, t, sv, R.part);
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
// pq_part: (Ap, p) is added here from the SpMV's partials (every block the
// same sum), and block 0 stores it in slot_pq for the host.
template <class TG>
__global__ __launch_bounds__(BS) void k_cg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ dinv, TG* __restrict__ g,
                                                  double* part, double* __restrict__ S, int slot_rho,
                                                  int slot_pq, const double* __restrict__ pq_part, int pq_np) {
    double pq;
    if (pq_part) {
        pq = block_sum_partials<BS>(pq_part, pq_np);
        if (blockIdx.x == 0 && threadIdx.x == 0) S[slot_pq] = pq;
    } else {
        pq = S[slot_pq];
    }
    const double rho = S[slot_rho];
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
        if (g) g[i] = TG(dinv[i] * ri);
        acc[0] += ri * ri;
    }
    block_partials<1, BS>(acc, part);
}

void launch_cg_update(int n, double* x, double* r, const double* p, const double* q, const double* dinv, void* gout,
                      bool g32, const Reducer& R, int slot_rho, int slot_pq, int slot_rr, hipStream_t s,
                      const double* pq_part, int pq_np, double* rr_part, int* rr_np) {
    const bool fused = pq_part != nullptr;
    int g = vec_blocks(n);
    if (fused && g > kFusedParts) g = kFusedParts;
    double* out = fused ? rr_part : R.part;
    if (g32)
        hipLaunchKernelGGL(k_cg_update<float>, dim3(g), dim3(BS), 0, s, n, x, r, p, q, dinv,
                           static_cast<float*>(gout), out, R.S, slot_rho, slot_pq, pq_part, pq_np);
    else
        hipLaunchKernelGGL(k_cg_update<double>, dim3(g), dim3(BS), 0, s, n, x, r, p, q, dinv,
                           static_cast<double*>(gout), out, R.S, slot_rho, slot_pq, pq_part, pq_np);
    if (fused) *rr_np = g;
    else finish(g, 1, R, slot_rr, slot_rr, s);
}

// p_new = z + beta p, beta = rho_new / rho.  new_part: rho_new = (r, z) is
// added here from the level-0 postsmoothing's partials (every block the same
// sum; block 0 stores it in slot_new).  rr_part: block 0 adds the update's
// (r, r) partials into slot_rr.  With Sh (host memory mapped into the device),
// block 0 then copies the first nsh scalar slots there: the iteration's last
// kernel hands its scalars to the host without a copy.
// hseq (non-null): after the slots, block 0 stores seq there (system scope),
// so a host waiting on that word knows the slots are complete.
__global__ __launch_bounds__(BS) void k_cg_dir(int n, const double* __restrict__ z, const double* __restrict__ p,
                                               double* __restrict__ pn, double* __restrict__ S, int slot_new,
                                               int slot_old, double* Sh, int nsh, const double* __restrict__ new_part,
                                               int new_np, const double* __restrict__ rr_part, int rr_np,
                                               int slot_rr, unsigned long long* hseq, unsigned long long seq) {
    const double rho_new = new_part ? block_sum_partials<BS>(new_part, new_np) : S[slot_new];
    if (blockIdx.x == 0 && (new_part || rr_part)) {
        const double rr = rr_part ? block_sum_partials<BS>(rr_part, rr_np) : 0.0;
        if (threadIdx.x == 0) {
            if (new_part) S[slot_new] = rho_new;
            if (rr_part) S[slot_rr] = rr;
        }
        __syncthreads();  // the slots just stored, for the copy below
    }
    const double beta = rho_new / S[slot_old];
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) pn[i] = z[i] + beta * p[i];
    if (Sh && blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < nsh; ++k) Sh[k] = S[k];
        if (hseq) {
            __threadfence_system();  // the slots before the sequence word
            __hip_atomic_store(hseq, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

void launch_cg_dir(int n, const double* z, const double* p, double* pn, double* S, int slot_new, int slot_old,
                   hipStream_t s, double* Sh, int nsh, const double* new_part, int new_np, const double* rr_part,
                   int rr_np, int slot_rr, unsigned long long* hseq, unsigned long long seq) {
    // every block adds the (r, z) partials itself, so with partials the grid
    // stays at kFusedParts blocks (grid-stride) to bound those reads
    int g = vec_blocks(n);
    if (new_part && g > kFusedParts) g = kFusedParts;
    hipLaunchKernelGGL(k_cg_dir, dim3(g), dim3(BS), 0, s, n, z, p, pn, S, slot_new, slot_old, Sh, nsh, new_part,
                       new_np, rr_part, rr_np, slot_rr, hseq, seq);
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
// With Sh (host memory mapped into the device), block 0 also copies the first
// nsh scalar slots there and then, with hseq, stores seq (system scope), as
// the PCG direction kernel does: the iteration's scalars reach the host
// without a copy, and the host learns they are complete from that word.
__global__ __launch_bounds__(BS) void k_bicg_dir(int n, const double* __restrict__ r, const double* __restrict__ p,
                                                 const double* __restrict__ v, double* __restrict__ pn,
                                                 const double* __restrict__ S, int slot_rho, int slot_rv, int slot_tt,
                                                 int slot_ts, int slot_rhonew, double* Sh, int nsh,
                                                 unsigned long long* hseq, unsigned long long seq) {
    const double alpha = S[slot_rho] / S[slot_rv], omega = S[slot_ts] / S[slot_tt];
    const double beta = (S[slot_rhonew] / S[slot_rho]) * (alpha / omega);
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) pn[i] = r[i] + beta * (p[i] - omega * v[i]);
    if (Sh && blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < nsh; ++k) Sh[k] = S[k];
        if (hseq) {
            __threadfence_system();  // the slots before the sequence word
            __hip_atomic_store(hseq, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

void launch_bicg_dir(int n, const double* r, const double* p, const double* v, double* pn, const double* S,
                     int slot_rho, int slot_rv, int slot_tt, int slot_ts, int slot_rhonew, hipStream_t s, double* Sh,
                     int nsh, unsigned long long* hseq, unsigned long long seq) {
    hipLaunchKernelGGL(k_bicg_dir, dim3(vec_blocks(n)), dim3(BS), 0, s, n, r, p, v, pn, S, slot_rho, slot_rv,
                       slot_tt, slot_ts, slot_rhonew, Sh, nsh, hseq, seq);
}

// x += z (one step of the stationary iteration)
__global__ __launch_bounds__(BS) void k_add(int n, double* __restrict__ x, const double* __restrict__ z) {
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) x[i] += z[i];
}

void launch_add(int n, double* x, const double* z, hipStream_t s) {
    hipLaunchKernelGGL(k_add, dim3(vec_blocks(n)), dim3(BS), 0, s, n, x, z);
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
