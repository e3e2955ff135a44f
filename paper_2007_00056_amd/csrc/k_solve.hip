// Solve-phase kernels: CSR SpMV, the fused V-cycle level kernels of
// Algorithm 1 (damped Jacobi, residual, piecewise-constant restriction and
// prolongation), the coarsest dense solve, and the vector kernels of
// Algorithm 4 (PCG) and Algorithm 5 (BiCGStab).
//
// CSR rows are processed by groups of LPR consecutive lanes (LPR in 1..16):
// each lane walks the row with stride LPR, so a group reads a contiguous row
// segment, and a butterfly shuffle combines the lanes.  Level kernels map
// blocks XCD-contiguously so neighbouring rows share an L2.
#include "amg_device.hpp"
#include "amg_internal.hpp"

namespace amg {

namespace {
constexpr int BS = 256;

inline int level_blocks(int64_t rows, int lpr) {
    int64_t b = (rows * lpr + BS - 1) / BS;
    return (int)(b < 1 ? 1 : b);
}

inline int red_blocks(int64_t rows, int lpr) {
    int64_t b = (rows * lpr + BS - 1) / BS;
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
    if (avg <= 1.5) return 1;
    if (avg <= 3.0) return 2;
    if (avg <= 6.0) return 4;
    if (avg <= 12.0) return 8;
    return 16;
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
// y = A x
// ---------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(BS) void k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                             const double* __restrict__ v, const double* __restrict__ x,
                                             double* __restrict__ y) {
    const int t = xcd_block(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    const int row = t / LPR, lane = t % LPR;
    double s = row < n ? row_ax<LPR>(row, lane, rp, ci, v, x) : 0.0;
    s = group_sum<LPR>(s);
    if (row < n && lane == 0) y[row] = s;
}

void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t s) {
#define CALL(W) hipLaunchKernelGGL(k_spmv<W>, dim3(level_blocks(L.n, W)), dim3(BS), 0, s, L.n, L.rp, L.ci, L.v, x, y)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

// ---------------------------------------------------------------------------
// Down-sweep of Algorithm 1 on one level, fused: presmoothing from the zero
// guess x = w D^{-1} f, residual r = f - A x and restriction f_c = P^T r.
// A group of 4*LPR lanes owns one coarse row; sub-group q handles member q
// (members ascending) and the member residuals are added in that order.
// ---------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(BS) void k_resid_restrict(int nc, const int4* __restrict__ mem,
                                                       const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ dinv,
                                                       const double* __restrict__ f, double w,
                                                       double* __restrict__ fc) {
    constexpr int G = 4 * LPR;
    const int t = xcd_block(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    const int J = t / G, sub = (t % G) / LPR, lane = t % LPR;
    int i = -1;
    if (J < nc) {
        const int4 m = mem[J];
        i = sub == 0 ? m.x : sub == 1 ? m.y : sub == 2 ? m.z : m.w;
    }
    double s = 0.0;
    if (i >= 0) {
        const int b = rp[i], e = rp[i + 1];
        for (int k = b + lane; k < e; k += LPR) {
            const int j = ci[k];
            s += v[k] * (dinv[j] * f[j]);
        }
    }
    s = group_sum<LPR>(s);
    const double ri = i >= 0 ? f[i] - w * s : 0.0;
    const int base = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const double r0 = __shfl(ri, base, kWave);
    const double r1 = __shfl(ri, base + LPR, kWave);
    const double r2 = __shfl(ri, base + 2 * LPR, kWave);
    const double r3 = __shfl(ri, base + 3 * LPR, kWave);
    if (J < nc && (t % G) == 0) fc[J] = ((r0 + r1) + r2) + r3;
}

void launch_resid_restrict(const LevelView& L, int nc, const double* f, double w, double* fc, hipStream_t s) {
#define CALL(W)                                                                                                 \
    hipLaunchKernelGGL(k_resid_restrict<W>, dim3(level_blocks((int64_t)nc * 4, W)), dim3(BS), 0, s, nc, L.mem, \
                       L.rp, L.ci, L.v, L.dinv, f, w, fc)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

// ---------------------------------------------------------------------------
// Up-sweep of Algorithm 1 on one level, fused: prolongation x = x_pre + P e
// (x_pre = w D^{-1} f recomputed on the fly) and one damped-Jacobi
// postsmoothing sweep z = x + w D^{-1} (f - A x).
// ---------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(BS) void k_prolong_post(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ f, const int* __restrict__ agg,
                                                     const double* __restrict__ e, double w,
                                                     double* __restrict__ z) {
    const int t = xcd_block(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    const int row = t / LPR, lane = t % LPR;
    double s = 0.0;
    if (row < n) {
        const int b = rp[row], end = rp[row + 1];
        for (int k = b + lane; k < end; k += LPR) {
            const int j = ci[k];
            s += v[k] * (w * (dinv[j] * f[j]) + e[agg[j]]);
        }
    }
    s = group_sum<LPR>(s);
    if (row < n && lane == 0) {
        const double di = dinv[row], fi = f[row];
        const double xi = w * (di * fi) + e[agg[row]];
        z[row] = xi + w * (di * (fi - s));
    }
}

void launch_prolong_post(const LevelView& L, const double* f, const double* e, double w, double* z, hipStream_t s) {
#define CALL(W)                                                                                                       \
    hipLaunchKernelGGL(k_prolong_post<W>, dim3(level_blocks(L.n, W)), dim3(BS), 0, s, L.n, L.rp, L.ci, L.v, L.dinv, \
                       f, L.agg, e, w, z)
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
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
    const int t = xcd_block(blockIdx.x, gridDim.x) * BS + threadIdx.x;
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

// Coarsest level: x = A_L^{-1} f with the inverse stored column-major.
__global__ __launch_bounds__(64) void k_dense_apply(int n, const double* __restrict__ ainv_t,
                                                   const double* __restrict__ f, double* __restrict__ x) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += ainv_t[(size_t)j * n + i] * f[j];
    x[i] = s;
}

void launch_dense_apply(int n, const double* ainv_t, const double* f, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_apply, dim3((n + 63) / 64), dim3(64), 0, s, n, ainv_t, f, x);
}

// ---------------------------------------------------------------------------
// Krylov kernels.  Reductions go through reduce_store (deterministic); the
// scalars of the recurrences are read from device slots, so no host round
// trip sits between the kernels of one iteration.  Update kernels skip the
// update when the denominator they depend on is zero or not finite; the host
// reports the breakdown after reading the slots.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool usable(double d) { return isfinite(d) && d != 0.0; }

template <int LPR>
__global__ __launch_bounds__(BS) void k_residual(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ v, const double* __restrict__ b,
                                                 const double* __restrict__ x, double* __restrict__ r, double* part,
                                                 unsigned* ticket, double* S, int slot) {
    double acc[1] = {0.0};
    const int stride = gridDim.x * BS / LPR;
    const int t = blockIdx.x * BS + threadIdx.x;
    const int lane = t % LPR;
    for (int row = t / LPR; row < n; row += stride) {
        const double s = group_sum<LPR>(row_ax<LPR>(row, lane, rp, ci, v, x));
        if (lane == 0) {
            const double ri = b[row] - s;
            r[row] = ri;
            acc[0] += ri * ri;
        }
    }
    const int sl[1] = {slot};
    reduce_store<1, BS>(acc, part, ticket, S, sl);
}

void launch_residual(const LevelView& A, const double* b, const double* x, double* r, const Reducer& R, int slot,
                     hipStream_t s) {
#define CALL(W)                                                                                             \
    hipLaunchKernelGGL(k_residual<W>, dim3(red_blocks(A.n, W)), dim3(BS), 0, s, A.n, A.rp, A.ci, A.v, b, x, r, \
                       R.part, R.ticket, R.S, slot)
    AMG_DISPATCH_LPR(A.lpr, CALL)
#undef CALL
}

__global__ __launch_bounds__(BS) void k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                            double* part, unsigned* ticket, double* S, int slot) {
    double acc[1] = {0.0};
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) acc[0] += a[i] * b[i];
    const int sl[1] = {slot};
    reduce_store<1, BS>(acc, part, ticket, S, sl);
}

void launch_dot(int n, const double* a, const double* b, const Reducer& R, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_dot, dim3(red_blocks(n, 1)), dim3(BS), 0, s, n, a, b, R.part, R.ticket, R.S, slot);
}

// q = A p and (d, q)
template <int LPR>
__global__ __launch_bounds__(BS) void k_spmv_dot(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ v, const double* __restrict__ p,
                                                 double* __restrict__ q, const double* __restrict__ d, double* part,
                                                 unsigned* ticket, double* S, int slot) {
    double acc[1] = {0.0};
    const int stride = gridDim.x * BS / LPR;
    const int t = blockIdx.x * BS + threadIdx.x;
    const int lane = t % LPR;
    for (int row = t / LPR; row < n; row += stride) {
        const double s = group_sum<LPR>(row_ax<LPR>(row, lane, rp, ci, v, p));
        if (lane == 0) {
            q[row] = s;
            acc[0] += d[row] * s;
        }
    }
    const int sl[1] = {slot};
    reduce_store<1, BS>(acc, part, ticket, S, sl);
}

void launch_spmv_dot(const LevelView& A, const double* p, double* q, const double* d, const Reducer& R, int slot,
                     hipStream_t s) {
#define CALL(W)                                                                                             \
    hipLaunchKernelGGL(k_spmv_dot<W>, dim3(red_blocks(A.n, W)), dim3(BS), 0, s, A.n, A.rp, A.ci, A.v, p, q, d, \
                       R.part, R.ticket, R.S, slot)
    AMG_DISPATCH_LPR(A.lpr, CALL)
#undef CALL
}

// t = A p, (t, t) and (t, sv)
template <int LPR>
__global__ __launch_bounds__(BS) void k_spmv_dot2(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double* __restrict__ v, const double* __restrict__ p,
                                                  double* __restrict__ tq, const double* __restrict__ sv,
                                                  double* part, unsigned* ticket, double* S, int slot_tt,
                                                  int slot_ts) {
    double acc[2] = {0.0, 0.0};
    const int stride = gridDim.x * BS / LPR;
    const int t = blockIdx.x * BS + threadIdx.x;
    const int lane = t % LPR;
    for (int row = t / LPR; row < n; row += stride) {
        const double s = group_sum<LPR>(row_ax<LPR>(row, lane, rp, ci, v, p));
        if (lane == 0) {
            tq[row] = s;
            acc[0] += s * s;
            acc[1] += s * sv[row];
        }
    }
    const int sl[2] = {slot_tt, slot_ts};
    reduce_store<2, BS>(acc, part, ticket, S, sl);
}

void launch_spmv_dot2(const LevelView& A, const double* p, double* t, const double* sv, const Reducer& R, int slot_tt,
                      int slot_ts, hipStream_t s) {
#define CALL(W)                                                                                               \
    hipLaunchKernelGGL(k_spmv_dot2<W>, dim3(red_blocks(A.n, W)), dim3(BS), 0, s, A.n, A.rp, A.ci, A.v, p, t, sv, \
                       R.part, R.ticket, R.S, slot_tt, slot_ts)
    AMG_DISPATCH_LPR(A.lpr, CALL)
#undef CALL
}

// Algorithm 4: alpha = (r,z)/(Ap,p); x += alpha p; r -= alpha Ap; (r,r).
__global__ __launch_bounds__(BS) void k_cg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  double* part, unsigned* ticket, double* S, int slot_rho,
                                                  int slot_pq, int slot_rr) {
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
        acc[0] += ri * ri;
    }
    const int sl[1] = {slot_rr};
    reduce_store<1, BS>(acc, part, ticket, S, sl);
}

void launch_cg_update(int n, double* x, double* r, const double* p, const double* q, const Reducer& R, int slot_rho,
                      int slot_pq, int slot_rr, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update, dim3(red_blocks(n, 1)), dim3(BS), 0, s, n, x, r, p, q, R.part, R.ticket, R.S,
                       slot_rho, slot_pq, slot_rr);
}

// p_new = z + beta p, beta = rho_new / rho
__global__ __launch_bounds__(BS) void k_cg_dir(int n, const double* __restrict__ z, const double* __restrict__ p,
                                               double* __restrict__ pn, const double* __restrict__ S, int slot_new,
                                               int slot_old) {
    const double beta = S[slot_new] / S[slot_old];
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) pn[i] = z[i] + beta * p[i];
}

void launch_cg_dir(int n, const double* z, const double* p, double* pn, const double* S, int slot_new, int slot_old,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir, dim3(level_blocks(n, 1)), dim3(BS), 0, s, n, z, p, pn, S, slot_new, slot_old);
}

// Algorithm 5: s = r - alpha v, alpha = rho / (rbar, v)
__global__ __launch_bounds__(BS) void k_bicg_s(int n, const double* __restrict__ r, const double* __restrict__ v,
                                               double* __restrict__ sv, const double* __restrict__ S, int slot_rho,
                                               int slot_rv) {
    const double alpha = S[slot_rho] / S[slot_rv];
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) sv[i] = r[i] - alpha * v[i];
}

void launch_bicg_s(int n, const double* r, const double* v, double* sv, const double* S, int slot_rho, int slot_rv,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_s, dim3(level_blocks(n, 1)), dim3(BS), 0, s, n, r, v, sv, S, slot_rho, slot_rv);
}

// x += alpha pt + omega st; r = s - omega t; (r,r) and (r, rbar)
__global__ __launch_bounds__(BS) void k_bicg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ pt, const double* __restrict__ st,
                                                    const double* __restrict__ sv, const double* __restrict__ t,
                                                    const double* __restrict__ rb, double* part, unsigned* ticket,
                                                    double* S, int slot_rho, int slot_rv, int slot_tt, int slot_ts,
                                                    int slot_rr, int slot_rhonew) {
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
    const int sl[2] = {slot_rr, slot_rhonew};
    reduce_store<2, BS>(acc, part, ticket, S, sl);
}

void launch_bicg_update(int n, double* x, double* r, const double* pt, const double* st, const double* sv,
                        const double* t, const double* rb, const Reducer& R, int slot_rho, int slot_rv, int slot_tt,
                        int slot_ts, int slot_rr, int slot_rhonew, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_update, dim3(red_blocks(n, 1)), dim3(BS), 0, s, n, x, r, pt, st, sv, t, rb, R.part,
                       R.ticket, R.S, slot_rho, slot_rv, slot_tt, slot_ts, slot_rr, slot_rhonew);
}

// p_new = r + beta (p - omega v), beta = (rho_new / rho) (alpha / omega)
__global__ __launch_bounds__(BS) void k_bicg_dir(int n, const double* __restrict__ r, const double* __restrict__ p,
                                                 const double* __restrict__ v, double* __restrict__ pn,
                                                 const double* __restrict__ S, int slot_rho, int slot_rv, int slot_tt,
                                                 int slot_ts, int slot_rhonew) {
    const double alpha = S[slot_rho] / S[slot_rv], omega = S[slot_ts] / S[slot_tt];
    const double beta = (S[slot_rhonew] / S[slot_rho]) * (alpha / omega);
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) pn[i] = r[i] + beta * (p[i] - omega * v[i]);
}

void launch_bicg_dir(int n, const double* r, const double* p, const double* v, double* pn, const double* S,
                     int slot_rho, int slot_rv, int slot_tt, int slot_ts, int slot_rhonew, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_dir, dim3(level_blocks(n, 1)), dim3(BS), 0, s, n, r, p, v, pn, S, slot_rho, slot_rv,
                       slot_tt, slot_ts, slot_rhonew);
}

__global__ __launch_bounds__(BS) void k_zero(int n, double* __restrict__ x) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

void launch_scale_zero(int n, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(level_blocks(n, 1)), dim3(BS), 0, s, n, x);
}

__global__ __launch_bounds__(BS) void k_check_finite(int n, const double* __restrict__ a,
                                                     const double* __restrict__ b, int* err) {
    bool bad = false;
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) bad |= !isfinite(a[i]) || !isfinite(b[i]);
    if (bad) atomicOr(err, ERR_NONFINITE);
}

void launch_check_finite(int n, const double* a, const double* b, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(red_blocks(n, 1)), dim3(BS), 0, s, n, a, b, err);
}

}  // namespace amg
