// V-cycle level kernels of Algorithm 1 with damped-Jacobi smoothing from a
// zero guess (one pre- and one post-sweep), piecewise-constant restriction and
// prolongation, and the exact coarsest solve.  Templated on the value type T
// of the preconditioner: double, or float with float accumulation when the
// preconditioner runs in single precision.  The level-0 right-hand side
// (TIN) and result (TOUT) may be double while T is float; the coarsest solve
// always computes in double.
//
// Data flow per level: g = D^{-1} f is written by whoever produces f; the
// down-sweep forms r = f - w A g and f_c = P^T r (with g_c); the up-sweep
// reads the prolongated iterate xp = w g + P e, which the coarser level wrote
// by scattering each of its results to its aggregate's fine rows, and smooths
// z = xp + w (g - D^{-1} A xp).
#include <hip/hip_ext.h>

#include <type_traits>

#include "amg_internal.hpp"
#include "amg_stream.hpp"

namespace amg {

namespace {
constexpr int BS = kStreamBS;

inline int level_blocks(int64_t rows, int lpr) {
    int64_t b = (rows * lpr + BS - 1) / BS;
    return (int)(b < 1 ? 1 : b);
}

// Small levels run all their blocks on one XCD, so each kernel of the
// V-cycle finds the previous one's vectors in the same L2: a launch of nb
// working blocks takes nb * kNumXcd blocks (workgroups go to the XCDs in
// turn) and only every kNumXcd-th block works.
constexpr int kPinMaxBlocks = 32;
inline int pin_of(int nb) { return nb <= kPinMaxBlocks ? 1 : 0; }
inline dim3 pinned_grid(int nb) { return dim3(pin_of(nb) ? nb * kNumXcd : nb); }
// this block's working index, or -1 for a block that only fills the other XCDs
__device__ __forceinline__ int pinned_block(int pin) {
    if (!pin) return blockIdx.x;
    return blockIdx.x % kNumXcd == 0 ? (int)(blockIdx.x / kNumXcd) : -1;
}

template <int LPR, class T>
__device__ __forceinline__ T row_ax(int row, int lane, const int* __restrict__ rp, const int* __restrict__ ci,
                                    const T* __restrict__ v, const T* __restrict__ x) {
    T s = T(0);
    const int b = rp[row], e = rp[row + 1];
    for (int k = b + lane; k < e; k += LPR) s += v[k] * x[ci[k]];
    return s;
}
}  // namespace

#define AMG_DISPATCH_LPR(lpr, CALL) \
    switch (lpr) {                  \
        case 1: CALL(1); break;     \
        case 2: CALL(2); break;     \
        case 4: CALL(4); break;     \
        case 8: CALL(8); break;     \
        default: CALL(16); break;   \
    }

// ---------------------------------------------------------------------------
// Large levels (CSR-stream)
// ---------------------------------------------------------------------------
// r = f - w A g : residual after the zero-guess presmoothing sweep
template <class T, class TIN, int RB>
__global__ __launch_bounds__(RB) void k_vc_resid(int n, const int* __restrict__ rp, EntAx<T> ent,
                                                 const TIN* __restrict__ f, T w, T* __restrict__ r) {
    __shared__ T prod[kStreamChunk];
    for (int b = xcd_block(blockIdx.x, gridDim.x); b * RB < n; b += gridDim.x) {
        const T s = stream_rows<T, RB>(b * RB, n, rp, ent, prod);
        const int row = b * RB + threadIdx.x;
        if (row < n) r[row] = T(f[row]) - w * s;
    }
}

// f_c = P^T r (members added in ascending order) and g_c = D_c^{-1} f_c
template <class T>
__global__ __launch_bounds__(BS) void k_vc_restrict(int nc, const int4* __restrict__ mem, const T* __restrict__ r,
                                                    const T* __restrict__ dinv_c, T* __restrict__ fc,
                                                    T* __restrict__ gc) {
    const int J = blockIdx.x * BS + threadIdx.x;
    if (J >= nc) return;
    const int4 m = mem[J];
    T s = r[m.x];
    if (m.y >= 0) s += r[m.y];
    if (m.z >= 0) s += r[m.z];
    if (m.w >= 0) s += r[m.w];
    fc[J] = s;
    gc[J] = dinv_c[J] * s;
}

// z = xp + w (g - D^{-1} A xp).  MODE 1 also forms block partials of (f, z)
// in double; MODE 2 scatters z to the finer level's prolongated iterate.
// GF: g = D^{-1} f is formed here from the level's right-hand side f (in
// double, whoever wrote g formed exactly this product), so g is not read.
template <class T, class TOUT, int MODE, int RB, bool GF>
__global__ __launch_bounds__(RB) void k_vc_post(int n, const int* __restrict__ rp, EntAx<T> ent,
                                                const T* __restrict__ g, const T* __restrict__ dinv, T w,
                                                TOUT* __restrict__ z, const double* __restrict__ f, double* part,
                                                ScatterT<T> sc) {
    __shared__ T prod[kStreamChunk];
    double acc[1] = {0.0};
    for (int b = xcd_block(blockIdx.x, gridDim.x); b * RB < n; b += gridDim.x) {
        const T s = stream_rows<T, RB>(b * RB, n, rp, ent, prod);
        const int row = b * RB + threadIdx.x;
        if (row < n) {
            const T di = dinv[row];
            const T gi = GF ? di * T(f[row]) : g[row];
            const T zi = ent.x[row] + w * (gi - di * s);
            z[row] = TOUT(zi);
            if (MODE == 1) acc[0] += f[row] * double(zi);
            if (MODE == 2) sc(row, zi);
        }
    }
    if (MODE == 1) block_partials<1, RB>(acc, part);
}

// The launchers pick the rows-per-block instantiation from the level.
#define AMG_DISPATCH_RB(rb, CALL) \
    switch (rb) {                 \
        case 128: CALL(128); break; \
        case 512: CALL(512); break; \
        default: CALL(256); break;  \
    }

inline int rb_blocks(int n, int rb) {
    const int b = (n + rb - 1) / rb;
    return b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks;
}

template <class T, class TIN>
void vc_stream_resid(const VLevel<T>& L, const TIN* f, const T* g, T w, T* r, hipStream_t s) {
#define CALL(RB)                                                                                                \
    hipLaunchKernelGGL((k_vc_resid<T, TIN, RB>), dim3(rb_blocks(L.n, RB)), dim3(RB), 0, s, L.n, L.rp,           \
                       EntAx<T>{L.v, L.ci, g}, f, w, r)
    AMG_DISPATCH_RB(L.rb, CALL)
#undef CALL
}

template <class T>
void vc_restrict(int nc, const int4* mem, const T* r, const T* dinv_c, T* fc, T* gc, hipStream_t s) {
    hipLaunchKernelGGL(k_vc_restrict<T>, dim3(level_blocks(nc, 1)), dim3(BS), 0, s, nc, mem, r, dinv_c, fc, gc);
}

template <class T, class TOUT, int MODE, int RB, bool GF>
void post_launch(int gsz, hipStream_t s, hipEvent_t t0, hipEvent_t t1, int n, const int* rp, const EntAx<T>& ent,
                 const T* g, const T* dinv, T w, TOUT* z, const double* f, double* part, const ScatterT<T>& sc) {
    // with t0/t1 the dispatch itself records the kernel's start and end
    if (t0)
        hipExtLaunchKernelGGL((k_vc_post<T, TOUT, MODE, RB, GF>), dim3(gsz), dim3(RB), 0, s, t0, t1, 0, n, rp, ent, g,
                              dinv, w, z, f, part, sc);
    else
        hipLaunchKernelGGL((k_vc_post<T, TOUT, MODE, RB, GF>), dim3(gsz), dim3(RB), 0, s, n, rp, ent, g, dinv, w, z, f,
                           part, sc);
}

template <class T, class TOUT, int MODE, bool GF>
int post_rb(int rb, int n, hipStream_t s, hipEvent_t t0, hipEvent_t t1, const int* rp, const EntAx<T>& ent,
            const T* g, const T* dinv, T w, TOUT* z, const double* f, double* part, const ScatterT<T>& sc,
            int cap = kRedBlocks) {
    const int gsz = rb_blocks(n, rb) < cap ? rb_blocks(n, rb) : cap;
    if (rb == 128) post_launch<T, TOUT, MODE, 128, GF>(gsz, s, t0, t1, n, rp, ent, g, dinv, w, z, f, part, sc);
    else if (rb == 512) post_launch<T, TOUT, MODE, 512, GF>(gsz, s, t0, t1, n, rp, ent, g, dinv, w, z, f, part, sc);
    else post_launch<T, TOUT, MODE, 256, GF>(gsz, s, t0, t1, n, rp, ent, g, dinv, w, z, f, part, sc);
    return gsz;
}

template <class T, class TOUT>
int vc_stream_post(const VLevel<T>& L, const T* xp, const T* g, T w, TOUT* z, const double* f, const Reducer* R,
                   int slot, const ScatterT<T>* sc, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    const int rb = L.rb == 128 || L.rb == 512 ? L.rb : 256;
    const EntAx<T> ent{L.v, L.ci, xp};
    const ScatterT<T> none{nullptr, nullptr, nullptr, T(0)};
    // a double level 0 forms g = D^{-1} f itself instead of reading it
    constexpr bool kCanGF = std::is_same<T, double>::value && std::is_same<TOUT, double>::value;
    const bool gf = kCanGF && f != nullptr;
    if (R) {
        const int cap = slot == kPartialsOnly ? kFusedParts : kRedBlocks;
        const int np =
            gf ? post_rb<T, TOUT, 1, kCanGF>(rb, L.n, s, t0, t1, L.rp, ent, g, L.dinv, w, z, f, R->part, none, cap)
               : post_rb<T, TOUT, 1, false>(rb, L.n, s, t0, t1, L.rp, ent, g, L.dinv, w, z, f, R->part, none, cap);
        if (slot == kPartialsOnly) return np;
        launch_finish(np, 1, *R, slot, slot, s);
    } else if (sc) {
        post_rb<T, TOUT, 2, false>(rb, L.n, s, t0, t1, L.rp, ent, g, L.dinv, w, z, nullptr, nullptr, *sc);
    } else if (gf) {
        post_rb<T, TOUT, 0, kCanGF>(rb, L.n, s, t0, t1, L.rp, ent, g, L.dinv, w, z, f, nullptr, none);
    } else {
        post_rb<T, TOUT, 0, false>(rb, L.n, s, t0, t1, L.rp, ent, g, L.dinv, w, z, nullptr, nullptr, none);
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Small levels (launch latency dominates): lane groups of LPR lanes per row.
// The down-sweep is fused: a group of 4*LPR lanes owns one coarse row,
// sub-group q handles member q (members ascending), and the member residuals
// are added in that order.
// ---------------------------------------------------------------------------
template <int LPR, class T, class TIN>
__global__ __launch_bounds__(BS) void k_vc_resid_restrict(int nc, const int4* __restrict__ mem,
                                                          const int* __restrict__ rp, const int* __restrict__ ci,
                                                          const T* __restrict__ v, const T* __restrict__ g,
                                                          const TIN* __restrict__ f, T w,
                                                          const T* __restrict__ dinv_c, T* __restrict__ fc,
                                                          T* __restrict__ gc, int pin) {
    constexpr int G = 4 * LPR;
    const int blk = pinned_block(pin);
    if (blk < 0) return;
    const int t = blk * BS + threadIdx.x;
    const int J = t / G, sub = (t % G) / LPR, lane = t % LPR;
    int i = -1;
    if (J < nc) {
        const int4 m = mem[J];
        i = sub == 0 ? m.x : sub == 1 ? m.y : sub == 2 ? m.z : m.w;
    }
    T s = T(0);
    if (i >= 0) s = row_ax<LPR>(i, lane, rp, ci, v, g);
    s = group_sum<LPR>(s);
    const T ri = i >= 0 ? T(f[i]) - w * s : T(0);
    const int base = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const T r0 = __shfl(ri, base, kWave);
    const T r1 = __shfl(ri, base + LPR, kWave);
    const T r2 = __shfl(ri, base + 2 * LPR, kWave);
    const T r3 = __shfl(ri, base + 3 * LPR, kWave);
    if (J < nc && (t % G) == 0) {
        const T fj = ((r0 + r1) + r2) + r3;
        fc[J] = fj;
        gc[J] = dinv_c[J] * fj;
    }
}

template <class T, class TIN>
void vc_resid_restrict(const VLevel<T>& L, int nc, const TIN* f, const T* g, T w, const T* dinv_c, T* fc, T* gc,
                       hipStream_t s) {
#define CALL(W)                                                                                          \
    {                                                                                                    \
        const int nb = level_blocks((int64_t)nc * 4, W);                                                 \
        hipLaunchKernelGGL((k_vc_resid_restrict<W, T, TIN>), pinned_grid(nb), dim3(BS), 0, s, nc, L.mem, \
                           L.rp, L.ci, L.v, g, f, w, dinv_c, fc, gc, pin_of(nb));                        \
    }
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

template <int LPR, class T, class TOUT, bool SCAT>
__global__ __launch_bounds__(BS) void k_vc_prolong_post(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci, const T* __restrict__ v,
                                                        const T* __restrict__ dinv, const T* __restrict__ g,
                                                        const T* __restrict__ xp, T w, TOUT* __restrict__ z,
                                                        ScatterT<T> sc, int pin) {
    const int blk = pinned_block(pin);
    if (blk < 0) return;
    const int t = blk * BS + threadIdx.x;
    const int row = t / LPR, lane = t % LPR;
    T s = row < n ? row_ax<LPR>(row, lane, rp, ci, v, xp) : T(0);
    s = group_sum<LPR>(s);
    if (row < n && lane == 0) {
        const T zi = xp[row] + w * (g[row] - dinv[row] * s);
        z[row] = TOUT(zi);
        if (SCAT) sc(row, zi);
    }
}

template <class T, class TOUT>
void vc_prolong_post(const VLevel<T>& L, const T* xp, const T* g, T w, TOUT* z, const ScatterT<T>* sc,
                     hipStream_t s) {
    const ScatterT<T> none{nullptr, nullptr, nullptr, T(0)};
#define CALL(W)                                                                                          \
    {                                                                                                    \
        const int nb = level_blocks(L.n, W);                                                             \
        if (sc)                                                                                          \
            hipLaunchKernelGGL((k_vc_prolong_post<W, T, TOUT, true>), pinned_grid(nb), dim3(BS), 0, s, L.n, \
                               L.rp, L.ci, L.v, L.dinv, g, xp, w, z, *sc, pin_of(nb));                   \
        else                                                                                             \
            hipLaunchKernelGGL((k_vc_prolong_post<W, T, TOUT, false>), pinned_grid(nb), dim3(BS), 0, s, L.n, \
                               L.rp, L.ci, L.v, L.dinv, g, xp, w, z, none, pin_of(nb));                  \
    }
    AMG_DISPATCH_LPR(L.lpr, CALL)
#undef CALL
}

// ---------------------------------------------------------------------------
// Level-0 scaling g = D^{-1} f, and the coarsest level x = A_L^{-1} f in
// double with the inverse stored column-major.  With a scatter, x also
// becomes the finer level's prolongated iterate.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(BS) void k_vc_scale_dinv(int n, const double* __restrict__ dinv,
                                                      const double* __restrict__ f, T* __restrict__ g) {
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) g[i] = T(dinv[i] * f[i]);
}

template <class T>
void vc_scale_dinv(int n, const double* dinv, const double* f, T* g, hipStream_t s) {
    int b = (n + BS - 1) / BS;
    b = b < 1 ? 1 : (b > kRedBlocks ? kRedBlocks : b);
    hipLaunchKernelGGL(k_vc_scale_dinv<T>, dim3(b), dim3(BS), 0, s, n, dinv, f, g);
}

constexpr int DENSE_BS = 512;    // 8 waves
constexpr int DENSE_ROWS = kWave;  // rows per block, one per lane
constexpr int DENSE_WAVES = DENSE_BS / kWave;

// x = A_L^{-1} f: a block owns 64 rows (one per lane, coalesced reads of the
// column-major inverse); its 8 waves split the columns round-robin, each wave
// keeps DENSE_ACC sums over its columns in turn (so that many loads are in
// flight: the product is latency-bound at a few hundred rows), and the sums
// are added in a fixed order, then the waves' in wave order, so the result is
// reproducible.
constexpr int DENSE_ACC = 8;
template <class T, class TIN, class TOUT>
__global__ __launch_bounds__(DENSE_BS) void k_vc_dense(int n, const double* __restrict__ ainv_t,
                                                       const TIN* __restrict__ f, TOUT* __restrict__ x,
                                                       ScatterT<T> sc, int pin) {
    __shared__ double fs[kDenseMaxRows];
    __shared__ double part[DENSE_WAVES][DENSE_ROWS];
    const int blk = pinned_block(pin);
    if (blk < 0) return;
    for (int j = threadIdx.x; j < n; j += DENSE_BS) fs[j] = double(f[j]);
    __syncthreads();
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int i = blk * DENSE_ROWS + lane;
    double acc[DENSE_ACC];
#pragma unroll
    for (int k = 0; k < DENSE_ACC; ++k) acc[k] = 0.0;
    if (i < n) {
        // a group of DENSE_ACC columns a step, loaded together: a column past the
        // end loads column j0 again (in bounds) and is not added, so no load
        // waits behind a branch
        for (int j0 = w; j0 < n; j0 += DENSE_ACC * DENSE_WAVES) {
            double a[DENSE_ACC];
#pragma unroll
            for (int k = 0; k < DENSE_ACC; ++k) {
                const int j = j0 + k * DENSE_WAVES;
                a[k] = ainv_t[(size_t)(j < n ? j : j0) * n + i];
            }
#pragma unroll
            for (int k = 0; k < DENSE_ACC; ++k) {
                const int j = j0 + k * DENSE_WAVES;
                if (j < n) acc[k] += a[k] * fs[j];
            }
        }
    }
#pragma unroll
    for (int k = DENSE_ACC / 2; k > 0; k /= 2)
#pragma unroll
        for (int q = 0; q < k; ++q) acc[q] += acc[q + k];
    part[w][lane] = acc[0];
    __syncthreads();
    if (w == 0 && i < n) {
        double xi = part[0][lane];
#pragma unroll
        for (int k = 1; k < DENSE_WAVES; ++k) xi += part[k][lane];
        x[i] = TOUT(xi);
        if (sc.mem) sc(i, T(xi));
    }
}

template <class T, class TIN, class TOUT>
void vc_dense_apply(int n, const double* ainv_t, const TIN* f, TOUT* x, const ScatterT<T>* sc, hipStream_t s) {
    const ScatterT<T> none{nullptr, nullptr, nullptr, T(0)};
    const int nb = (n + DENSE_ROWS - 1) / DENSE_ROWS;
    hipLaunchKernelGGL((k_vc_dense<T, TIN, TOUT>), pinned_grid(nb), dim3(DENSE_BS), 0, s, n, ainv_t, f, x,
                       sc ? *sc : none, pin_of(nb));
}

// float copies of the level values and inverse diagonals, rounded to nearest
__global__ __launch_bounds__(BS) void k_cast_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) b[i] = float(a[i]);
}

void launch_cast_f32(int64_t n, const double* a, float* b, hipStream_t s) {
    if (n <= 0) return;
    int64_t blk = (n + BS - 1) / BS;
    if (blk > kRedBlocks) blk = kRedBlocks;
    hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)blk), dim3(BS), 0, s, n, a, b);
}

// explicit instantiations: the double cycle, and the float cycle with a
// double right-hand side and result on level 0
#define AMG_INST(T)                                                                                                 \
    template void vc_stream_resid<T, T>(const VLevel<T>&, const T*, const T*, T, T*, hipStream_t);                   \
    template void vc_restrict<T>(int, const int4*, const T*, const T*, T*, T*, hipStream_t);                         \
    template int vc_stream_post<T, T>(const VLevel<T>&, const T*, const T*, T, T*, const double*, const Reducer*,   \
                                      int, const ScatterT<T>*, hipStream_t, hipEvent_t, hipEvent_t);                 \
    template void vc_resid_restrict<T, T>(const VLevel<T>&, int, const T*, const T*, T, const T*, T*, T*,            \
                                          hipStream_t);                                                               \
    template void vc_prolong_post<T, T>(const VLevel<T>&, const T*, const T*, T, T*, const ScatterT<T>*,            \
                                        hipStream_t);                                                                 \
    template void vc_scale_dinv<T>(int, const double*, const double*, T*, hipStream_t);                              \
    template void vc_dense_apply<T, T, T>(int, const double*, const T*, T*, const ScatterT<T>*, hipStream_t);
AMG_INST(double)
AMG_INST(float)
#undef AMG_INST
template void vc_stream_resid<float, double>(const VLevel<float>&, const double*, const float*, float, float*,
                                             hipStream_t);
template int vc_stream_post<float, double>(const VLevel<float>&, const float*, const float*, float, double*,
                                            const double*, const Reducer*, int, const ScatterT<float>*, hipStream_t,
                                            hipEvent_t, hipEvent_t);
template void vc_resid_restrict<float, double>(const VLevel<float>&, int, const double*, const float*, float,
                                               const float*, float*, float*, hipStream_t);
template void vc_prolong_post<float, double>(const VLevel<float>&, const float*, const float*, float, double*,
                                             const ScatterT<float>*, hipStream_t);

}  // namespace amg
