// Kernels of batched solves: many independent systems stored one after
// another ("segments") and advanced together, each launch covering every
// system.  Rows of the level operators are independent, so the V-cycle runs
// the ordinary CSR-stream level kernels on the concatenated levels; what needs
// the segment structure is here: the per-system Krylov scalars, the coarsest
// solves, and the copies that assemble a batch.
//
// Every reduction block lies inside one segment and covers 256 rows at a
// fixed offset from the segment's start; a segment's block partials are added
// in a fixed order.  A system's scalars therefore depend on its own data
// only, not on which other systems share the batch.  A mask (one int per
// segment) switches finished systems off: their blocks write a zero partial
// and leave every vector untouched.
#include "amg_internal.hpp"
#include "amg_stream.hpp"

namespace amg {

namespace {
constexpr int BS = kStreamBS;  // rows per reduction block
constexpr int GATHER_CHUNK = 2048;

__device__ __forceinline__ bool usable(double d) { return isfinite(d) && d != 0.0; }

__device__ __forceinline__ double* slot(double* S, int seg, int k) { return S + (size_t)seg * kBatchSlots + k; }
__device__ __forceinline__ double slotv(const double* S, int seg, int k) { return S[(size_t)seg * kBatchSlots + k]; }
}  // namespace

// q = A p over a block's rows; partial (d, q)
__global__ __launch_bounds__(BS) void k_bspmv_dot(BatchTab T, const int* __restrict__ rp, EntAx<double> ent,
                                                  double* __restrict__ q, const double* __restrict__ d,
                                                  double* part) {
    __shared__ double prod[kStreamChunk];
    const int2 b = T.blk[blockIdx.x];
    if (!T.mask[b.x]) {
        if (threadIdx.x == 0) part[blockIdx.x] = 0.0;
        return;
    }
    const int end = T.seg_end[b.x];
    const double s = stream_rows<double>(b.y, end, rp, ent, prod);
    const int row = b.y + threadIdx.x;
    double acc[1] = {0.0};
    if (row < end) {
        q[row] = s;
        acc[0] = d[row] * s;
    }
    block_partials<1, BS>(acc, part);
}

// r = b - A x, g = D^{-1} r (as TG); partial (r, r)
template <class TG>
__global__ __launch_bounds__(BS) void k_bresidual(BatchTab T, const int* __restrict__ rp, EntAx<double> ent,
                                                  const double* __restrict__ b, double* __restrict__ r,
                                                  const double* __restrict__ dinv, TG* __restrict__ g, double* part) {
    __shared__ double prod[kStreamChunk];
    const int2 bk = T.blk[blockIdx.x];
    if (!T.mask[bk.x]) {
        if (threadIdx.x == 0) part[blockIdx.x] = 0.0;
        return;
    }
    const int end = T.seg_end[bk.x];
    const double s = stream_rows<double>(bk.y, end, rp, ent, prod);
    const int row = bk.y + threadIdx.x;
    double acc[1] = {0.0};
    if (row < end) {
        const double ri = b[row] - s;
        r[row] = ri;
        g[row] = TG(dinv[row] * ri);
        acc[0] = ri * ri;
    }
    block_partials<1, BS>(acc, part);
}

// partial (a, c)
__global__ __launch_bounds__(BS) void k_bdot(BatchTab T, const double* __restrict__ a, const double* __restrict__ c,
                                             double* part) {
    const int2 bk = T.blk[blockIdx.x];
    double acc[1] = {0.0};
    if (T.mask[bk.x]) {
        const int row = bk.y + threadIdx.x;
        if (row < T.seg_end[bk.x]) acc[0] = a[row] * c[row];
    }
    block_partials<1, BS>(acc, part);
}

// S[seg][slot] = sum of the segment's block partials (one wave per segment)
__global__ __launch_bounds__(kWave) void k_bfinish(const int* __restrict__ seg_blk, const int* __restrict__ mask,
                                                   const double* __restrict__ part, double* __restrict__ S,
                                                   int slot_k) {
    const int seg = blockIdx.x;
    if (!mask[seg]) return;
    const int b0 = seg_blk[seg], b1 = seg_blk[seg + 1];
    double s = 0.0;
    for (int b = b0 + (int)threadIdx.x; b < b1; b += kWave) s += part[b];
    s = group_sum<kWave>(s);
    if (threadIdx.x == 0) *slot(S, seg, slot_k) = s;
}

// Algorithm 4: alpha = (r,z)/(Ap,p); x += alpha p; r -= alpha Ap; g = D^{-1} r;
// partial (r, r).  A segment whose denominators are unusable keeps x and r.
template <class TG>
__global__ __launch_bounds__(BS) void k_bcg_update(BatchTab T, double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   const double* __restrict__ dinv, TG* __restrict__ g, double* part,
                                                   const double* __restrict__ S, int slot_rho, int slot_pq) {
    const int2 bk = T.blk[blockIdx.x];
    double acc[1] = {0.0};
    if (T.mask[bk.x]) {
        const double rho = slotv(S, bk.x, slot_rho), pq = slotv(S, bk.x, slot_pq);
        const bool ok = usable(pq) && isfinite(rho);
        const double alpha = ok ? rho / pq : 0.0;
        const int i = bk.y + threadIdx.x;
        if (i < T.seg_end[bk.x]) {
            double ri = r[i];
            if (ok) {
                x[i] += alpha * p[i];
                ri -= alpha * q[i];
                r[i] = ri;
            }
            g[i] = TG(dinv[i] * ri);
            acc[0] = ri * ri;
        }
    }
    block_partials<1, BS>(acc, part);
}

// p_new = z + beta p, beta = rho_new / rho
__global__ __launch_bounds__(BS) void k_bcg_dir(BatchTab T, const double* __restrict__ z,
                                                const double* __restrict__ p, double* __restrict__ pn,
                                                const double* __restrict__ S, int slot_new, int slot_old) {
    const int2 bk = T.blk[blockIdx.x];
    if (!T.mask[bk.x]) return;
    const double beta = slotv(S, bk.x, slot_new) / slotv(S, bk.x, slot_old);
    const int i = bk.y + threadIdx.x;
    if (i < T.seg_end[bk.x]) pn[i] = z[i] + beta * p[i];
}

// Algorithm 5 over a batch.  s = r - alpha v, alpha = rho / (rbar, v)
__global__ __launch_bounds__(BS) void k_bbicg_s(BatchTab T, const double* __restrict__ r,
                                                const double* __restrict__ v, double* __restrict__ sv,
                                                const double* __restrict__ S, int slot_rho, int slot_rv) {
    const int2 bk = T.blk[blockIdx.x];
    if (!T.mask[bk.x]) return;
    const double alpha = slotv(S, bk.x, slot_rho) / slotv(S, bk.x, slot_rv);
    const int i = bk.y + threadIdx.x;
    if (i < T.seg_end[bk.x]) sv[i] = r[i] - alpha * v[i];
}

// t = A s; partials (t, t) at part[b] and (t, s) at part[nblk + b]
__global__ __launch_bounds__(BS) void k_bspmv_dot2(BatchTab T, const int* __restrict__ rp, EntAx<double> ent,
                                                   double* __restrict__ t, const double* __restrict__ sv,
                                                   double* part) {
    __shared__ double prod[kStreamChunk];
    const int2 bk = T.blk[blockIdx.x];
    double acc[2] = {0.0, 0.0};
    if (T.mask[bk.x]) {  // uniform per block
        const int end = T.seg_end[bk.x];
        const double s = stream_rows<double>(bk.y, end, rp, ent, prod);
        const int row = bk.y + threadIdx.x;
        if (row < end) {
            t[row] = s;
            acc[0] = s * s;
            acc[1] = s * sv[row];
        }
    }
    block_partials<2, BS>(acc, part);
}

// x += alpha pt + omega st; r = s - omega t; partials (r, r) and (r, rbar).
// A segment whose scalars are unusable keeps x and r.
__global__ __launch_bounds__(BS) void k_bbicg_update(BatchTab T, double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ pt, const double* __restrict__ st,
                                                     const double* __restrict__ sv, const double* __restrict__ t,
                                                     const double* __restrict__ rb, double* part,
                                                     const double* __restrict__ S, int slot_rho, int slot_rv,
                                                     int slot_tt, int slot_ts) {
    const int2 bk = T.blk[blockIdx.x];
    double acc[2] = {0.0, 0.0};
    if (T.mask[bk.x]) {
        const double rho = slotv(S, bk.x, slot_rho), rv = slotv(S, bk.x, slot_rv);
        const double tt = slotv(S, bk.x, slot_tt), ts = slotv(S, bk.x, slot_ts);
        const bool ok = usable(rho) && usable(rv) && usable(tt) && isfinite(ts);
        const double alpha = ok ? rho / rv : 0.0, omega = ok ? ts / tt : 0.0;
        const int i = bk.y + threadIdx.x;
        if (i < T.seg_end[bk.x]) {
            double ri = r[i];
            if (ok) {
                x[i] = x[i] + alpha * pt[i] + omega * st[i];
                ri = sv[i] - omega * t[i];
                r[i] = ri;
            }
            acc[0] = ri * ri;
            acc[1] = ri * rb[i];
        }
    }
    block_partials<2, BS>(acc, part);
}

// p_new = r + beta (p - omega v), beta = (rho_new / rho) (alpha / omega)
__global__ __launch_bounds__(BS) void k_bbicg_dir(BatchTab T, const double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ v,
                                                  double* __restrict__ pn, const double* __restrict__ S, int slot_rho,
                                                  int slot_rv, int slot_tt, int slot_ts, int slot_rhonew) {
    const int2 bk = T.blk[blockIdx.x];
    if (!T.mask[bk.x]) return;
    const int g = bk.x;
    const double alpha = slotv(S, g, slot_rho) / slotv(S, g, slot_rv);
    const double omega = slotv(S, g, slot_ts) / slotv(S, g, slot_tt);
    const double beta = (slotv(S, g, slot_rhonew) / slotv(S, g, slot_rho)) * (alpha / omega);
    const int i = bk.y + threadIdx.x;
    if (i < T.seg_end[g]) pn[i] = r[i] + beta * (p[i] - omega * v[i]);
}

__global__ __launch_bounds__(BS) void k_bzero(BatchTab T, double* __restrict__ x) {
    const int2 bk = T.blk[blockIdx.x];
    if (!T.mask[bk.x]) return;
    const int i = bk.y + threadIdx.x;
    if (i < T.seg_end[bk.x]) x[i] = 0.0;
}

// Coarsest solves x = A_L^{-1} f of every segment (explicit inverse, column
// major), 64 rows per block with the columns split over 8 waves; each wave
// keeps ACC sums over its columns in turn (loads in flight), added in a fixed
// order, then the waves' in wave order; each result is scattered to the
// segment's finer level.  Block b handles rows 64*tab[b].y.. of segment
// tab[b].x.
template <class T>
__global__ __launch_bounds__(512) void k_bdense(const BDense<T>* __restrict__ dd, const int2* __restrict__ tab) {
    constexpr int ROWS = 64, WAVES = 8, ACC = 8;
    __shared__ double fs[kDenseMaxRows];
    __shared__ double psum[WAVES][ROWS];
    const int2 bk = tab[blockIdx.x];
    const BDense<T> d = dd[bk.x];
    const int n = d.n;
    for (int j = threadIdx.x; j < n; j += 512) fs[j] = double(d.f[j]);
    __syncthreads();
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int i = bk.y * ROWS + lane;
    double acc[ACC];
#pragma unroll
    for (int k = 0; k < ACC; ++k) acc[k] = 0.0;
    if (i < n) {
        // a group of ACC columns a step, loaded together: a column past the
        // end loads column j0 again (in bounds) and is not added, so no load
        // waits behind a branch
        for (int j0 = w; j0 < n; j0 += ACC * WAVES) {
            double a[ACC];
#pragma unroll
            for (int k = 0; k < ACC; ++k) {
                const int j = j0 + k * WAVES;
                a[k] = d.ainv_t[(size_t)(j < n ? j : j0) * n + i];
            }
#pragma unroll
            for (int k = 0; k < ACC; ++k) {
                const int j = j0 + k * WAVES;
                if (j < n) acc[k] += a[k] * fs[j];
            }
        }
    }
#pragma unroll
    for (int k = ACC / 2; k > 0; k /= 2)
#pragma unroll
        for (int q = 0; q < k; ++q) acc[q] += acc[q + k];
    psum[w][lane] = acc[0];
    __syncthreads();
    if (w == 0 && i < n) {
        double xi = psum[0][lane];
#pragma unroll
        for (int k = 1; k < WAVES; ++k) xi += psum[k][lane];
        d.x[i] = T(xi);
        d.sc(d.row0 + i, T(xi));
    }
}

// Batch assembly: piece p copies count elements from src to dst, adding `add`
// to int32 elements and to the non-negative components of int4 elements.
__global__ __launch_bounds__(BS) void k_gather(const GatherPiece* __restrict__ pcs, const int2* __restrict__ tab) {
    const int2 bk = tab[blockIdx.x];
    const GatherPiece P = pcs[bk.x];
    const int64_t e0 = (int64_t)bk.y * GATHER_CHUNK;
    const int64_t e1 = e0 + GATHER_CHUNK < P.count ? e0 + GATHER_CHUNK : P.count;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += BS) {
        switch (P.kind) {
            case 0:
                static_cast<int*>(P.dst)[e] = static_cast<const int*>(P.src)[e] + P.add;
                break;
            case 1:
                static_cast<double*>(P.dst)[e] = static_cast<const double*>(P.src)[e];
                break;
            case 2:
                static_cast<float*>(P.dst)[e] = static_cast<const float*>(P.src)[e];
                break;
            case 4:
                static_cast<float*>(P.dst)[e] = float(static_cast<const double*>(P.src)[e]);
                break;
            default: {
                int4 m = static_cast<const int4*>(P.src)[e];
                m.x += P.add;  // the first member always exists
                if (m.y >= 0) m.y += P.add;
                if (m.z >= 0) m.z += P.add;
                if (m.w >= 0) m.w += P.add;
                static_cast<int4*>(P.dst)[e] = m;
            }
        }
    }
}

int gather_chunk() { return GATHER_CHUNK; }

void launch_bspmv_dot(int nblk, const BatchTab& T, const int* rp, const int* ci, const double* v, const double* p,
                      double* q, const double* d, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_bspmv_dot, dim3(nblk), dim3(BS), 0, s, T, rp, EntAx<double>{v, ci, p}, q, d, part);
}

void launch_bresidual(int nblk, const BatchTab& T, const int* rp, const int* ci, const double* v, const double* x,
                      const double* b, double* r, const double* dinv, void* g, bool g32, double* part,
                      hipStream_t s) {
    if (g32)
        hipLaunchKernelGGL(k_bresidual<float>, dim3(nblk), dim3(BS), 0, s, T, rp, EntAx<double>{v, ci, x}, b, r, dinv,
                           static_cast<float*>(g), part);
    else
        hipLaunchKernelGGL(k_bresidual<double>, dim3(nblk), dim3(BS), 0, s, T, rp, EntAx<double>{v, ci, x}, b, r,
                           dinv, static_cast<double*>(g), part);
}

void launch_bdot(int nblk, const BatchTab& T, const double* a, const double* c, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_bdot, dim3(nblk), dim3(BS), 0, s, T, a, c, part);
}

void launch_bfinish(int nseg, const int* seg_blk, const int* mask, const double* part, double* S, int slot_k,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_bfinish, dim3(nseg), dim3(kWave), 0, s, seg_blk, mask, part, S, slot_k);
}

void launch_bcg_update(int nblk, const BatchTab& T, double* x, double* r, const double* p, const double* q,
                       const double* dinv, void* g, bool g32, double* part, const double* S, int slot_rho,
                       int slot_pq, hipStream_t s) {
    if (g32)
        hipLaunchKernelGGL(k_bcg_update<float>, dim3(nblk), dim3(BS), 0, s, T, x, r, p, q, dinv,
                           static_cast<float*>(g), part, S, slot_rho, slot_pq);
    else
        hipLaunchKernelGGL(k_bcg_update<double>, dim3(nblk), dim3(BS), 0, s, T, x, r, p, q, dinv,
                           static_cast<double*>(g), part, S, slot_rho, slot_pq);
}

void launch_bcg_dir(int nblk, const BatchTab& T, const double* z, const double* p, double* pn, const double* S,
                    int slot_new, int slot_old, hipStream_t s) {
    hipLaunchKernelGGL(k_bcg_dir, dim3(nblk), dim3(BS), 0, s, T, z, p, pn, S, slot_new, slot_old);
}

void launch_bbicg_s(int nblk, const BatchTab& T, const double* r, const double* v, double* sv, const double* S,
                    int slot_rho, int slot_rv, hipStream_t s) {
    hipLaunchKernelGGL(k_bbicg_s, dim3(nblk), dim3(BS), 0, s, T, r, v, sv, S, slot_rho, slot_rv);
}

void launch_bspmv_dot2(int nblk, const BatchTab& T, const int* rp, const int* ci, const double* v, const double* st,
                       double* t, const double* sv, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_bspmv_dot2, dim3(nblk), dim3(BS), 0, s, T, rp, EntAx<double>{v, ci, st}, t, sv, part);
}

void launch_bbicg_update(int nblk, const BatchTab& T, double* x, double* r, const double* pt, const double* st,
                         const double* sv, const double* t, const double* rb, double* part, const double* S,
                         int slot_rho, int slot_rv, int slot_tt, int slot_ts, hipStream_t s) {
    hipLaunchKernelGGL(k_bbicg_update, dim3(nblk), dim3(BS), 0, s, T, x, r, pt, st, sv, t, rb, part, S, slot_rho,
                       slot_rv, slot_tt, slot_ts);
}

void launch_bbicg_dir(int nblk, const BatchTab& T, const double* r, const double* p, const double* v, double* pn,
                      const double* S, int slot_rho, int slot_rv, int slot_tt, int slot_ts, int slot_rhonew,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_bbicg_dir, dim3(nblk), dim3(BS), 0, s, T, r, p, v, pn, S, slot_rho, slot_rv, slot_tt,
                       slot_ts, slot_rhonew);
}

void launch_bzero(int nblk, const BatchTab& T, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_bzero, dim3(nblk), dim3(BS), 0, s, T, x);
}

template <class T>
void launch_bdense(int nblk, const BDense<T>* dd, const int2* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_bdense<T>, dim3(nblk), dim3(512), 0, s, dd, tab);
}
template void launch_bdense<double>(int, const BDense<double>*, const int2*, hipStream_t);
template void launch_bdense<float>(int, const BDense<float>*, const int2*, hipStream_t);

void launch_gather(int nblk, const GatherPiece* pcs, const int2* tab, hipStream_t s) {
    if (nblk > 0) hipLaunchKernelGGL(k_gather, dim3(nblk), dim3(BS), 0, s, pcs, tab);
}

}  // namespace amg
