// Setup-phase kernels: CSR validation and D^{-1}, coarse numbering of a
// matching (Algorithm 2) by prefix sum, the 0/1 Galerkin product P^T A P,
// aggregate member lists, and the dense LU + inverse of the coarsest level.
// The matching itself is in k_hem.hip.
#include "amg_device.hpp"
#include "amg_internal.hpp"

namespace amg {

namespace {
constexpr int BS = 256;
inline int blocks_for(int64_t work, int bs = BS, int cap = 1 << 30) {
    int64_t b = (work + bs - 1) / bs;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}
}  // namespace

// ---------------------------------------------------------------------------
// Validation of level 0 and inverse diagonal (the Jacobi smoother's D^{-1}).
// Row bounds are checked before any entry of the row is read.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_validate(int n, int64_t nnz, const int* __restrict__ rp,
                                                 const int* __restrict__ ci, const double* __restrict__ v,
                                                 double* __restrict__ dinv, int* err) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const int b = rp[i], e = rp[i + 1];
    int bits = 0;
    if (i == 0 && b != 0) bits |= ERR_STRUCT;
    if (i == n - 1 && (int64_t)e != nnz) bits |= ERR_STRUCT;
    if (b < 0 || e < b || (int64_t)e > nnz) {
        atomicOr(err, bits | ERR_STRUCT);
        return;
    }
    double d = 0.0;
    bool has_d = false;
    int prev = -1;
    // no early exit, so the loads of several entries are in flight together
#pragma unroll 4
    for (int k = b; k < e; ++k) {
        const int c = ci[k];
        const double x = v[k];
        if (c < 0 || c >= n || c <= prev) bits |= ERR_STRUCT;
        prev = c;
        if (!isfinite(x)) bits |= ERR_NONFINITE;
        if (c == i) {
            has_d = true;
            d = x;
        }
    }
    if (!has_d || d == 0.0) bits |= ERR_DIAG;
    dinv[i] = has_d && d != 0.0 ? 1.0 / d : 0.0;
    if (bits) atomicOr(err, bits);
}

void launch_validate(int n, int64_t nnz, const int* rp, const int* ci, const double* v, double* dinv, int* err,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(blocks_for(n)), dim3(BS), 0, s, n, nnz, rp, ci, v, dinv, err);
}

__global__ __launch_bounds__(BS) void k_dinv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                             const double* __restrict__ v, double* __restrict__ dinv, int* err) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) d = v[k];
    if (d == 0.0 || !isfinite(d)) atomicOr(err, ERR_DIAG);
    dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
}

void launch_dinv(int n, const int* rp, const int* ci, const double* v, double* dinv, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_dinv, dim3(blocks_for(n)), dim3(BS), 0, s, n, rp, ci, v, dinv, err);
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum (three phases: tile sums, scan of tile sums, apply).
// ---------------------------------------------------------------------------
namespace {
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BS * SCAN_ITEMS;

__device__ __forceinline__ int block_excl_scan(int x, int& total) {
    __shared__ int sh[BS / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int inc = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) sh[wid] = inc;
    __syncthreads();
    int pre = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < BS / kWave; ++w) {
        const int t = sh[w];
        if (w < wid) pre += t;
        total += t;
    }
    __syncthreads();
    return pre + inc - x;
}
}  // namespace

__global__ __launch_bounds__(BS) void k_scan_tiles(const int* __restrict__ in, int n, int* __restrict__ tsum) {
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int s = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t)
        if (base + t < n) s += in[base + t];
    int total;
    block_excl_scan(s, total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(BS) void k_scan_top(int* tsum, int nt) {
    int carry = 0;
    for (int base = 0; base < nt; base += BS) {
        const int i = base + threadIdx.x;
        const int x = i < nt ? tsum[i] : 0;
        int total;
        const int ex = block_excl_scan(x, total);
        if (i < nt) tsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tsum[nt] = carry;
}

__global__ __launch_bounds__(BS) void k_scan_apply(const int* __restrict__ in, int n, const int* __restrict__ tsum,
                                                   int nt, int* __restrict__ out) {
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int loc[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        loc[t] = base + t < n ? in[base + t] : 0;
        s += loc[t];
    }
    int total;
    int ex = block_excl_scan(s, total) + tsum[blockIdx.x];
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        if (base + t < n) out[base + t] = ex;
        ex += loc[t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tsum[nt];
}

// The words a pass hands to the host, gathered by one small launch: the
// matching's 8 counters, the coarse row count, the coarse entry count and the
// error word.
__global__ void k_pass_words(int* __restrict__ out, const int* __restrict__ cnt, const int* __restrict__ ncp,
                             const int* __restrict__ nnzc, const int* __restrict__ err) {
    const int t = threadIdx.x;
    if (t < 8) out[t] = cnt[t];
    else if (t == 8) out[8] = *ncp;
    else if (t == 9) out[9] = *nnzc;
    else if (t == 10) out[10] = *err;
}

void launch_pass_words(int* out, const int* cnt, const int* ncp, const int* nnzc, const int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_pass_words, dim3(1), dim3(kWave), 0, s, out, cnt, ncp, nnzc, err);
}

size_t scan_tmp_ints(int n) { return (size_t)(n + SCAN_TILE - 1) / SCAN_TILE + 1; }

void launch_scan(const int* in, int n, int* out, int* tmp, hipStream_t s) {
    const int nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt > 0) hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(BS), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BS), 0, s, tmp, nt);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt > 0 ? nt : 1), dim3(BS), 0, s, in, n, tmp, nt, out);
}

// Algorithm 2 hands out coarse ids when the smaller vertex of a pair (or a
// singleton) is visited: ids are ranks of the aggregates' minimum vertex.
__global__ __launch_bounds__(BS) void k_leader_flags(int n, const int* __restrict__ mate, int* __restrict__ flag) {
    const int v = blockIdx.x * BS + threadIdx.x;
    if (v >= n) return;
    const int m = mate[v];
    flag[v] = (m < 0 || v < m) ? 1 : 0;
}

__global__ __launch_bounds__(BS) void k_assign_ids(int n, const int* __restrict__ mate, const int* __restrict__ ids,
                                                   int* __restrict__ agg, int* __restrict__ lead) {
    const int v = blockIdx.x * BS + threadIdx.x;
    if (v >= n) return;
    const int m = mate[v];
    if (m >= 0 && m < v) return;
    const int id = ids[v];
    agg[v] = id;
    if (m >= 0) agg[m] = id;
    lead[id] = v;
}

void launch_leader_flags(int n, const int* mate, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_leader_flags, dim3(blocks_for(n)), dim3(BS), 0, s, n, mate, flag);
}

void launch_assign_ids(int n, const int* mate, const int* ids, int* agg, int* lead, hipStream_t s) {
    hipLaunchKernelGGL(k_assign_ids, dim3(blocks_for(n)), dim3(BS), 0, s, n, mate, ids, agg, lead);
}

// ---------------------------------------------------------------------------
// Galerkin product of one matching pass, A_c = P^T B P with P_{i,agg(i)} = 1
// (Section 2.1.1).  Coarse row I has members lead[I] < mate[lead[I]]; entry
// (I,J) sums b_ij over the members in ascending order and, within a member,
// over its columns in ascending order, the first term initialising the sum.
// The fixed order makes the values bit-identical on every run.  A thread owns
// one coarse row and keeps its sorted (column, sum) list in its own LDS
// columns (a list this long indexed by position does not stay in registers);
// rows with more than RAP_CAP distinct columns go to a slower in-place path.
// ---------------------------------------------------------------------------
namespace {
constexpr int RAP_CAP = 32;
constexpr int RAP_BS = 128;
constexpr int RAP_WIN = 8;

// Sorted (column, sum) list of one thread: entry t at key[t * RAP_BS] (the
// threads of a block interleave, so a wave's accesses hit distinct banks).
// The first value added for a column initialises its sum; later values are
// added in call order.
template <bool WITH_VAL>
struct LdsAcc {
    int* key;
    double* val;
    int len;

    __device__ __forceinline__ int& k(int t) const { return key[t * RAP_BS]; }
    __device__ __forceinline__ double& x(int t) const { return val[t * RAP_BS]; }

    // false (list unchanged) when a new column does not fit
    __device__ __forceinline__ bool add(int J, double v) {
        int lo = 0, hi = len;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (k(mid) < J) lo = mid + 1;
            else hi = mid;
        }
        if (lo < len && k(lo) == J) {
            if (WITH_VAL) x(lo) += v;
            return true;
        }
        if (len == RAP_CAP) return false;
        for (int t = len; t > lo; --t) {
            k(t) = k(t - 1);
            if (WITH_VAL) x(t) = x(t - 1);
        }
        k(lo) = J;
        if (WITH_VAL) x(lo) = v;
        ++len;
        return true;
    }
};
}  // namespace

// Entries of a member row are taken in windows of RAP_WIN whose column and
// aggregate loads are issued together, then added in entry order.
template <bool WITH_VAL>
__device__ __forceinline__ bool rap_row(LdsAcc<WITH_VAL>& acc, int e0, int e1, const int* __restrict__ ci,
                                        const double* __restrict__ v, const int* __restrict__ agg) {
    for (int b = e0; b < e1; b += RAP_WIN) {
        int c[RAP_WIN], J[RAP_WIN];
        double x[RAP_WIN];
#pragma unroll
        for (int t = 0; t < RAP_WIN; ++t) c[t] = b + t < e1 ? ci[b + t] : -1;
#pragma unroll
        for (int t = 0; t < RAP_WIN; ++t) {
            J[t] = c[t] >= 0 ? agg[c[t]] : -1;
            x[t] = (WITH_VAL && c[t] >= 0) ? v[b + t] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < RAP_WIN; ++t)
            if (J[t] >= 0 && !acc.add(J[t], x[t])) return false;
    }
    return true;
}

// Rows are counted up to nmax (an upper bound of the coarse size *ncp); rows
// past the coarse size count zero, so a scan over nmax rows gives the offsets.
__global__ __launch_bounds__(RAP_BS) void k_rap_count(int nmax, const int* __restrict__ ncp,
                                                      const int* __restrict__ lead, const int* __restrict__ mate,
                                                      const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const int* __restrict__ agg, int* __restrict__ rowcnt,
                                                      int* __restrict__ ovf, int* novf) {
    const int I = blockIdx.x * RAP_BS + threadIdx.x;
    if (I >= nmax) return;
    if (I >= *ncp) {
        rowcnt[I] = 0;
        return;
    }
    __shared__ int skey[RAP_CAP * RAP_BS];
    const int m0 = lead[I];
    const int m1 = mate[m0];
    LdsAcc<false> acc{skey + threadIdx.x, nullptr, 0};
    bool ok = rap_row<false>(acc, rp[m0], rp[m0 + 1], ci, nullptr, agg);
    if (ok && m1 >= 0) ok = rap_row<false>(acc, rp[m1], rp[m1 + 1], ci, nullptr, agg);
    if (ok) {
        rowcnt[I] = acc.len;
    } else {
        rowcnt[I] = 0;
        ovf[atomicAdd(novf, 1)] = I;
    }
}

__global__ __launch_bounds__(RAP_BS) void k_rap_fill(int nc, const int* __restrict__ lead,
                                                     const int* __restrict__ mate, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const double* __restrict__ v,
                                                     const int* __restrict__ agg, const int* __restrict__ crp,
                                                     int* __restrict__ cci, double* __restrict__ cv) {
    const int I = blockIdx.x * RAP_BS + threadIdx.x;
    if (I >= nc) return;
    __shared__ int skey[RAP_CAP * RAP_BS];
    __shared__ double sval[RAP_CAP * RAP_BS];
    const int m0 = lead[I];
    const int m1 = mate[m0];
    LdsAcc<true> acc{skey + threadIdx.x, sval + threadIdx.x, 0};
    if (!rap_row<true>(acc, rp[m0], rp[m0 + 1], ci, v, agg)) return;  // overflow row: slow path
    if (m1 >= 0 && !rap_row<true>(acc, rp[m1], rp[m1 + 1], ci, v, agg)) return;
    const int o = crp[I];
    for (int t = 0; t < acc.len; ++t) {
        cci[o + t] = acc.k(t);
        cv[o + t] = acc.x(t);
    }
}

// Overflow rows (more than RAP_CAP distinct coarse columns): one wave per
// row.  The row's entries, in member-then-column order, are staged in LDS
// with their coarse columns; a stable rank (by column, then entry order)
// sorts them, and the first lane of each run of equal columns adds the run
// in entry order, so the sums are the same as on the fast path.  Rows longer
// than RAP_SLOW_CAP entries fall back to one lane working in place.
namespace {
constexpr int RAP_SLOW_CAP = 1024;

__device__ __forceinline__ int rap_entry(int k, int l0, int b0, int b1) { return k < l0 ? b0 + k : b1 + (k - l0); }

// serial fallback: distinct columns of a long row
__device__ int rap_count_serial(const int mm[2], const int* __restrict__ rp, const int* __restrict__ ci,
                                const int* __restrict__ agg) {
    int count = 0;
    for (int a = 0; a < 2; ++a) {
        if (mm[a] < 0) continue;
        for (int e = rp[mm[a]]; e < rp[mm[a] + 1]; ++e) {
            const int J = agg[ci[e]];
            bool seen = false;
            for (int b = 0; b <= a && !seen; ++b) {
                if (mm[b] < 0) continue;
                const int end = (b == a) ? e : rp[mm[b] + 1];
                for (int f = rp[mm[b]]; f < end; ++f)
                    if (agg[ci[f]] == J) {
                        seen = true;
                        break;
                    }
            }
            count += !seen;
        }
    }
    return count;
}

// serial fallback: sorted insertion into the row's own output segment
__device__ void rap_fill_serial(const int mm[2], const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, const int* __restrict__ agg, int o,
                                int* __restrict__ cci, double* __restrict__ cv) {
    int len = 0;
    for (int a = 0; a < 2; ++a) {
        if (mm[a] < 0) continue;
        for (int e = rp[mm[a]]; e < rp[mm[a] + 1]; ++e) {
            const int J = agg[ci[e]];
            int lo = 0, hi = len;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cci[o + mid] < J) lo = mid + 1;
                else hi = mid;
            }
            if (lo < len && cci[o + lo] == J) {
                cv[o + lo] += v[e];
            } else {
                for (int q = len; q > lo; --q) {
                    cci[o + q] = cci[o + q - 1];
                    cv[o + q] = cv[o + q - 1];
                }
                cci[o + lo] = J;
                cv[o + lo] = v[e];
                ++len;
            }
        }
    }
}
}  // namespace

template <bool FILL>
__global__ __launch_bounds__(kWave) void k_rap_slow(const int* __restrict__ ovf, const int* novf,
                                                    const int* __restrict__ lead, const int* __restrict__ mate,
                                                    const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const double* __restrict__ v, const int* __restrict__ agg,
                                                    int* __restrict__ rowcnt, const int* __restrict__ crp,
                                                    int* __restrict__ cci, double* __restrict__ cv) {
    __shared__ int key[RAP_SLOW_CAP], skey[RAP_SLOW_CAP];
    __shared__ double val[RAP_SLOW_CAP], sval[RAP_SLOW_CAP];
    __shared__ int s_cnt;
    const int lane = threadIdx.x;
    const int nrows = *novf;
    for (int t = blockIdx.x; t < nrows; t += gridDim.x) {
        const int I = ovf[t];
        const int m0 = lead[I];
        const int mm[2] = {m0, mate[m0]};
        const int b0 = rp[m0], l0 = rp[m0 + 1] - b0;
        const int b1 = mm[1] >= 0 ? rp[mm[1]] : 0, l1 = mm[1] >= 0 ? rp[mm[1] + 1] - b1 : 0;
        const int L = l0 + l1;
        if (L > RAP_SLOW_CAP) {
            if (lane == 0) {
                if (FILL) rap_fill_serial(mm, rp, ci, v, agg, crp[I], cci, cv);
                else rowcnt[I] = rap_count_serial(mm, rp, ci, agg);
            }
            continue;
        }
        if (lane == 0) s_cnt = 0;
        for (int k = lane; k < L; k += kWave) {
            const int e = rap_entry(k, l0, b0, b1);
            key[k] = agg[ci[e]];
            if (FILL) val[k] = v[e];
        }
        __syncthreads();
        int distinct = 0;
        for (int k = lane; k < L; k += kWave) {
            const int J = key[k];
            int less = 0, before = 0;
            for (int j = 0; j < L; ++j) {
                const int K = key[j];
                less += K < J;
                before += (K == J) & (j < k);
            }
            distinct += before == 0;
            if (FILL) {
                skey[less + before] = J;
                sval[less + before] = val[k];
            }
        }
        if (!FILL) {
            if (distinct) atomicAdd(&s_cnt, distinct);
            __syncthreads();
            if (lane == 0) rowcnt[I] = s_cnt;
            __syncthreads();
            continue;
        }
        __syncthreads();
        const int o = crp[I];
        for (int p = lane; p < L; p += kWave) {
            const int J = skey[p];
            if (p > 0 && skey[p - 1] == J) continue;  // not the start of a run
            int d = 0;  // runs before this one = distinct columns below J
            for (int q = 0; q < p; ++q) d += (q == 0 || skey[q - 1] != skey[q]);
            double sum = sval[p];
            for (int q = p + 1; q < L && skey[q] == J; ++q) sum += sval[q];
            cci[o + d] = J;
            cv[o + d] = sum;
        }
        __syncthreads();
    }
}

void launch_rap_count(int nmax, const int* ncp, const int* lead, const int* mate, const int* rp, const int* ci,
                      const int* agg, int* rowcnt, int* ovf, int* novf, hipStream_t s) {
    hipLaunchKernelGGL(k_rap_count, dim3(blocks_for(nmax, RAP_BS)), dim3(RAP_BS), 0, s, nmax, ncp, lead, mate, rp, ci,
                       agg, rowcnt, ovf, novf);
}

void launch_rap_count_slow(int nc, const int* ovf, const int* novf, const int* lead, const int* mate, const int* rp,
                           const int* ci, const int* agg, int* rowcnt, hipStream_t s) {
    hipLaunchKernelGGL(k_rap_slow<false>, dim3(blocks_for(nc, 1, 512)), dim3(kWave), 0, s, ovf, novf, lead, mate, rp,
                       ci, nullptr, agg, rowcnt, nullptr, nullptr, nullptr);
}

void launch_rap_fill(int nc, const int* lead, const int* mate, const int* rp, const int* ci, const double* v,
                     const int* agg, const int* crp, int* cci, double* cv, hipStream_t s) {
    hipLaunchKernelGGL(k_rap_fill, dim3(blocks_for(nc, RAP_BS)), dim3(RAP_BS), 0, s, nc, lead, mate, rp, ci, v, agg,
                       crp, cci, cv);
}

void launch_rap_fill_slow(int nc, const int* ovf, const int* novf, const int* lead, const int* mate, const int* rp,
                          const int* ci, const double* v, const int* agg, const int* crp, int* cci, double* cv,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_rap_slow<true>, dim3(blocks_for(nc, 1, 512)), dim3(kWave), 0, s, ovf, novf, lead, mate, rp,
                       ci, v, agg, nullptr, crp, cci, cv);
}

// ---------------------------------------------------------------------------
// Level maps: composed aggregate map and member lists of the coarse rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_compose(int n, const int* __restrict__ a1, const int* __restrict__ a2,
                                                int* __restrict__ out) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < n) out[i] = a2[a1[i]];
}

void launch_compose(int n, const int* agg1, const int* agg2, int* out, hipStream_t s) {
    hipLaunchKernelGGL(k_compose, dim3(blocks_for(n)), dim3(BS), 0, s, n, agg1, agg2, out);
}

__device__ __forceinline__ void cswap(int& a, int& b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// lead2 == nullptr: a level made of a single pass (members of pass-1 pairs).
__global__ __launch_bounds__(BS) void k_members(int nc, const int* __restrict__ lead2, const int* __restrict__ mate2,
                                                const int* __restrict__ lead1, const int* __restrict__ mate1,
                                                int4* __restrict__ mem) {
    const int J = blockIdx.x * BS + threadIdx.x;
    if (J >= nc) return;
    constexpr int BIG = 0x7fffffff;
    int m[4] = {BIG, BIG, BIG, BIG};
    if (lead2 == nullptr) {
        const int a = lead1[J], b = mate1[a];
        m[0] = a;
        m[1] = b < 0 ? BIG : b;
    } else {
        const int I1 = lead2[J], I2 = mate2[I1];
        const int a1 = lead1[I1], b1 = mate1[a1];
        m[0] = a1;
        m[1] = b1 < 0 ? BIG : b1;
        if (I2 >= 0) {
            const int a2 = lead1[I2], b2 = mate1[a2];
            m[2] = a2;
            m[3] = b2 < 0 ? BIG : b2;
        }
    }
    cswap(m[0], m[1]);
    cswap(m[2], m[3]);
    cswap(m[0], m[2]);
    cswap(m[1], m[3]);
    cswap(m[1], m[2]);
    int4 o;
    o.x = m[0] == BIG ? -1 : m[0];
    o.y = m[1] == BIG ? -1 : m[1];
    o.z = m[2] == BIG ? -1 : m[2];
    o.w = m[3] == BIG ? -1 : m[3];
    mem[J] = o;
}

void launch_members(int nc, const int* lead2, const int* mate2, const int* lead1, const int* mate1, int4* mem,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_members, dim3(blocks_for(nc)), dim3(BS), 0, s, nc, lead2, mate2, lead1, mate1, mem);
}

// ---------------------------------------------------------------------------
// Coarsest level (Section 2, coarse level solver): dense partial-pivot LU,
// largest |pivot| with the lowest row on ties, then the explicit inverse so
// that each V-cycle applies the exact coarse solve as one dense product
// (n <= 1024).
// ---------------------------------------------------------------------------
// Row i of the block: entries rp[i]..rp[i+1]-1 of ci/v, columns shifted by
// col_add (a diagonal block of a larger matrix starts at column -col_add).
__global__ __launch_bounds__(BS) void k_dense_assemble(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v, double* __restrict__ a,
                                                       int col_add) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int c = ci[k] + col_add;
        if (c >= 0 && c < n) a[(size_t)i * n + c] = v[k];
    }
}

void launch_dense_assemble(int n, const int* rp, const int* ci, const double* v, double* a, hipStream_t s,
                           int col_add) {
    hipLaunchKernelGGL(k_dense_assemble, dim3(blocks_for(n)), dim3(BS), 0, s, n, rp, ci, v, a, col_add);
}

// Start of each system inside a concatenated level and its coarse level:
// out[2j] = agg[off[j]] (first coarse row), out[2j+1] = crp[out[2j]].
__global__ __launch_bounds__(BS) void k_seg_starts(int m, const int* __restrict__ off, const int* __restrict__ agg,
                                                   const int* __restrict__ crp, int* __restrict__ out) {
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= m) return;
    const int c = agg[off[j]];
    out[2 * j] = c;
    out[2 * j + 1] = crp[c];
}

void launch_seg_starts(int m, const int* off, const int* agg, const int* crp, int* out, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_starts, dim3(blocks_for(m)), dim3(BS), 0, s, m, off, agg, crp, out);
}

namespace {
constexpr int LU_BS = 1024;
constexpr int INV_BS = 256;

// Block-wide argmax of (|value|, lowest index on ties) over LU_BS threads.
__device__ __forceinline__ void lu_argmax(double& v, int& i, double* sv, int* si) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(i, off);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        sv[wid] = v;
        si[wid] = i;
    }
    __syncthreads();
    v = sv[0];
    i = si[0];
    for (int w = 1; w < LU_BS / kWave; ++w)
        if (sv[w] > v || (sv[w] == v && si[w] < i)) {
            v = sv[w];
            i = si[w];
        }
}
}  // namespace

// Blocked right-looking LU with partial pivoting in place (row-major a, unit
// lower L below the diagonal; P A = L U with perm[i] = original row of
// position i).  Panels of NB columns: k_lu_panel factors the panel's rows
// k0.. in LDS (pivot = largest |value|, lowest row on ties), then k_lu_rest
// applies the panel's interchanges to every other column and, right of the
// panel, forms U12 = L11^{-1} A12 and A22 -= L21 U12.  Each entry receives its
// updates in the order of the unblocked algorithm, whatever NB.  The panel of
// the remaining m = n - k0 rows must fit LDS: NB = 16 up to 1024 rows, 8 up
// to 2048, 4 up to 4096 (n <= 4096).
constexpr int LU_COLS = 64;        // columns per block of k_lu_rest
constexpr int LU_LDS_DOUBLES = 18432;  // 144 KiB of panel

template <int NB>
constexpr int lu_ldp() { return NB >= 8 ? NB + 1 : NB; }  // padded LDS row of the panel

template <int NB>
__global__ __launch_bounds__(LU_BS) void k_lu_panel(int n, int k0, double* __restrict__ a, int* __restrict__ perm,
                                                    int* __restrict__ piv, int* err) {
    constexpr int LDP = lu_ldp<NB>();
    __shared__ double P[LU_LDS_DOUBLES];
    __shared__ double sv[LU_BS / kWave];
    __shared__ int si[LU_BS / kWave];
    if (*err & ERR_SINGULAR) return;  // an earlier panel failed (uniform)
    const int tid = threadIdx.x;
    const int kb = min(NB, n - k0), m = n - k0;
    if (k0 == 0)
        for (int i = tid; i < n; i += LU_BS) perm[i] = i;
    if (tid < kb) piv[k0 + tid] = k0 + tid;  // valid even if this panel fails
    for (int t = tid; t < m * NB; t += LU_BS) {
        const int r = t / NB, c = t % NB;
        P[r * LDP + c] = c < kb ? a[(size_t)(k0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < kb; ++c) {
        double best = -1.0;
        int bi = m;
        for (int r = c + tid; r < m; r += LU_BS) {
            const double v = fabs(P[r * LDP + c]);
            if (v > best) {  // rows ascend per thread: strict '>' keeps the lowest
                best = v;
                bi = r;
            }
        }
        lu_argmax(best, bi, sv, si);
        if (!(best > 0.0) || !isfinite(best)) {  // uniform across the block
            if (tid == 0) atomicOr(err, ERR_SINGULAR);
            return;
        }
        if (bi != c && tid < NB) {
            const double t = P[c * LDP + tid];
            P[c * LDP + tid] = P[bi * LDP + tid];
            P[bi * LDP + tid] = t;
        }
        if (tid == 0) piv[k0 + c] = k0 + bi;
        __syncthreads();
        const double d = P[c * LDP + c];
        for (int r = c + 1 + tid; r < m; r += LU_BS) {
            const double l = P[r * LDP + c] / d;
            P[r * LDP + c] = l;
            for (int j = c + 1; j < kb; ++j) P[r * LDP + j] -= l * P[c * LDP + j];
        }
        __syncthreads();
    }
    for (int t = tid; t < m * NB; t += LU_BS) {
        const int r = t / NB, c = t % NB;
        if (c < kb) a[(size_t)(k0 + r) * n + k0 + c] = P[r * LDP + c];
    }
    if (tid == 0)
        for (int c = 0; c < kb; ++c) {
            const int p = piv[k0 + c];
            if (p != k0 + c) {
                const int t = perm[k0 + c];
                perm[k0 + c] = perm[p];
                perm[p] = t;
            }
        }
}

// A block owns LU_COLS columns; 4 groups of 64 threads share its rows.
template <int NB>
__global__ __launch_bounds__(256) void k_lu_rest(int n, int k0, double* __restrict__ a, const int* __restrict__ piv,
                                                 const int* err) {
    __shared__ double L11[NB][NB];
    __shared__ double U[NB][LU_COLS];
    if (*err & ERR_SINGULAR) return;  // uniform
    const int kb = min(NB, n - k0);
    const int cl = threadIdx.x % LU_COLS, rg = threadIdx.x / LU_COLS;
    const int j = blockIdx.x * LU_COLS + cl;
    const bool mine = j < n && (j < k0 || j >= k0 + kb);
    const bool right = mine && j >= k0 + kb;
    for (int t = threadIdx.x; t < kb * kb; t += 256) L11[t / kb][t % kb] = a[(size_t)(k0 + t / kb) * n + k0 + t % kb];
    if (rg == 0 && mine)
        for (int c = 0; c < kb; ++c) {
            const int p = piv[k0 + c];
            if (p > k0 + c && p < n) {
                const double t = a[(size_t)(k0 + c) * n + j];
                a[(size_t)(k0 + c) * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        }
    __syncthreads();
    if (rg == 0 && right)
        for (int i = 0; i < kb; ++i) {
            double u = a[(size_t)(k0 + i) * n + j];
            for (int q = 0; q < i; ++q) u -= L11[i][q] * U[q][cl];
            U[i][cl] = u;
            a[(size_t)(k0 + i) * n + j] = u;
        }
    __syncthreads();
    if (right)
        for (int r = k0 + kb + rg; r < n; r += 4) {
            const double* l = a + (size_t)r * n + k0;
            double s = a[(size_t)r * n + j];
            for (int q = 0; q < kb; ++q) s -= l[q] * U[q][cl];
            a[(size_t)r * n + j] = s;
        }
}

// Columns of A^{-1} = U^{-1} L^{-1} P, INV_COLS per block, held in LDS as
// x[i * INV_COLS + c].  Both substitutions go by blocks of 16 rows: the
// block's rows first subtract the contributions of the rows already solved
// (one dot per row and column, all threads), then lane c of the first wave
// finishes column c through the 16x16 diagonal block kept in LDS.  Writes
// the inverse column-major: ainv_t[c * n + i] = (A^{-1})_{ic}.
template <int INV_COLS, int XCAP>
__global__ __launch_bounds__(INV_BS) void k_dense_inverse(int n, const double* __restrict__ lu,
                                                          const int* __restrict__ perm, double* __restrict__ ainv_t) {
    constexpr int RB = 16;
    __shared__ double x[XCAP];  // n * INV_COLS <= XCAP
    __shared__ double D[RB][RB + 1];
    const int c0 = blockIdx.x * INV_COLS;
    const int tid = threadIdx.x;
    for (int t = tid; t < n * INV_COLS; t += INV_BS) {
        const int i = t / INV_COLS, cc = t % INV_COLS;
        x[t] = perm[i] == c0 + cc ? 1.0 : 0.0;
    }
    __syncthreads();
    const int oi = tid / INV_COLS, oc = tid % INV_COLS;  // (row in block, column) of this thread's output
    for (int b0 = 0; b0 < n; b0 += RB) {  // unit lower
        const int bs = min(RB, n - b0);
        if (oi < bs) {
            const double* l = lu + (size_t)(b0 + oi) * n;
            double s = 0.0;
            for (int k = 0; k < b0; ++k) s += l[k] * x[k * INV_COLS + oc];
            x[(b0 + oi) * INV_COLS + oc] -= s;
        }
        for (int t = tid; t < bs * bs; t += INV_BS) D[t / bs][t % bs] = lu[(size_t)(b0 + t / bs) * n + b0 + t % bs];
        __syncthreads();
        if (tid < INV_COLS)
            for (int i = 1; i < bs; ++i) {
                double s = 0.0;
                for (int k = 0; k < i; ++k) s += D[i][k] * x[(b0 + k) * INV_COLS + tid];
                x[(b0 + i) * INV_COLS + tid] -= s;
            }
        __syncthreads();
    }
    for (int b0 = ((n - 1) / RB) * RB; b0 >= 0; b0 -= RB) {  // upper
        const int bs = min(RB, n - b0);
        if (oi < bs) {
            const double* u = lu + (size_t)(b0 + oi) * n;
            double s = 0.0;
            for (int k = b0 + bs; k < n; ++k) s += u[k] * x[k * INV_COLS + oc];
            x[(b0 + oi) * INV_COLS + oc] -= s;
        }
        for (int t = tid; t < bs * bs; t += INV_BS) D[t / bs][t % bs] = lu[(size_t)(b0 + t / bs) * n + b0 + t % bs];
        __syncthreads();
        if (tid < INV_COLS)
            for (int i = bs - 1; i >= 0; --i) {
                double s = 0.0;
                for (int k = i + 1; k < bs; ++k) s += D[i][k] * x[(b0 + k) * INV_COLS + tid];
                x[(b0 + i) * INV_COLS + tid] = (x[(b0 + i) * INV_COLS + tid] - s) / D[i][i];
            }
        __syncthreads();
    }
    for (int t = tid; t < n * INV_COLS; t += INV_BS) {
        const int cc = t / n, i = t % n;
        if (c0 + cc < n) ainv_t[(size_t)(c0 + cc) * n + i] = x[i * INV_COLS + cc];
    }
}

// piv: int32[2n] scratch (permutation, then the panels' pivot rows).  n <= 4096.
void launch_dense_lu_inverse(int n, double* a, int* piv, double* ainv_t, int* err, hipStream_t s) {
    int* perm = piv;
    int* steps = piv + n;
    const dim3 rest_grid((n + LU_COLS - 1) / LU_COLS);
#define LU_STEP(NB)                                                                                           \
    hipLaunchKernelGGL(k_lu_panel<NB>, dim3(1), dim3(LU_BS), 0, s, n, k0, a, perm, steps, err);             \
    hipLaunchKernelGGL(k_lu_rest<NB>, rest_grid, dim3(256), 0, s, n, k0, a, steps, (const int*)err);        \
    k0 += NB
    static_assert(4096 * lu_ldp<4>() <= LU_LDS_DOUBLES && 2048 * lu_ldp<8>() <= LU_LDS_DOUBLES &&
                      1024 * lu_ldp<16>() <= LU_LDS_DOUBLES, "panel LDS");
    for (int k0 = 0; k0 < n;) {
        const int m = n - k0;
        if (m > 2048) {
            LU_STEP(4);
        } else if (m > 1024) {
            LU_STEP(8);
        } else {
            LU_STEP(16);
        }
    }
#undef LU_STEP
    if (n <= 512)
        hipLaunchKernelGGL((k_dense_inverse<16, 8192>), dim3((n + 15) / 16), dim3(INV_BS), 0, s, n, a, perm, ainv_t);
    else if (n <= 1024)
        hipLaunchKernelGGL((k_dense_inverse<8, 8192>), dim3((n + 7) / 8), dim3(INV_BS), 0, s, n, a, perm, ainv_t);
    else if (n <= 2048)
        hipLaunchKernelGGL((k_dense_inverse<8, 16384>), dim3((n + 7) / 8), dim3(INV_BS), 0, s, n, a, perm, ainv_t);
    else
        hipLaunchKernelGGL((k_dense_inverse<4, 16384>), dim3((n + 3) / 4), dim3(INV_BS), 0, s, n, a, perm, ainv_t);
}

}  // namespace amg
