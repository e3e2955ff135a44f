// Setup-phase kernels: CSR validation and D^{-1}, node-based heavy edge
// matching (Section 2.1.1, Algorithm 2) as rounds of locally dominant edges,
// coarse numbering by prefix sum, the 0/1 Galerkin product P^T A P, aggregate
// member lists, and the dense LU + inverse of the coarsest level.
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
    for (int k = b; k < e; ++k) {
        const int c = ci[k];
        if (c < 0 || c >= n || c <= prev) {
            bits |= ERR_STRUCT;
            break;
        }
        prev = c;
        const double x = v[k];
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
// Heavy edge matching.
//
// Visiting vertices in ascending order (Algorithm 2) is the greedy matching
// over edges {u < w} (a_uw stored in row u, non-zero) in increasing key
// (u, -|a_uw|, w).  Greedy matching in a strict edge order equals repeated
// rounds of locally dominant edges: each undecided vertex points along its
// smallest-key edge to an undecided neighbour, mutual pointers match, and a
// vertex with no undecided neighbour is a singleton.  Under this key a vertex
// points to its smallest undecided lower neighbour if it has one, otherwise
// to its heaviest undecided higher neighbour (lowest index on ties).  Only a
// vertex without undecided lower neighbours ("ready") can start a match, so
// each round scans a worklist of ready vertices, and a per-vertex count of
// undecided lower neighbours adds vertices to the next list as they become
// ready.  Decisions carry the round number: a vertex counts as undecided in
// round r while its stamp is >= r, so all reads in a round see the state at
// the start of the round whatever the interleaving.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_col(const int* __restrict__ ci, int lo, int hi, int c) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int x = ci[mid];
        if (x == c) return mid;
        if (x < c) lo = mid + 1;
        else hi = mid;
    }
    return -1;
}

// counters: cnt[0..2] worklist sizes (ring of 3), cnt[5] sum over rows of
// (#upper - #lower) entries, cnt[6] the number of rounds that had work,
// cnt[7] set when the single-workgroup pass hit its round limit.
template <int SIDE>
__global__ __launch_bounds__(BS) void k_hem_init(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ v, uint8_t* __restrict__ lowok,
                                                 HemRecT<SIDE>* __restrict__ rec, int* __restrict__ lcnt,
                                                 int* __restrict__ dec, int* __restrict__ mate,
                                                 int* __restrict__ wl0, int* cnt, int* err) {
    const int y = blockIdx.x * BS + threadIdx.x;
    if (y >= n) return;
    dec[y] = kUndecided;
    mate[y] = -1;
    int c = 0, nlow = 0, nup = 0, bad = 0, nh = 0, nl = 0;
    bool ovf = false;
    int hj[SIDE], lx[SIDE];
    double hw[SIDE];
#pragma unroll
    for (int t = 0; t < SIDE; ++t) {
        hj[t] = -1;
        lx[t] = -1;
        hw[t] = 0.0;
    }
    for (int k = rp[y]; k < rp[y + 1]; ++k) {
        const int u = ci[k];
        uint8_t ok = 0;
        if (u < y) {
            ++nlow;
            const int pos = find_col(ci, rp[u], rp[u + 1], y);
            if (pos < 0) bad = 1;
            else if (v[pos] != 0.0) ok = 1;
            if (ok) {  // lower edge-neighbour, columns arrive ascending
                if (nl < SIDE) {
#pragma unroll
                    for (int t = 0; t < SIDE; ++t)
                        if (t == nl) lx[t] = u;
                    ++nl;
                } else {
                    ovf = true;
                }
            }
        } else if (u > y) {
            ++nup;
            const double a = v[k];
            if (a != 0.0) {  // higher neighbour: keep sorted by |a| descending, column ascending
                if (nh < SIDE) {
                    const double w = fabs(a);
                    int pos = 0;
#pragma unroll
                    for (int t = 0; t < SIDE; ++t)
                        if (t < nh && hw[t] >= w) pos = t + 1;
#pragma unroll
                    for (int t = SIDE - 1; t > 0; --t)
                        if (t > pos && t <= nh) {
                            hw[t] = hw[t - 1];
                            hj[t] = hj[t - 1];
                        }
#pragma unroll
                    for (int t = 0; t < SIDE; ++t)
                        if (t == pos) {
                            hw[t] = w;
                            hj[t] = u;
                        }
                    ++nh;
                } else {
                    ovf = true;
                }
            }
        }
        lowok[k] = ok;
        c += ok;
    }
    HemRecT<SIDE> R;
    R.hdr = nh | (nl << 8) | (ovf ? kRecOverflow : 0);
#pragma unroll
    for (int t = 0; t < SIDE; ++t) {
        R.h[t] = hj[t];
        R.l[t] = lx[t];
    }
    R.pad = 0;
    rec[y] = R;
    lcnt[y] = c;
    if (bad) atomicOr(err, ERR_NONSYM);
    if (nup != nlow) atomicAdd(&cnt[5], nup - nlow);
    if (c == 0) wl0[atomicAdd(&cnt[0], 1)] = y;
}

namespace {
struct HemState {
    const int* __restrict__ rp;
    const int* __restrict__ ci;
    const double* __restrict__ v;
    const uint8_t* __restrict__ lowok;
    const void* __restrict__ rec;  // HemRecT<SIDE>[n]
    int* dec;
    int* mate;
    int* lcnt;
};

// Appends to the next worklist through a block-local LDS list; entries that
// do not fit go straight to global memory.
struct Appender {
    int* s_list;
    int* s_cnt;
    int cap;
    int* gout;
    int* gcnt;
    __device__ __forceinline__ void push(int x) const {
        const int p = atomicAdd(s_cnt, 1);
        if (p < cap) s_list[p] = x;
        else gout[atomicAdd(gcnt, 1)] = x;
    }
};

constexpr int HEM_WIN = 8;  // row entries whose loads are issued together

template <int SCOPE>
__device__ __forceinline__ int dec_counter(int* p) {
    return __hip_atomic_fetch_add(p, -1, __ATOMIC_RELAXED, SCOPE);
}

// x has just been decided: its higher neighbours lose one undecided lower
// neighbour; those that reach zero are ready for the next round.  The
// counter updates of a window are issued before any result is used.
template <int SCOPE>
__device__ __forceinline__ void hem_release(const HemState& S, int x, const Appender& A) {
    const int e0 = S.rp[x], e1 = S.rp[x + 1];
    for (int b = e0; b < e1; b += HEM_WIN) {
        int ys[HEM_WIN], old[HEM_WIN];
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t) {
            const int e = b + t;
            ys[t] = -1;
            if (e < e1) {
                const int y = S.ci[e];
                if (y > x && S.v[e] != 0.0) ys[t] = y;
            }
        }
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t) old[t] = ys[t] >= 0 ? dec_counter<SCOPE>(&S.lcnt[ys[t]]) : 0;
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t)
            if (ys[t] >= 0 && old[t] == 1) A.push(ys[t]);
    }
}

// Heaviest undecided higher neighbour of u (lowest index on ties), or -1.
__device__ __forceinline__ int hem_best(const HemState& S, int r, int u, int e0, int e1) {
    int best = -1;
    double k = -1.0;
    for (int b = e0; b < e1; b += HEM_WIN) {
        int js[HEM_WIN];
        double ws[HEM_WIN];
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t) {
            const int e = b + t;
            js[t] = -1;
            ws[t] = 0.0;
            if (e < e1) {
                const int j = S.ci[e];
                const double a = S.v[e];
                if (j > u && a != 0.0) {
                    js[t] = j;
                    ws[t] = fabs(a);
                }
            }
        }
        bool und[HEM_WIN];
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t) und[t] = js[t] >= 0 && S.dec[js[t]] >= r;
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t)
            if (und[t] && ws[t] > k) {  // ascending column order: strict '>' keeps the lowest index
                k = ws[t];
                best = js[t];
            }
    }
    return best;
}

// Smallest undecided lower neighbour of w (over edges (x, w) stored non-zero
// in row x), or -1.
__device__ __forceinline__ int hem_back(const HemState& S, int r, int w) {
    const int e0 = S.rp[w], e1 = S.rp[w + 1];
    for (int b = e0; b < e1; b += HEM_WIN) {
        int xs[HEM_WIN];
        bool stop = false;
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t) {
            const int e = b + t;
            xs[t] = -1;
            if (e < e1) {
                const int x = S.ci[e];
                if (x >= w) stop = true;
                else if (S.lowok[e]) xs[t] = x;
            }
        }
        bool und[HEM_WIN];
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t) und[t] = xs[t] >= 0 && S.dec[xs[t]] >= r;
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t)
            if (und[t]) return xs[t];  // columns ascend: the first is the smallest
        if (stop) break;
    }
    return -1;
}

// Counter updates for the higher neighbours listed in a record, all issued
// before any result is used.
template <int SCOPE, int SIDE>
__device__ __forceinline__ void rec_release(const HemState& S, const HemRecT<SIDE>& R, int x, const Appender& A) {
    if (R.hdr & kRecOverflow) {
        hem_release<SCOPE>(S, x, A);
        return;
    }
    const int nh = R.hdr & 255;
    int old[SIDE];
#pragma unroll
    for (int t = 0; t < SIDE; ++t) old[t] = t < nh ? dec_counter<SCOPE>(&S.lcnt[R.h[t]]) : 0;
#pragma unroll
    for (int t = 0; t < SIDE; ++t)
        if (t < nh && old[t] == 1) A.push(R.h[t]);
}

// Round r for a ready vertex u.  A vertex counts as undecided while its stamp
// is >= r, so every read sees the state at the start of the round.  Records
// list u's higher neighbours in preference order (heaviest first, lowest
// index on ties) and the target's lower edge-neighbours in ascending order, so
// "first undecided entry" is the pointer of either side.
template <int SCOPE, int SIDE>
__device__ __forceinline__ void hem_visit(const HemState& S, int r, int u, const Appender& A) {
    const HemRecT<SIDE>* __restrict__ recs = static_cast<const HemRecT<SIDE>*>(S.rec);
    const HemRecT<SIDE> R = recs[u];
    const int du = S.dec[u];
    if (du < r) return;  // decided earlier (as a match target): stale entry
    int best = -1;
    if (R.hdr & kRecOverflow) {
        best = hem_best(S, r, u, S.rp[u], S.rp[u + 1]);
    } else {
        const int nh = R.hdr & 255;
        int d[SIDE];
#pragma unroll
        for (int t = 0; t < SIDE; ++t) d[t] = t < nh ? S.dec[R.h[t]] : -1;
#pragma unroll
        for (int t = SIDE - 1; t >= 0; --t)
            if (t < nh && d[t] >= r) best = R.h[t];
    }
    if (best < 0) {  // no undecided neighbour: unaggregated singleton
        S.dec[u] = r;
        S.mate[u] = -1;
        rec_release<SCOPE, SIDE>(S, R, u, A);
        return;
    }
    const HemRecT<SIDE> B = recs[best];
    int back = -1;
    if (B.hdr & kRecOverflow) {
        back = hem_back(S, r, best);
    } else {
        const int nl = (B.hdr >> 8) & 255;
        int d[SIDE];
#pragma unroll
        for (int t = 0; t < SIDE; ++t) d[t] = t < nl ? S.dec[B.l[t]] : -1;
#pragma unroll
        for (int t = SIDE - 1; t >= 0; --t)
            if (t < nl && d[t] >= r) back = B.l[t];
    }
    if (back == u) {  // best points back: mutual, matched
        S.dec[u] = r;
        S.dec[best] = r;
        S.mate[u] = best;
        S.mate[best] = u;
        rec_release<SCOPE, SIDE>(S, R, u, A);
        rec_release<SCOPE, SIDE>(S, B, best, A);
    } else {
        A.push(u);  // still ready, retry next round
    }
}

constexpr int HEM_BS = 512;
constexpr int HEM_LCAP = 4096;
constexpr int HEM_BS1 = 1024;
constexpr int HEM_LCAP1 = 8192;
}  // namespace

// One round over the worklist; the decided vertices' neighbours that become
// ready, and the ready vertices that failed, form the next list.
template <int SIDE>
__global__ __launch_bounds__(HEM_BS) void k_hem_round(int r, HemState S, const int* __restrict__ win,
                                                  int* __restrict__ wout, int* cnt, int slot_in, int slot_out,
                                                  int zero_w) {
    __shared__ int s_list[HEM_LCAP];
    __shared__ int s_cnt, s_base;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        if (blockIdx.x == 0) cnt[zero_w] = 0;
    }
    __syncthreads();
    const int m = cnt[slot_in];
    if (m > 0 && blockIdx.x == 0 && threadIdx.x == 0) cnt[6] = r + 1;  // rounds with work
    const Appender A{s_list, &s_cnt, HEM_LCAP, wout, &cnt[slot_out]};
    for (int idx = blockIdx.x * HEM_BS + threadIdx.x; idx < m; idx += gridDim.x * HEM_BS)
        hem_visit<__HIP_MEMORY_SCOPE_AGENT, SIDE>(S, r, win[idx], A);
    __syncthreads();
    const int k = min(s_cnt, HEM_LCAP);
    if (threadIdx.x == 0 && k > 0) s_base = atomicAdd(&cnt[slot_out], k);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += HEM_BS) wout[s_base + i] = s_list[i];
}

// Small matrices: one workgroup runs every round, separated by barriers.
// Each round decides at least the smallest undecided vertex, so n + 1 rounds
// always suffice; the bound only guards against invalid input.
template <int SIDE>
__global__ __launch_bounds__(HEM_BS1) void k_hem_all(int n, HemState S, int* wl0, int* wl1, int* cnt) {
    __shared__ int s_list[HEM_LCAP1];
    __shared__ int s_cnt, s_next, s_m;
    if (threadIdx.x == 0) s_m = cnt[0];
    __syncthreads();
    int* win = wl0;
    int* wout = wl1;
    int r = 0;
    for (; r <= n + 1; ++r) {
        const int m = s_m;
        if (m == 0) break;
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_next = 0;
        }
        __syncthreads();
        const Appender A{s_list, &s_cnt, HEM_LCAP1, wout, &s_next};
        for (int idx = threadIdx.x; idx < m; idx += HEM_BS1) hem_visit<__HIP_MEMORY_SCOPE_WORKGROUP, SIDE>(S, r, win[idx], A);
        __syncthreads();
        const int k = min(s_cnt, HEM_LCAP1);
        const int base = s_next;
        for (int i = threadIdx.x; i < k; i += HEM_BS1) wout[base + i] = s_list[i];
        __syncthreads();
        if (threadIdx.x == 0) s_m = base + k;
        int* t = win;
        win = wout;
        wout = t;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[6] = r;
        if (s_m != 0) cnt[7] = 1;
    }
}

#define AMG_HEM_SIDE(side, CALL) \
    switch (side) {                \
        case 7: CALL(7); break;    \
        case 15: CALL(15); break;  \
        default: CALL(31); break;  \
    }

void launch_hem_init(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
#define CALL(SD)                                                                                               \
    hipLaunchKernelGGL(k_hem_init<SD>, dim3(blocks_for(n)), dim3(BS), 0, s, n, rp, ci, v, w.lowok,              \
                       static_cast<HemRecT<SD>*>(w.rec), w.lcnt, w.dec, w.mate, w.wl[0], w.cnt, w.err)
    AMG_HEM_SIDE(w.side, CALL)
#undef CALL
}

int hem_next_count_slot(int round) { return round % 3; }

void launch_hem_round(int r, int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
    const int g = blocks_for(n, HEM_BS, 96);
    const HemState S{rp, ci, v, w.lowok, w.rec, w.dec, w.mate, w.lcnt};
#define CALL(SD)                                                                                          \
    hipLaunchKernelGGL(k_hem_round<SD>, dim3(g), dim3(HEM_BS), 0, s, r, S, w.wl[r & 1], w.wl[(r + 1) & 1], \
                       w.cnt, r % 3, (r + 1) % 3, (r + 2) % 3)
    AMG_HEM_SIDE(w.side, CALL)
#undef CALL
}

void launch_hem_all(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
    const HemState S{rp, ci, v, w.lowok, w.rec, w.dec, w.mate, w.lcnt};
#define CALL(SD) \
    hipLaunchKernelGGL(k_hem_all<SD>, dim3(1), dim3(HEM_BS1), 0, s, n, S, w.wl[0], w.wl[1], w.cnt)
    AMG_HEM_SIDE(w.side, CALL)
#undef CALL
}
#undef AMG_HEM_SIDE

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
// one coarse row and keeps its sorted (column, sum) list in registers; rows
// with more than RAP_CAP distinct columns go to a slower in-place path.
// ---------------------------------------------------------------------------
namespace {
constexpr int RAP_CAP = 32;
constexpr int RAP_BS = 128;
constexpr int RAP_WIN = 8;
}

// Entries of a member row are taken in windows of RAP_WIN whose column and
// aggregate loads are issued together, then added in entry order.
template <bool WITH_VAL>
__device__ __forceinline__ bool rap_row(SortedAcc<RAP_CAP>& acc, int e0, int e1, const int* __restrict__ ci,
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
            if (J[t] >= 0 && !acc.template add<WITH_VAL>(J[t], x[t])) return false;
    }
    return true;
}

__global__ __launch_bounds__(RAP_BS) void k_rap_count(int nc, const int* __restrict__ lead,
                                                      const int* __restrict__ mate, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const int* __restrict__ agg,
                                                      int* __restrict__ rowcnt, int* __restrict__ ovf, int* novf) {
    const int I = blockIdx.x * RAP_BS + threadIdx.x;
    if (I >= nc) return;
    const int m0 = lead[I];
    const int m1 = mate[m0];
    SortedAcc<RAP_CAP> acc;
    acc.clear();
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
    const int m0 = lead[I];
    const int m1 = mate[m0];
    SortedAcc<RAP_CAP> acc;
    acc.clear();
    if (!rap_row<true>(acc, rp[m0], rp[m0 + 1], ci, v, agg)) return;  // overflow row: slow path
    if (m1 >= 0 && !rap_row<true>(acc, rp[m1], rp[m1 + 1], ci, v, agg)) return;
    const int o = crp[I];
#pragma unroll
    for (int t = 0; t < RAP_CAP; ++t) {
        if (t < acc.len) {
            cci[o + t] = acc.key[t];
            cv[o + t] = acc.val[t];
        }
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

void launch_rap_count(int nc, const int* lead, const int* mate, const int* rp, const int* ci, const int* agg,
                      int* rowcnt, int* ovf, int* novf, hipStream_t s) {
    hipLaunchKernelGGL(k_rap_count, dim3(blocks_for(nc, RAP_BS)), dim3(RAP_BS), 0, s, nc, lead, mate, rp, ci, agg,
                       rowcnt, ovf, novf);
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
__global__ __launch_bounds__(BS) void k_dense_assemble(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v, double* __restrict__ a) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) a[(size_t)i * n + ci[k]] = v[k];
}

void launch_dense_assemble(int n, const int* rp, const int* ci, const double* v, double* a, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_assemble, dim3(blocks_for(n)), dim3(BS), 0, s, n, rp, ci, v, a);
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

// Right-looking LU with partial pivoting in place (row-major a, unit lower L
// below the diagonal).  perm[i] = original row of position i (P A = L U).
// One workgroup; the pivot row and the multipliers of each step sit in LDS.
__global__ __launch_bounds__(LU_BS) void k_dense_lu(int n, double* __restrict__ a, int* __restrict__ perm, int* err) {
    __shared__ double rowk[1024], colk[1024];
    __shared__ int sperm[1024];
    __shared__ double sv[LU_BS / kWave];
    __shared__ int si[LU_BS / kWave];
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += LU_BS) sperm[i] = i;
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = n;
        for (int i = k + tid; i < n; i += LU_BS) {
            const double t = fabs(a[(size_t)i * n + k]);
            if (t > best) {  // rows ascend per thread: strict '>' keeps the lowest
                best = t;
                bi = i;
            }
        }
        lu_argmax(best, bi, sv, si);
        if (!(best > 0.0) || !isfinite(best)) {  // uniform across the block
            if (tid == 0) atomicOr(err, ERR_SINGULAR);
            return;
        }
        const int p = bi;
        // row swap (all columns), recorded in the permutation
        if (p != k)
            for (int j = tid; j < n; j += LU_BS) {
                const double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        if (tid == 0 && p != k) {
            const int t = sperm[k];
            sperm[k] = sperm[p];
            sperm[p] = t;
        }
        __syncthreads();
        const double d = a[(size_t)k * n + k];
        for (int j = k + 1 + tid; j < n; j += LU_BS) rowk[j] = a[(size_t)k * n + j];
        for (int i = k + 1 + tid; i < n; i += LU_BS) {
            const double l = a[(size_t)i * n + k] / d;
            colk[i] = l;
            a[(size_t)i * n + k] = l;
        }
        __syncthreads();
        const int m = n - k - 1;
        for (int t = tid; t < m * m; t += LU_BS) {
            const int i = k + 1 + t / m, j = k + 1 + t % m;
            a[(size_t)i * n + j] -= colk[i] * rowk[j];
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += LU_BS) perm[i] = sperm[i];
}

// Columns of A^{-1} = U^{-1} L^{-1} P, INV_COLS per block, held in LDS as
// x[i * INV_COLS + c] (at most 64 KiB).  Each row of a substitution is a dot
// product split over INV_SLICES lanes (fixed order) and reduced with
// shuffles.  Writes the inverse column-major: ainv_t[c * n + i] = (A^{-1})_{ic}.
template <int INV_COLS>
__global__ __launch_bounds__(INV_BS) void k_dense_inverse(int n, const double* __restrict__ lu,
                                                          const int* __restrict__ perm, double* __restrict__ ainv_t) {
    constexpr int INV_SLICES = INV_BS / INV_COLS;
    extern __shared__ double x[];
    const int c0 = blockIdx.x * INV_COLS;
    const int c = threadIdx.x / INV_SLICES, sl = threadIdx.x % INV_SLICES;
    for (int t = threadIdx.x; t < n * INV_COLS; t += INV_BS) {
        const int i = t / INV_COLS, cc = t % INV_COLS;
        x[t] = perm[i] == c0 + cc ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = 1; i < n; ++i) {  // unit lower
        double s = 0.0;
        for (int k = sl; k < i; k += INV_SLICES) s += lu[(size_t)i * n + k] * x[k * INV_COLS + c];
        for (int off = INV_SLICES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (sl == 0) x[i * INV_COLS + c] -= s;
        __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {  // upper
        double s = 0.0;
        for (int k = i + 1 + sl; k < n; k += INV_SLICES) s += lu[(size_t)i * n + k] * x[k * INV_COLS + c];
        for (int off = INV_SLICES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (sl == 0) x[i * INV_COLS + c] = (x[i * INV_COLS + c] - s) / lu[(size_t)i * n + i];
        __syncthreads();
    }
    for (int t = threadIdx.x; t < n * INV_COLS; t += INV_BS) {
        const int cc = t / n, i = t % n;
        if (c0 + cc < n) ainv_t[(size_t)(c0 + cc) * n + i] = x[i * INV_COLS + cc];
    }
}

void launch_dense_lu_inverse(int n, double* a, int* perm, double* ainv_t, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_lu, dim3(1), dim3(LU_BS), 0, s, n, a, perm, err);
    if (n <= 512)
        hipLaunchKernelGGL(k_dense_inverse<16>, dim3((n + 15) / 16), dim3(INV_BS), sizeof(double) * (size_t)n * 16, s,
                           n, a, perm, ainv_t);
    else
        hipLaunchKernelGGL(k_dense_inverse<8>, dim3((n + 7) / 8), dim3(INV_BS), sizeof(double) * (size_t)n * 8, s, n,
                           a, perm, ainv_t);
}

}  // namespace amg
