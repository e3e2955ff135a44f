// Node-based heavy edge matching (Section 2.1.1, Algorithm 2) on the GPU.
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
//
// Drivers: one workgroup with the round stamps, ready counters and worklists
// in LDS (passes up to kHemLdsRows rows; a round costs the two adjacency
// record loads), the same per system of a block-diagonal batch, and tiles of
// consecutive rows with one such workgroup each, all in one launch (larger
// passes; the tiles exchange decisions through one published word per
// vertex).  One kernel launch per round over the whole GPU and one workgroup
// with the state in global memory remain for passes the tiles do not take.
#include <cstdint>

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
}  // namespace

constexpr int INIT_GRP = 4;  // row entries whose loads k_hem_init issues together

// Position of column c in ci[lo, hi) (ascending), or -1: rows of up to 8
// entries in one load step, longer ones by bisection.
__device__ __forceinline__ int find_col_short(const int* __restrict__ ci, int lo, int hi, int c) {
    if (hi - lo > 8) return find_col(ci, lo, hi, c);
    int x[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) x[t] = lo + t < hi ? ci[lo + t] : -1;
    int p = -1;
#pragma unroll
    for (int t = 7; t >= 0; --t)
        if (x[t] == c) p = lo + t;
    return p;
}

// counters: cnt[0..2] worklist sizes (ring of 3), cnt[5] sum over rows of
// (#upper - #lower) entries, cnt[6] the number of rounds that had work,
// cnt[7] set when a single-workgroup pass hit its round limit.
template <int SIDE>
__global__ __launch_bounds__(BS) void k_hem_init(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ v, uint8_t* __restrict__ lowok,
                                                 HemRecT<SIDE>* __restrict__ rec, int* __restrict__ lcnt,
                                                 int* __restrict__ dec, int* __restrict__ mate,
                                                 int* __restrict__ wl0, int* cnt, int* err) {
    const int y = blockIdx.x * BS + threadIdx.x;
    int nlow = 0, nup = 0;
    if (y < n) {
        dec[y] = kUndecided;
        mate[y] = -1;
        int c = 0, bad = 0, nh = 0, nl = 0;
        bool hitr = false, lotr = false;
        int hj[SIDE], lx[SIDE];
        double hw[SIDE];
#pragma unroll
        for (int t = 0; t < SIDE; ++t) {
            hj[t] = -1;
            lx[t] = -1;
            hw[t] = 0.0;
        }
        // Entries in groups of INIT_GRP: the loads of a group (columns, the rows
        // of the lower neighbours, the mirrored entries' values) are issued
        // together, then the entries are taken in order.
        const int e0 = rp[y], e1 = rp[y + 1];
        for (int k0 = e0; k0 < e1; k0 += INIT_GRP) {
            int us[INIT_GRP], pos[INIT_GRP];
            double own[INIT_GRP], mir[INIT_GRP];
#pragma unroll
            for (int t = 0; t < INIT_GRP; ++t) {
                us[t] = k0 + t < e1 ? ci[k0 + t] : y;
                own[t] = k0 + t < e1 ? v[k0 + t] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < INIT_GRP; ++t) pos[t] = us[t] < y ? find_col_short(ci, rp[us[t]], rp[us[t] + 1], y) : -1;
#pragma unroll
            for (int t = 0; t < INIT_GRP; ++t) mir[t] = pos[t] >= 0 ? v[pos[t]] : 0.0;
#pragma unroll
            for (int q = 0; q < INIT_GRP; ++q) {
                const int k = k0 + q;
                if (k >= e1) break;
                const int u = us[q];
                uint8_t ok = 0;
                if (u < y) {
                    ++nlow;
                    if (pos[q] < 0) bad = 1;
                    else if (mir[q] != 0.0) ok = 1;
                    if (ok) {  // lower edge-neighbour, columns arrive ascending
                        if (nl < SIDE) {
#pragma unroll
                            for (int t = 0; t < SIDE; ++t)
                                if (t == nl) lx[t] = u;
                            ++nl;
                        } else {
                            lotr = true;  // the smallest SIDE are kept
                        }
                    }
                } else if (u > y) {
                    ++nup;
                    const double a = own[q];
                    if (a != 0.0) {  // higher neighbour: the first SIDE by |a| descending, column ascending
                        const double w = fabs(a);
                        int at = 0;
#pragma unroll
                        for (int t = 0; t < SIDE; ++t)
                            if (t < nh && hw[t] >= w) at = t + 1;
                        if (at < SIDE) {
#pragma unroll
                            for (int t = SIDE - 1; t > 0; --t)
                                if (t > at && t <= nh) {  // a full list drops its last entry
                                    hw[t] = hw[t - 1];
                                    hj[t] = hj[t - 1];
                                }
#pragma unroll
                            for (int t = 0; t < SIDE; ++t)
                                if (t == at) {
                                    hw[t] = w;
                                    hj[t] = u;
                                }
                        }
                        if (nh < SIDE) ++nh;
                        else hitr = true;
                    }
                }
                lowok[k] = ok;
                c += ok;
            }
        }
        HemRecT<SIDE> R;
        R.hdr = nh | (nl << 8) | (hitr ? kRecHiTrunc : 0) | (lotr ? kRecLoTrunc : 0) | (hitr || lotr ? kRecOverflow : 0);
#pragma unroll
        for (int t = 0; t < SIDE; ++t) {
            R.h[t] = hj[t];
            R.l[t] = lx[t];
        }
        R.pad = 0;
        rec[y] = R;
        lcnt[y] = c;
        if (bad) atomicOr(err, ERR_NONSYM);
        if (c == 0) wl0[atomicAdd(&cnt[0], 1)] = y;
    }
    // The pattern check, summed over the block and added only when nonzero:
    // adds to one word from every block serialise across the XCDs.  With one
    // add per wave, the first pass of a 128^3 grid (where every wave holds a
    // row at the end of a grid line) took 1.83 ms instead of 1.56 ms; a
    // block's boundary rows mostly cancel.
    __shared__ int s_diff[BS / kWave];
    int diff = nup - nlow;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) diff += __shfl_xor(diff, o);
    if (threadIdx.x % kWave == 0) s_diff[threadIdx.x / kWave] = diff;
    __syncthreads();
    if (threadIdx.x == 0) {
        int d = 0;
#pragma unroll
        for (int k = 0; k < BS / kWave; ++k) d += s_diff[k];
        if (d != 0) atomicAdd(&cnt[5], d);
    }
}

namespace {
// Read-only inputs of a pass and the partner output.
struct HemState {
    const int* __restrict__ rp;
    const int* __restrict__ ci;
    const double* __restrict__ v;
    const uint8_t* __restrict__ lowok;
    const void* __restrict__ rec;  // HemRecT<SIDE>[n]
    int* mate;
};

// Round stamps and ready counters in global memory (atomics at SCOPE).
template <int SCOPE>
struct GlobalSt {
    int* dec;
    int* lcnt;
    __device__ __forceinline__ int get(int i) const { return dec[i]; }
    __device__ __forceinline__ void set(int i, int r) const { dec[i] = r; }
    // returns the count before the decrement
    __device__ __forceinline__ int drop(int y) const {
        return __hip_atomic_fetch_add(&lcnt[y], -1, __ATOMIC_RELAXED, SCOPE);
    }
    // drop(y) when take, else an atomic add of zero on the counter of self (a
    // decided vertex): the updates of a list are then issued back to back with
    // one wait, where a branch around each would wait for every one in turn
    // (returns 0 when not take)
    __device__ __forceinline__ int drop_if(int y, bool take, int self) const {
        const int old = __hip_atomic_fetch_add(&lcnt[take ? y : self], take ? -1 : 0, __ATOMIC_RELAXED, SCOPE);
        return take ? old : 0;
    }
};

// The same in LDS: 16-bit stamps (0xffff = undecided) and 16-bit counters
// packed two to a word.  A counter is only decremented while positive, so
// the subtraction never borrows from its neighbour.
// Vertices off .. off+n-1 are held at LDS index (vertex - off).
struct LdsSt {
    uint16_t* dec;
    unsigned* lcnt2;
    int off;
    __device__ __forceinline__ int get(int i) const { return dec[i - off]; }
    __device__ __forceinline__ void set(int i, int r) const { dec[i - off] = (uint16_t)r; }
    __device__ __forceinline__ int drop(int y) const {
        y -= off;
        const unsigned sh = 16u * (unsigned)(y & 1);
        const unsigned old = atomicSub(&lcnt2[y >> 1], 1u << sh);
        return (int)((old >> sh) & 0xffffu);
    }
    // as GlobalSt::drop_if (self: a vertex of the range)
    __device__ __forceinline__ int drop_if(int y, bool take, int self) const {
        const int i = (take ? y : self) - off;
        const unsigned sh = 16u * (unsigned)(i & 1);
        const unsigned old = atomicSub(&lcnt2[i >> 1], take ? 1u << sh : 0u);
        return take ? (int)((old >> sh) & 0xffffu) : 0;
    }
};

// Appends to the next worklist through a block-local LDS list of element
// type E (holding vertex - off); entries that do not fit go to a global list.
template <class E>
struct Appender {
    E* s_list;
    int* s_cnt;
    int cap;
    int* gout;
    int* gcnt;
    int off = 0;
    __device__ __forceinline__ void push(int x) const {
        const int p = atomicAdd(s_cnt, 1);
        if (p < cap) s_list[p] = (E)(x - off);
        else gout[atomicAdd(gcnt, 1)] = x;
    }
};

constexpr int HEM_WIN = 8;  // row entries whose loads are issued together

// x has just been decided: its higher neighbours lose one undecided lower
// neighbour; those that reach zero are ready for the next round.  The
// counter updates of a window are issued before any result is used.
template <class St, class Ap>
__device__ __forceinline__ void hem_release(const HemState& S, const St& st, int x, const Ap& A) {
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
        for (int t = 0; t < HEM_WIN; ++t) old[t] = st.drop_if(ys[t], ys[t] >= 0, x);
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t)
            if (ys[t] >= 0 && old[t] == 1) A.push(ys[t]);
    }
}

// Heaviest undecided higher neighbour of u (lowest index on ties), or -1.
template <class St>
__device__ __forceinline__ int hem_best(const HemState& S, const St& st, int r, int u, int e0, int e1) {
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
        for (int t = 0; t < HEM_WIN; ++t) und[t] = js[t] >= 0 && st.get(js[t]) >= r;
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
template <class St>
__device__ __forceinline__ int hem_back(const HemState& S, const St& st, int r, int w) {
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
        for (int t = 0; t < HEM_WIN; ++t) und[t] = xs[t] >= 0 && st.get(xs[t]) >= r;
#pragma unroll
        for (int t = 0; t < HEM_WIN; ++t)
            if (und[t]) return xs[t];  // columns ascend: the first is the smallest
        if (stop) break;
    }
    return -1;
}

// Counter updates for the higher neighbours listed in a record, all issued
// before any result is used.
template <class St, int SIDE, class Ap>
__device__ __forceinline__ void rec_release(const HemState& S, const St& st, const HemRecT<SIDE>& R, int x,
                                            const Ap& A) {
    if (R.hdr & kRecHiTrunc) {
        hem_release(S, st, x, A);
        return;
    }
    const int nh = R.hdr & 255;
    int old[SIDE];
#pragma unroll
    for (int t = 0; t < SIDE; ++t) old[t] = st.drop_if(R.h[t], t < nh, x);
#pragma unroll
    for (int t = 0; t < SIDE; ++t)
        if (t < nh && old[t] == 1) A.push(R.h[t]);
}

// Round r for a ready vertex u.  Records list u's higher neighbours in
// preference order (heaviest first, lowest index on ties) and the target's
// lower edge-neighbours in ascending order, so "first undecided entry" is the
// pointer of either side; a truncated list decides only when it holds an
// undecided entry.  With WAVE_OK, a visit that needs a CSR row (a pointer
// past a truncated list, or the release of a truncated higher list) is not
// done here: the function returns true before any change and the caller
// hands u to a whole wave (hem_visit_wave) later in the round.
template <class St, int SIDE, bool WAVE_OK, class Ap>
__device__ __forceinline__ bool hem_visit(const HemState& S, const St& st, int r, int u, const Ap& A) {
    const HemRecT<SIDE>* __restrict__ recs = static_cast<const HemRecT<SIDE>*>(S.rec);
    const HemRecT<SIDE> R = recs[u];
    if (st.get(u) < r) return false;  // decided earlier (as a match target): stale entry
    int best = -1;
    {
        const int nh = R.hdr & 255;
        int d[SIDE];
#pragma unroll
        for (int t = 0; t < SIDE; ++t) d[t] = t < nh ? st.get(R.h[t]) : -1;
#pragma unroll
        for (int t = SIDE - 1; t >= 0; --t)
            if (t < nh && d[t] >= r) best = R.h[t];
    }
    if (best < 0 && (R.hdr & kRecHiTrunc)) {  // every listed choice decided: the row decides
        if (WAVE_OK) return true;
        best = hem_best(S, st, r, u, S.rp[u], S.rp[u + 1]);
    }
    if (best < 0) {  // no undecided neighbour: unaggregated singleton
        st.set(u, r);
        S.mate[u] = -1;
        rec_release(S, st, R, u, A);
        return false;
    }
    const HemRecT<SIDE> B = recs[best];
    int back = -1;
    {
        const int nl = (B.hdr >> 8) & 255;
        int d[SIDE];
#pragma unroll
        for (int t = 0; t < SIDE; ++t) d[t] = t < nl ? st.get(B.l[t]) : -1;
#pragma unroll
        for (int t = SIDE - 1; t >= 0; --t)
            if (t < nl && d[t] >= r) back = B.l[t];
    }
    if (back < 0 && (B.hdr & kRecLoTrunc)) {
        if (WAVE_OK) return true;
        back = hem_back(S, st, r, best);
    }
    if (back == u) {  // best points back: mutual, matched
        if (WAVE_OK && ((R.hdr | B.hdr) & kRecHiTrunc)) return true;  // releases scan rows
        st.set(u, r);
        st.set(best, r);
        S.mate[u] = best;
        S.mate[best] = u;
        rec_release(S, st, R, u, A);
        rec_release(S, st, B, best, A);
    } else {
        A.push(u);  // still ready, retry next round
    }
    return false;
}

// Wave reductions of the cooperative visit.
__device__ __forceinline__ void wave_best(double& w, int& j) {  // |a| descending, column ascending
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ow = __shfl_xor(w, off);
        const int oj = __shfl_xor(j, off);
        if (ow > w || (ow == w && oj < j)) {
            w = ow;
            j = oj;
        }
    }
}
__device__ __forceinline__ int wave_min(int x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off));
    return x;
}
// first lane (in list order) whose entry is undecided, or -1
__device__ __forceinline__ int wave_first(bool und, int val) {
    const unsigned long long m = __ballot(und);
    return m ? __shfl(val, __ffsll((long long)m) - 1) : -1;
}

// Release of x by a whole wave: its record's higher-neighbour list, or its
// CSR row when the record overflowed, spread over the lanes.
template <class St, class Ap>
__device__ __forceinline__ void wave_release(const HemState& S, const St& st, int x, int hdr, int myh,
                                             const Ap& A) {
    const int lane = threadIdx.x % kWave;
    if (hdr & kRecHiTrunc) {
        for (int e = S.rp[x] + lane; e < S.rp[x + 1]; e += kWave) {
            const int y = S.ci[e];
            if (y > x && S.v[e] != 0.0 && st.drop(y) == 1) A.push(y);
        }
    } else if (lane < (hdr & 255)) {
        if (st.drop(myh) == 1) A.push(myh);
    }
}

// The visit of hem_visit with all 64 lanes of a wave on one vertex u (u is
// wave-uniform): row scans take one load step per 64 entries and the
// choices are wave reductions, so long rows cost a few dependent loads.
template <class St, int SIDE, class Ap>
__device__ __forceinline__ void hem_visit_wave(const HemState& S, const St& st, int r, int u, const Ap& A) {
    const int lane = threadIdx.x % kWave;
    const int* __restrict__ ru = reinterpret_cast<const int*>(static_cast<const HemRecT<SIDE>*>(S.rec) + u);
    const int hdr = ru[0];
    const int myh = lane < SIDE ? ru[1 + lane] : -1;
    if (st.get(u) < r) return;
    int best;
    if (hdr & kRecHiTrunc) {
        double bw = -1.0;
        int bj = INT_MAX;
        for (int e = S.rp[u] + lane; e < S.rp[u + 1]; e += kWave) {
            const int j = S.ci[e];
            const double a = S.v[e];
            if (j > u && a != 0.0 && st.get(j) >= r) {
                const double w = fabs(a);
                if (w > bw || (w == bw && j < bj)) {
                    bw = w;
                    bj = j;
                }
            }
        }
        wave_best(bw, bj);
        best = bw < 0.0 ? -1 : bj;
    } else {
        best = wave_first(lane < (hdr & 255) && st.get(myh) >= r, myh);
    }
    if (best < 0) {
        if (lane == 0) {
            st.set(u, r);
            S.mate[u] = -1;
        }
        wave_release(S, st, u, hdr, myh, A);
        return;
    }
    const int* __restrict__ rb = reinterpret_cast<const int*>(static_cast<const HemRecT<SIDE>*>(S.rec) + best);
    const int bhdr = rb[0];
    const int bh = lane < SIDE ? rb[1 + lane] : -1;
    int back;
    if (bhdr & kRecLoTrunc) {
        int mx = INT_MAX;
        for (int e = S.rp[best] + lane; e < S.rp[best + 1]; e += kWave) {
            const int x = S.ci[e];
            if (x < best && S.lowok[e] && st.get(x) >= r) mx = min(mx, x);
        }
        mx = wave_min(mx);
        back = mx == INT_MAX ? -1 : mx;
    } else {
        const int bl = lane < SIDE ? rb[1 + SIDE + lane] : -1;
        back = wave_first(lane < ((bhdr >> 8) & 255) && st.get(bl) >= r, bl);
    }
    if (back == u) {
        if (lane == 0) {
            st.set(u, r);
            st.set(best, r);
            S.mate[u] = best;
            S.mate[best] = u;
        }
        wave_release(S, st, u, hdr, myh, A);
        wave_release(S, st, best, bhdr, bh, A);
    } else if (lane == 0) {
        A.push(u);
    }
}

// One round over a list of ready vertices (items idx < m, fetched by `item`):
// single-lane visits first, then the deferred long rows one wave each.
template <class St, int SIDE, int NT, class Ap, class Item>
__device__ __forceinline__ void hem_round_body(const HemState& S, const St& st, int r, int m, int first, int stride,
                                               const Item& item, const Ap& A, int* s_wave, int* s_nw, int wcap) {
    for (int idx = first; idx < m; idx += stride) {
        const int u = item(idx);
        if (hem_visit<St, SIDE, true>(S, st, r, u, A)) {
            const int p = atomicAdd(s_nw, 1);
            if (p < wcap) s_wave[p] = u;
            else hem_visit<St, SIDE, false>(S, st, r, u, A);
        }
    }
    __syncthreads();
    const int nw = min(*s_nw, wcap);
    for (int k = threadIdx.x / kWave; k < nw; k += NT / kWave) hem_visit_wave<St, SIDE>(S, st, r, s_wave[k], A);
    __syncthreads();
}

constexpr int HEM_BS = 512;
constexpr int HEM_LCAP = 4096;
// Threads of the workgroup-wide drivers with LDS state (one workgroup, systems
// of a batch, tiles): records of 31 entries a side need the registers of 512.
template <int SIDE>
constexpr int hem_nt() {
    return SIDE > 15 ? 512 : 1024;
}
constexpr int HEM_LCAP1 = 8192;
constexpr int HEM_WCAP = 1024;  // vertices deferred to the wave path per block and round
constexpr int HL_LCAP = 4096;   // LDS worklist entries of the LDS-state driver
constexpr int HL_WCAP = 512;
}  // namespace

// One round over the worklist; the decided vertices' neighbours that become
// ready, and the ready vertices that failed, form the next list.
template <int SIDE>
__global__ __launch_bounds__(HEM_BS) void k_hem_round(int r, int n, HemState S, int* dec, int* lcnt,
                                                  const int* __restrict__ win, int* __restrict__ wout, int* cnt,
                                                  int slot_in, int slot_out, int zero_w) {
    __shared__ int s_list[HEM_LCAP];
    __shared__ int s_wave[HEM_WCAP];
    __shared__ int s_cnt, s_base, s_nw;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_nw = 0;
        if (blockIdx.x == 0) cnt[zero_w] = 0;
    }
    __syncthreads();
    // the list size and this thread's first entry are loaded together
    // (entries past the size are ignored)
    const int first = blockIdx.x * HEM_BS + threadIdx.x;
    const int m = cnt[slot_in];
    const int u0 = first < n ? win[first] : -1;
    if (m > 0 && blockIdx.x == 0 && threadIdx.x == 0) cnt[6] = r + 1;  // rounds with work
    const Appender<int> A{s_list, &s_cnt, HEM_LCAP, wout, &cnt[slot_out]};
    const GlobalSt<__HIP_MEMORY_SCOPE_AGENT> st{dec, lcnt};
    hem_round_body<GlobalSt<__HIP_MEMORY_SCOPE_AGENT>, SIDE, HEM_BS>(
        S, st, r, m, first, gridDim.x * HEM_BS, [&](int i) { return i == first ? u0 : win[i]; }, A, s_wave, &s_nw,
        HEM_WCAP);
    const int k = min(s_cnt, HEM_LCAP);
    if (threadIdx.x == 0 && k > 0) s_base = atomicAdd(&cnt[slot_out], k);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += HEM_BS) wout[s_base + i] = s_list[i];
}

// Mid-size passes: one workgroup runs every round, separated by barriers,
// with the state in global memory.  Each round decides at least the smallest
// undecided vertex, so n + 1 rounds always suffice; the bound only guards
// against invalid input.  Records of 31 entries a side take the registers of
// 512 threads, as in the LDS-state drivers; with 1024 they would spill.
template <int SIDE>
__global__ __launch_bounds__(hem_nt<SIDE>()) void k_hem_all(int n, HemState S, int* dec, int* lcnt, int* wl0, int* wl1,
                                                     int* cnt) {
    __shared__ int s_list[HEM_LCAP1];
    __shared__ int s_wave[HEM_WCAP];
    __shared__ int s_cnt, s_next, s_m, s_nw;
    constexpr int NT = hem_nt<SIDE>();
    if (threadIdx.x == 0) s_m = cnt[0];
    __syncthreads();
    const GlobalSt<__HIP_MEMORY_SCOPE_WORKGROUP> st{dec, lcnt};
    int* win = wl0;
    int* wout = wl1;
    int r = 0;
    for (; r <= n + 1; ++r) {
        const int m = s_m;
        if (m == 0) break;
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_next = 0;
            s_nw = 0;
        }
        __syncthreads();
        const Appender<int> A{s_list, &s_cnt, HEM_LCAP1, wout, &s_next};
        hem_round_body<GlobalSt<__HIP_MEMORY_SCOPE_WORKGROUP>, SIDE, NT>(
            S, st, r, m, threadIdx.x, NT, [&](int i) { return win[i]; }, A, s_wave, &s_nw, HEM_WCAP);
        const int k = min(s_cnt, HEM_LCAP1);
        const int base = s_next;
        for (int i = threadIdx.x; i < k; i += NT) wout[base + i] = s_list[i];
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

// Small passes (n <= kHemLdsRows): one workgroup with the round stamps, the
// ready counters and the worklists in LDS, for the vertices off .. off+n-1
// (no edge leaves the range).  A list is its LDS part followed by a global
// part for entries beyond the LDS capacity.  The first list is the kg0
// entries of gin, or with scan the vertices whose counter is zero.  Returns
// the rounds run; *left is nonzero when the round bound was hit.
template <int SIDE>
__device__ __forceinline__ int hem_lds_body(int off, int n, const HemState& S, const int* __restrict__ lcnt_g, int* gin,
                            int* gout, int kg0, bool scan, int* left) {
    __shared__ uint16_t s_dec[kHemLdsRows];
    __shared__ unsigned s_lcnt2[kHemLdsRows / 2];
    __shared__ uint16_t s_la[HL_LCAP], s_lb[HL_LCAP];
    __shared__ int s_wave[HL_WCAP];
    __shared__ int s_cnt, s_gnext, s_nw;
    for (int i = threadIdx.x; i < n; i += hem_nt<SIDE>()) s_dec[i] = 0xffff;
    for (int i = threadIdx.x; 2 * i < n; i += hem_nt<SIDE>()) {
        const unsigned lo = (unsigned)lcnt_g[off + 2 * i];
        const unsigned hi = 2 * i + 1 < n ? (unsigned)lcnt_g[off + 2 * i + 1] : 0u;
        s_lcnt2[i] = lo | (hi << 16);
    }
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_gnext = 0;
    }
    __syncthreads();
    const LdsSt st{s_dec, s_lcnt2, off};
    uint16_t* cur = s_la;
    uint16_t* nxt = s_lb;
    int kl = 0, kg = kg0;
    if (scan) {  // the first list: vertices with no lower edge-neighbour
        const Appender<uint16_t> A{cur, &s_cnt, HL_LCAP, gin, &s_gnext, off};
        for (int i = threadIdx.x; i < n; i += hem_nt<SIDE>())
            if (lcnt_g[off + i] == 0) A.push(off + i);
        __syncthreads();
        kl = min(s_cnt, HL_LCAP);
        kg = s_gnext;
        __syncthreads();
    }
    int r = 0;
    for (; r <= n + 1; ++r) {
        const int m = kl + kg;
        if (m == 0) break;
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_gnext = 0;
            s_nw = 0;
        }
        __syncthreads();
        const Appender<uint16_t> A{nxt, &s_cnt, HL_LCAP, gout, &s_gnext, off};
        const uint16_t* c = cur;
        const int* g = gin;
        const int klc = kl;
        hem_round_body<LdsSt, SIDE, hem_nt<SIDE>()>(
            S, st, r, m, threadIdx.x, hem_nt<SIDE>(), [&](int i) { return i < klc ? (int)c[i] + off : g[i - klc]; }, A,
            s_wave, &s_nw, HL_WCAP);
        kl = min(s_cnt, HL_LCAP);
        kg = s_gnext;
        __syncthreads();  // every thread has read the counts before the next reset
        uint16_t* t = cur;
        cur = nxt;
        nxt = t;
        int* tg = gin;
        gin = gout;
        gout = tg;
    }
    *left = kl + kg;
    return r;
}

template <int SIDE>
__global__ __launch_bounds__(hem_nt<SIDE>()) void k_hem_lds(int n, HemState S, const int* __restrict__ lcnt_g, int* wl0,
                                                     int* wl1, int* cnt) {
    int left = 0;
    const int r = hem_lds_body<SIDE>(0, n, S, lcnt_g, wl0, wl1, cnt[0], false, &left);
    if (threadIdx.x == 0) {
        cnt[6] = r;
        if (left != 0) cnt[7] = 1;
    }
}

// Systems stored one after another (a block-diagonal operator): block b
// matches system seg[b] = (first vertex, rows) with the LDS-state rounds when
// it has at most lim (<= kHemLdsRows) rows (larger ones are left to the other
// drivers), then marks its vertices as decided before round 0 in the global
// stamps so that those drivers skip them.  Global list space: the system's
// own rows of sl0 and sl1.
template <int SIDE>
__global__ __launch_bounds__(hem_nt<SIDE>()) void k_hem_lds_seg(const int2* __restrict__ seg, HemState S,
                                                         const int* __restrict__ lcnt_g, int* __restrict__ dec_g,
                                                         int* sl0, int* sl1, int* cnt, int lim) {
    const int2 sg = seg[blockIdx.x];
    const int off = sg.x, n = sg.y;
    if (n <= 0 || n > lim) return;  // uniform
    int left = 0;
    const int r = hem_lds_body<SIDE>(off, n, S, lcnt_g, sl0 + off, sl1 + off, 0, true, &left);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += hem_nt<SIDE>()) dec_g[off + i] = -1;
    if (threadIdx.x == 0) {
        atomicMax(&cnt[6], r);
        if (left != 0) atomicOr(&cnt[7], 1);
    }
}

// ---------------------------------------------------------------------------
// Tiled passes: the vertices are cut into tiles of T consecutive indices, one
// workgroup per tile, all in one launch.  A workgroup keeps its tile's round
// stamps, ready counters and worklists in LDS and runs rounds of its own, as
// the LDS-state driver does, while the other tiles run theirs.  A decision on
// a vertex u reads only u's neighbours and the states of its target's lower
// edge-neighbours below u, so a tile waits only on lower tiles, and the
// matching is the same greedy matching whatever the timing.
//
// dec_g[v] publishes each decision to the other tiles in one word: partner
// + 2, or 1 for a singleton (kUndecided before).  A vertex can only be taken
// by one of its lower edge-neighbours, so a reader learns whether y is taken
// from y's lower edge-neighbours' words alone; no read has to be ordered
// after another, and a stale word only makes a vertex wait for a later round.
//  * Vertices with lower edge-neighbours in lower tiles ("exposed") start
//    "pending": they count as undecided, but their own tile may neither match
//    them nor let them choose until those neighbours are all decided.  Then
//    the words tell whether one of them took the vertex, and one
//    compare-and-swap on its LDS stamp settles it (free, or taken: stamped
//    decided, counted and released by the thread that settles it).
//  * A vertex u whose target lies in a higher tile takes it once the target's
//    lower edge-neighbours below u read decided and none of them names it.
//    The thread waits for its own stores before the round ends, so later
//    rounds of the tile read the target's word as taken.
// A workgroup that runs past its time limit sets cnt[7] and stops; the host
// then repeats the pass with the round kernels.
// ---------------------------------------------------------------------------
namespace {
constexpr int kTileUnd = 0xffff;       // LDS stamp: undecided
constexpr int kTilePend = 0xfffe;      // LDS stamp: exposed, not settled yet
constexpr int kTileMaxRound = 0xfff0;  // rounds stop below the two stamps above
constexpr int kExposed = 1 << 20;      // lcnt flag set by k_hem_tile_prep
constexpr int TL_LCAP = 4096;          // LDS worklist entries per list

struct TileSt {
    uint16_t* sdec;   // LDS stamps of the tile
    unsigned* lcnt2;  // LDS ready counters, two 16-bit counters a word
    int off, m;       // the tile: vertices off .. off+m-1
    int* dec_g;
    __device__ __forceinline__ bool mine(int i) const { return (unsigned)(i - off) < (unsigned)m; }
    __device__ __forceinline__ int word(int i) const {
        return __hip_atomic_load(&dec_g[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // round-stamp view: undecided in round r while >= r
    __device__ __forceinline__ int get(int i) const {
        return mine(i) ? sdec[i - off] : (word(i) != kUndecided ? -1 : INT_MAX);
    }
    __device__ __forceinline__ int drop(int y) const {  // count before the decrement
        y -= off;
        const unsigned sh = 16u * (unsigned)(y & 1);
        const unsigned old = atomicSub(&lcnt2[y >> 1], 1u << sh);
        return (int)((old >> sh) & 0xffffu);
    }
    // as GlobalSt::drop_if; take implies mine(y), and a self outside the
    // tile gives the tile's first counter
    __device__ __forceinline__ int drop_if(int y, bool take, int self) const {
        const int i = take ? y - off : (mine(self) ? self - off : 0);
        const unsigned sh = 16u * (unsigned)(i & 1);
        const unsigned old = atomicSub(&lcnt2[i >> 1], take ? 1u << sh : 0u);
        return take ? (int)((old >> sh) & 0xffffu) : 0;
    }
    __device__ __forceinline__ void publish(int v, int partner) const {
        __hip_atomic_store(&dec_g[v], partner + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// x is decided: its higher neighbours in the tile lose an undecided lower
// neighbour (higher tiles read dec_g instead).
template <int SIDE, class Ap>
__device__ __forceinline__ void tile_release(const HemState& S, const TileSt& st, const HemRecT<SIDE>& R, int x,
                                             const Ap& A) {
    if (R.hdr & kRecHiTrunc) {
        for (int e = S.rp[x]; e < S.rp[x + 1]; ++e) {
            const int y = S.ci[e];
            if (y > x && st.mine(y) && S.v[e] != 0.0 && st.drop(y) == 1) A.push(y);
        }
        return;
    }
    const int nh = R.hdr & 255;
    int old[SIDE];
#pragma unroll
    for (int t = 0; t < SIDE; ++t) {
        const int y = t < nh ? R.h[t] : x;
        old[t] = st.drop_if(y, t < nh && st.mine(y), x);
    }
#pragma unroll
    for (int t = 0; t < SIDE; ++t)
        if (t < nh && old[t] == 1) A.push(R.h[t]);
}

enum { kUnsettled = 0, kFree = 1, kGone = 2 };

// Compare-and-swap of the 16-bit LDS stamp i; returns the stamp before.
__device__ __forceinline__ int cas_stamp(uint16_t* sdec, int i, int expect, int want) {
    unsigned* w = reinterpret_cast<unsigned*>(sdec) + (i >> 1);
    const unsigned sh = 16u * (unsigned)(i & 1);
    unsigned old = *w;
    for (;;) {
        const int h = (int)((old >> sh) & 0xffffu);
        if (h != expect) return h;
        const unsigned nw = (old & ~(0xffffu << sh)) | ((unsigned)want << sh);
        const unsigned got = atomicCAS(w, old, nw);
        if (got == old) return expect;
        old = got;  // the other half changed meanwhile, or this one
    }
}

// Settles the pending vertex y (record Ry) once its lower-tile edge-neighbours
// are decided (all: open == false; taken: one of them names y).  Returns
// kFree or kGone (taken, or matched in this round after another thread
// settled it free).  A vertex found taken is stamped r - 1 (unavailable at
// once), counted and released by the thread whose swap succeeds.
template <int SIDE, class Ap>
__device__ __forceinline__ int tile_settle(const HemState& S, const TileSt& st, const HemRecT<SIDE>& Ry, int y, int r,
                                           bool taken, const Ap& A, int* s_ndec) {
    const int old = cas_stamp(st.sdec, y - st.off, kTilePend, taken ? r - 1 : kTileUnd);
    if (old == kTilePend) {
        if (!taken) return kFree;
        atomicAdd(s_ndec, 1);
        tile_release<SIDE>(S, st, Ry, y, A);
        return kGone;
    }
    return old == kTileUnd ? kFree : kGone;
}

// Lower-tile edge-neighbours of y: open when one is undecided, taken when
// one names y as its partner.
template <int SIDE>
__device__ __forceinline__ void cross_lower(const HemState& S, const TileSt& st, const HemRecT<SIDE>& Ry, int y,
                                            bool& open, bool& taken) {
    open = false;
    taken = false;
    const int nl = (Ry.hdr >> 8) & 255;
    if ((Ry.hdr & kRecLoTrunc) && Ry.l[SIDE - 1] < st.off) {  // a full list; more lower-tile ones may follow
        for (int e = S.rp[y]; e < S.rp[y + 1]; ++e) {
            const int x = S.ci[e];
            if (x >= st.off) break;  // columns ascend
            if (!S.lowok[e]) continue;
            const int wx = st.word(x);
            open |= wx == kUndecided;
            taken |= wx == y + 2;
        }
        return;
    }
    int wx[SIDE];
#pragma unroll
    for (int t = 0; t < SIDE; ++t) wx[t] = t < nl && Ry.l[t] < st.off ? st.word(Ry.l[t]) : 0;
#pragma unroll
    for (int t = 0; t < SIDE; ++t) {
        open |= wx[t] == kUndecided;
        taken |= wx[t] == y + 2;
    }
}

// Smallest undecided lower edge-neighbour of w (stamp view of round r), or -1;
// named: an out-of-tile lower edge-neighbour below the result names w.  The
// listed neighbours decide unless all are decided and the list is truncated;
// then the CSR row does.
template <int SIDE>
__device__ __forceinline__ int tile_back(const HemState& S, const TileSt& st, const HemRecT<SIDE>& B, int w, int r,
                                         bool& named) {
    named = false;
    const int nl = (B.hdr >> 8) & 255;
    int d[SIDE];
    bool nm[SIDE];
#pragma unroll
    for (int t = 0; t < SIDE; ++t) {
        nm[t] = false;
        d[t] = -1;
        if (t < nl) {
            const int x = B.l[t];
            if (st.mine(x)) {
                d[t] = st.sdec[x - st.off];
            } else {
                const int wx = st.word(x);
                d[t] = wx == kUndecided ? INT_MAX : -1;
                nm[t] = wx == w + 2;
            }
        }
    }
    int back = -1;
#pragma unroll
    for (int t = SIDE - 1; t >= 0; --t)
        if (t < nl && d[t] >= r) back = B.l[t];
    if (back >= 0 || !(B.hdr & kRecLoTrunc)) {
#pragma unroll
        for (int t = 0; t < SIDE; ++t)
            if (t < nl && nm[t] && (back < 0 || B.l[t] < back)) named = true;
        return back;
    }
    for (int e = S.rp[w]; e < S.rp[w + 1]; ++e) {  // every listed one decided
        const int x = S.ci[e];
        if (x >= w) break;
        if (!S.lowok[e]) continue;
        if (st.mine(x)) {
            if (st.sdec[x - st.off] >= r) return x;
        } else {
            const int wx = st.word(x);
            if (wx == kUndecided) return x;
            named |= wx == w + 2;
        }
    }
    return -1;
}

// Round r for a ready vertex u of the tile (the visit of hem_visit, with the
// cross-tile rules above).
template <int SIDE, class Ap>
__device__ __forceinline__ void tile_visit(const HemState& S, const TileSt& st, int r, int u, const Ap& A,
                                           int* s_ndec) {
    const HemRecT<SIDE>* __restrict__ recs = static_cast<const HemRecT<SIDE>*>(S.rec);
    const HemRecT<SIDE> R = recs[u];
    const int su = st.sdec[u - st.off];
    if (su < r) return;  // decided earlier (as a match target): stale entry
    if (su == kTilePend) {  // most visits of a pending vertex find it still open
        bool open, taken;
        cross_lower<SIDE>(S, st, R, u, open, taken);
        if (open) {
            A.push(u);
            return;
        }
        if (tile_settle<SIDE>(S, st, R, u, r, taken, A, s_ndec) != kFree) return;
    }
    // the first preference's record, loaded with the states it is chosen by
    const bool spec = (R.hdr & 255) > 0;
    HemRecT<SIDE> B;
    if (spec) B = recs[R.h[0]];
    int best = -1;
    {
        const int nh = R.hdr & 255;
        int d[SIDE];
#pragma unroll
        for (int t = 0; t < SIDE; ++t) d[t] = t < nh ? st.get(R.h[t]) : -1;
#pragma unroll
        for (int t = SIDE - 1; t >= 0; --t)
            if (t < nh && d[t] >= r) best = R.h[t];
    }
    if (best < 0 && (R.hdr & kRecHiTrunc))  // every listed choice decided: the row decides
        best = hem_best(S, st, r, u, S.rp[u], S.rp[u + 1]);
    if (best < 0) {  // no undecided neighbour: unaggregated singleton
        st.sdec[u - st.off] = (uint16_t)r;
        S.mate[u] = -1;
        st.publish(u, -1);
        atomicAdd(s_ndec, 1);
        tile_release<SIDE>(S, st, R, u, A);
        return;
    }
    if (!spec || best != R.h[0]) B = recs[best];
    bool named;
    const int back = tile_back<SIDE>(S, st, B, best, r, named);
    if (back != u) {
        A.push(u);  // still ready, retry next round
        return;
    }
    if (st.mine(best)) {
        // a pending target: its lower-tile edge-neighbours are all below u,
        // hence decided; named says whether one of them took it
        if (st.sdec[best - st.off] == kTilePend && tile_settle<SIDE>(S, st, B, best, r, named, A, s_ndec) != kFree) {
            A.push(u);
            return;
        }
        st.sdec[u - st.off] = (uint16_t)r;
        st.sdec[best - st.off] = (uint16_t)r;
        S.mate[u] = best;
        S.mate[best] = u;
        st.publish(best, u);
        st.publish(u, best);
        atomicAdd(s_ndec, 2);
        tile_release<SIDE>(S, st, R, u, A);
        tile_release<SIDE>(S, st, B, best, A);
        return;
    }
    if (named) {  // taken from a lower tile
        A.push(u);
        return;
    }
    st.sdec[u - st.off] = (uint16_t)r;
    S.mate[u] = best;
    S.mate[best] = u;
    st.publish(best, u);
    st.publish(u, best);
    __builtin_amdgcn_s_waitcnt(0);  // stores complete before the round ends
    atomicAdd(s_ndec, 1);
    tile_release<SIDE>(S, st, R, u, A);
}

// ---------------------------------------------------------------------------
// Small tiles with their adjacency records in LDS.  A tile of up to
// kTileCRows rows keeps, besides its stamps and counters, a compact copy of
// each of its vertices' records: up to kCSide higher and kCSide lower
// neighbours as 16-bit offsets from the vertex.  A vertex whose record does
// not fit (longer lists, truncated lists, offsets beyond 16 bits) is marked
// and read from the global record instead.  A visit then reads global memory
// only for what lies outside the tile: the published words of out-of-tile
// neighbours, and only those the decision needs.
//  * The choice of u scans its preference list; an out-of-tile entry's word
//    is read only when it precedes the first undecided in-tile entry.
//  * The target's lower edge-neighbours in lower tiles are read only while
//    the target is pending: a target of this tile that is no longer pending
//    was settled free, so those neighbours are decided and none took it.
// The rules between tiles are those of the tiled pass above.
// ---------------------------------------------------------------------------
constexpr int kTileCRows = kHemTileCRows;  // largest tile of the compact-record driver
constexpr int kCSide = 4;         // entries a side of a compact record
constexpr int kCGlobal = 0x80;    // compact header flag: use the global record
constexpr int kCompactMaxTiles = 512;  // largest pass (in tiles) that takes compact tiles

struct CRecs {
    const uint8_t* hdr;  // per tile vertex: #higher | #lower << 3 | kCGlobal
    const int16_t* h;    // h[t * kTileCRows + i]: offset of the t-th higher neighbour of vertex off+i
    const int16_t* l;    // lower edge-neighbours, the same layout
    const HemRecT<7>* g;
    int off, m;
    // record of v: from LDS when v is a tile vertex with a compact record
    __device__ __forceinline__ void load(int v, HemRecT<7>& R) const {
        const int i = v - off;
        const int hd = (unsigned)i < (unsigned)m ? hdr[i] : kCGlobal;
        if (hd & kCGlobal) {
            R = g[v];
            return;
        }
        const int nh = hd & 7, nl = (hd >> 3) & 7;
        R.hdr = nh | (nl << 8);
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            R.h[t] = t < kCSide && t < nh ? v + h[t * kTileCRows + i] : -1;
            R.l[t] = t < kCSide && t < nl ? v + l[t * kTileCRows + i] : -1;
        }
        R.pad = 0;
    }
};

// Smallest undecided lower edge-neighbour of w (stamp view of round r), or -1,
// as tile_back; settled: w is a tile vertex that is not pending, so its
// lower-tile edge-neighbours are decided and none named it (not read).
__device__ __forceinline__ int tile_back_c(const HemState& S, const TileSt& st, const HemRecT<7>& B, int w, int r,
                                           bool settled, bool& named) {
    if (!settled) return tile_back<7>(S, st, B, w, r, named);
    named = false;
    const int nl = (B.hdr >> 8) & 255;
    int back = -1;
#pragma unroll
    for (int t = 6; t >= 0; --t) {
        if (t < nl) {
            const int x = B.l[t];
            if (st.mine(x) && st.sdec[x - st.off] >= r) back = x;
        }
    }
    if (back >= 0 || !(B.hdr & kRecLoTrunc)) return back;
    for (int e = S.rp[w]; e < S.rp[w + 1]; ++e) {  // every listed one decided
        const int x = S.ci[e];
        if (x >= w) break;
        if (x < st.off || !S.lowok[e]) continue;
        if (st.sdec[x - st.off] >= r) return x;
    }
    return -1;
}

// Round r for a ready vertex u of a compact tile: the visit of tile_visit
// with records from LDS and the out-of-tile reads cut to what decides.
template <class Ap>
__device__ __forceinline__ void tile_visit_c(const HemState& S, const TileSt& st, const CRecs& C, int r, int u,
                                             const Ap& A, int* s_ndec) {
    HemRecT<7> R;
    C.load(u, R);
    const int su = st.sdec[u - st.off];
    if (su < r) return;  // decided earlier (as a match target): stale entry
    if (su == kTilePend) {  // most visits of a pending vertex find it still open
        bool open, taken;
        cross_lower<7>(S, st, R, u, open, taken);
        if (open) {
            A.push(u);
            return;
        }
        if (tile_settle<7>(S, st, R, u, r, taken, A, s_ndec) != kFree) return;
    }
    const int nh = R.hdr & 255;
    const int b0 = nh > 0 ? R.h[0] : -1;
    HemRecT<7> B;
    if (b0 >= 0) C.load(b0, B);  // the first preference, loaded with the states it is chosen by
    int best = -1;
    {
        int fin = 7;  // first undecided tile entry in preference order
#pragma unroll
        for (int t = 6; t >= 0; --t)
            if (t < nh && st.mine(R.h[t]) && st.sdec[R.h[t] - st.off] >= r) fin = t;
        bool und[7];
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            und[t] = false;
            if (t < nh && t < fin && !st.mine(R.h[t])) und[t] = st.word(R.h[t]) == kUndecided;
        }
#pragma unroll
        for (int t = 6; t >= 0; --t)
            if (t < nh && (t == fin || und[t])) best = R.h[t];
    }
    if (best < 0 && (R.hdr & kRecHiTrunc))  // every listed choice decided: the row decides
        best = hem_best(S, st, r, u, S.rp[u], S.rp[u + 1]);
    if (best < 0) {  // no undecided neighbour: unaggregated singleton
        st.sdec[u - st.off] = (uint16_t)r;
        S.mate[u] = -1;
        st.publish(u, -1);
        atomicAdd(s_ndec, 1);
        tile_release<7>(S, st, R, u, A);
        return;
    }
    if (best != b0) C.load(best, B);
    const bool settled = st.mine(best) && st.sdec[best - st.off] != kTilePend;
    bool named;
    const int back = tile_back_c(S, st, B, best, r, settled, named);
    if (back != u) {
        A.push(u);  // still ready, retry next round
        return;
    }
    if (st.mine(best)) {
        if (!settled && tile_settle<7>(S, st, B, best, r, named, A, s_ndec) != kFree) {
            A.push(u);
            return;
        }
        st.sdec[u - st.off] = (uint16_t)r;
        st.sdec[best - st.off] = (uint16_t)r;
        S.mate[u] = best;
        S.mate[best] = u;
        st.publish(best, u);
        st.publish(u, best);
        atomicAdd(s_ndec, 2);
        tile_release<7>(S, st, R, u, A);
        tile_release<7>(S, st, B, best, A);
        return;
    }
    if (named) {  // taken from a lower tile
        A.push(u);
        return;
    }
    st.sdec[u - st.off] = (uint16_t)r;
    S.mate[u] = best;
    S.mate[best] = u;
    st.publish(best, u);
    st.publish(u, best);
    __builtin_amdgcn_s_waitcnt(0);  // stores complete before the round ends
    atomicAdd(s_ndec, 1);
    tile_release<7>(S, st, R, u, A);
}

// Releases of a compact vertex self: its in-tile higher neighbours h[0..nh)
// lose an undecided lower neighbour; those that reach zero are ready.
template <class Ap>
__device__ __forceinline__ void lean_release(const TileSt& st, const int* h, int nh, int self, const Ap& A) {
    int old[kCSide];
#pragma unroll
    for (int t = 0; t < kCSide; ++t) {
        const int y = t < nh ? h[t] : self;
        old[t] = st.drop_if(y, t < nh && st.mine(y), self);
    }
#pragma unroll
    for (int t = 0; t < kCSide; ++t)
        if (t < nh && old[t] == 1) A.push(h[t]);
}

// The visit of tile_visit_c for a vertex u with a compact record, written on
// the compact lists themselves (at most kCSide entries a side, no 7-entry
// record built); a target without a compact record (outside the tile, or
// with longer lists) hands the visit to tile_visit_c, before any change.
template <class Ap>
__device__ __forceinline__ void tile_visit_lean(const HemState& S, const TileSt& st, const CRecs& C, int r, int u,
                                                const Ap& A, int* s_ndec) {
    const int off = st.off;
    const int i = u - off;
    const int hd = C.hdr[i];
    const int su = st.sdec[i];
    if (hd & kCGlobal) {
        tile_visit_c(S, st, C, r, u, A, s_ndec);
        return;
    }
    if (su < r) return;  // decided earlier (as a match target): stale entry
    const int nh = hd & 7, nl = (hd >> 3) & 7;
    int h[kCSide], l[kCSide];
#pragma unroll
    for (int t = 0; t < kCSide; ++t) {
        h[t] = u + C.h[t * kTileCRows + i];
        l[t] = u + C.l[t * kTileCRows + i];
    }
    if (su == kTilePend) {  // lower-tile edge-neighbours: all decided, and did one take u?
        int wx[kCSide];
#pragma unroll
        for (int t = 0; t < kCSide; ++t) wx[t] = t < nl && l[t] < off ? st.word(l[t]) : 0;
        bool open = false, taken = false;
#pragma unroll
        for (int t = 0; t < kCSide; ++t) {
            open |= wx[t] == kUndecided;
            taken |= wx[t] == u + 2;
        }
        if (open) {
            A.push(u);
            return;
        }
        const int old = cas_stamp(st.sdec, i, kTilePend, taken ? r - 1 : kTileUnd);
        if (old == kTilePend) {
            if (taken) {
                atomicAdd(s_ndec, 1);
                lean_release(st, h, nh, u, A);
                return;
            }
        } else if (old != kTileUnd) {
            return;
        }
    }
    // the choice: first undecided entry in preference order; out-of-tile
    // words only for entries before the first undecided tile entry
    int fin = kCSide;
    bool inb[kCSide];
#pragma unroll
    for (int t = kCSide - 1; t >= 0; --t) {
        inb[t] = st.mine(h[t]);
        if (t < nh && inb[t] && st.sdec[h[t] - off] >= r) fin = t;
    }
    int best = -1;
    {
        bool und[kCSide];
#pragma unroll
        for (int t = 0; t < kCSide; ++t) und[t] = t < nh && t < fin && !inb[t] && st.word(h[t]) == kUndecided;
#pragma unroll
        for (int t = kCSide - 1; t >= 0; --t)
            if (t < nh && (t == fin || und[t])) best = h[t];
    }
    if (best < 0) {  // no undecided neighbour: unaggregated singleton
        st.sdec[i] = (uint16_t)r;
        S.mate[u] = -1;
        st.publish(u, -1);
        atomicAdd(s_ndec, 1);
        lean_release(st, h, nh, u, A);
        return;
    }
    const int j = best - off;
    const int hdb = st.mine(best) ? C.hdr[j] : kCGlobal;
    if (hdb & kCGlobal) {  // a target outside the tile or without a compact record
        tile_visit_c(S, st, C, r, u, A, s_ndec);
        return;
    }
    const bool settled = st.sdec[j] != kTilePend;
    const int nhb = hdb & 7, nlb = (hdb >> 3) & 7;
    int hb[kCSide], lb[kCSide];
#pragma unroll
    for (int t = 0; t < kCSide; ++t) {
        hb[t] = best + C.h[t * kTileCRows + j];
        lb[t] = best + C.l[t * kTileCRows + j];
    }
    // back: the target's smallest undecided lower edge-neighbour; named: one
    // of its lower-tile neighbours below back took it (read only while the
    // target is pending)
    int back = -1;
    bool named = false;
    {
        int d[kCSide];
        bool nm[kCSide];
#pragma unroll
        for (int t = 0; t < kCSide; ++t) {
            d[t] = -1;
            nm[t] = false;
            if (t < nlb) {
                const int x = lb[t];
                if (x >= off) {
                    d[t] = st.sdec[x - off];
                } else if (!settled) {
                    const int wx = st.word(x);
                    d[t] = wx == kUndecided ? INT_MAX : -1;
                    nm[t] = wx == best + 2;
                }
            }
        }
#pragma unroll
        for (int t = kCSide - 1; t >= 0; --t)
            if (t < nlb && d[t] >= r) back = lb[t];
#pragma unroll
        for (int t = 0; t < kCSide; ++t)
            if (t < nlb && nm[t] && (back < 0 || lb[t] < back)) named = true;
    }
    if (back != u) {
        A.push(u);  // still ready, retry next round
        return;
    }
    if (!settled) {  // a pending target: settle it (free, or taken from a lower tile)
        const int old = cas_stamp(st.sdec, j, kTilePend, named ? r - 1 : kTileUnd);
        if (old == kTilePend) {
            if (named) {
                atomicAdd(s_ndec, 1);
                lean_release(st, hb, nhb, best, A);
                A.push(u);
                return;
            }
        } else if (old != kTileUnd) {
            A.push(u);
            return;
        }
    }
    st.sdec[i] = (uint16_t)r;
    st.sdec[j] = (uint16_t)r;
    S.mate[u] = best;
    S.mate[best] = u;
    st.publish(best, u);
    st.publish(u, best);
    atomicAdd(s_ndec, 2);
    lean_release(st, h, nh, u, A);
    lean_release(st, hb, nhb, best, A);
}
}  // namespace

// Per vertex: the LDS ready counter (lcnt: undecided lower edge-neighbours in
// its own tile) and kExposed when it has lower edge-neighbours in lower
// tiles.  After k_hem_init.  A counter beyond 16 bits sets cnt[7] (the pass
// then runs the round kernels).
__global__ __launch_bounds__(BS) void k_hem_tile_prep(int n, int T, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const uint8_t* __restrict__ lowok,
                                                      int* __restrict__ lcnt, int* cnt) {
    const int y = blockIdx.x * BS + threadIdx.x;
    if (y >= n) return;
    const int t0 = (y / T) * T;
    int cross = 0;
    for (int k = rp[y]; k < rp[y + 1]; ++k) {
        if (ci[k] >= t0) break;  // columns ascend
        cross += lowok[k];
    }
    const int c = lcnt[y] - cross;
    if (c > 0xffff) atomicOr(&cnt[7], 2);
    lcnt[y] = c | (cross > 0 ? kExposed : 0);
}

// One workgroup per tile.  gl0/gl1: global list space (the tile's rows of
// each); tmo: time limit in wall-clock ticks.  COMPACT: tiles of at most
// kTileCRows rows with their records in LDS (SIDE 7).
template <int SIDE, bool COMPACT>
__global__ __launch_bounds__(hem_nt<SIDE>()) void k_hem_tile(int n, int T, HemState S, int* dec_g,
                                                      const int* __restrict__ lcnt_g, int* gl0, int* gl1, int* cnt,
                                                      long long tmo) {
    static_assert(!COMPACT || SIDE == 7, "compact records hold 7-entry records");
    constexpr int TR = COMPACT ? kTileCRows : kHemTileRows;
    constexpr int CR = COMPACT ? kTileCRows : 1;
    __shared__ uint16_t s_dec[TR];
    __shared__ unsigned s_lcnt2[TR / 2];
    __shared__ uint16_t s_la[TL_LCAP], s_lb[TL_LCAP];
    __shared__ uint8_t c_hdr[CR];
    __shared__ int16_t c_h[kCSide * CR], c_l[kCSide * CR];
    __shared__ int s_cnt, s_gnext, s_ndec, s_stop;
    const long long t_start = wall_clock64();
    if (cnt[7] & 2) return;  // a counter beyond 16 bits: the host repeats the pass with rounds
    const int off = blockIdx.x * T;
    const int m = min(T, n - off);
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_gnext = 0;
        s_ndec = 0;
        s_stop = 0;
    }
    __syncthreads();
    // Vertices decided before the pass (dec_g -1: systems of another driver)
    // count as done (LDS stamp 0); lower tiles may already publish others.
    int pre = 0;
    for (int i = threadIdx.x; i < m; i += hem_nt<SIDE>()) {
        const bool done = dec_g[off + i] == -1;
        pre += done;
        s_dec[i] = (uint16_t)(done ? 0 : ((lcnt_g[off + i] & kExposed) ? kTilePend : kTileUnd));
    }
    for (int i = threadIdx.x; 2 * i < m; i += hem_nt<SIDE>()) {
        const unsigned lo = (unsigned)lcnt_g[off + 2 * i] & 0xffffu;
        const unsigned hi = 2 * i + 1 < m ? (unsigned)lcnt_g[off + 2 * i + 1] & 0xffffu : 0u;
        s_lcnt2[i] = lo | (hi << 16);
    }
    if (pre) atomicAdd(&s_ndec, pre);
    if (COMPACT) {  // compact copies of the tile's records
        const HemRecT<7>* __restrict__ g = static_cast<const HemRecT<7>*>(S.rec);
        for (int i = threadIdx.x; i < m; i += hem_nt<SIDE>()) {
            const int v = off + i;
            const HemRecT<7> R = g[v];
            const int nh = R.hdr & 255, nl = (R.hdr >> 8) & 255;
            bool fit = !(R.hdr & kRecOverflow) && nh <= kCSide && nl <= kCSide;
            int16_t dh[kCSide], dl[kCSide];
#pragma unroll
            for (int t = 0; t < kCSide; ++t) {
                const int a = t < nh ? R.h[t] - v : 0, b = t < nl ? R.l[t] - v : 0;
                fit = fit && a >= -32768 && a <= 32767 && b >= -32768 && b <= 32767;
                dh[t] = (int16_t)a;
                dl[t] = (int16_t)b;
            }
#pragma unroll
            for (int t = 0; t < kCSide; ++t) {
                c_h[t * CR + i] = dh[t];
                c_l[t * CR + i] = dl[t];
            }
            c_hdr[i] = (uint8_t)(fit ? nh | (nl << 3) : kCGlobal);
        }
    }
    __syncthreads();
    const TileSt st{s_dec, s_lcnt2, off, m, dec_g};
    const CRecs C{c_hdr, c_h, c_l, static_cast<const HemRecT<7>*>(S.rec), off, COMPACT ? m : 0};
    int* gin = gl0 + off;
    int* gout = gl1 + off;
    uint16_t* cur = s_la;
    uint16_t* nxt = s_lb;
    int kl, kg;
    {  // the first list: undecided vertices without undecided lower neighbours in the tile
        const Appender<uint16_t> A{cur, &s_cnt, TL_LCAP, gin, &s_gnext, off};
        for (int i = threadIdx.x; i < m; i += hem_nt<SIDE>())
            if (s_dec[i] != 0 && (lcnt_g[off + i] & 0xffff) == 0) A.push(off + i);
        __syncthreads();
        kl = min(s_cnt, TL_LCAP);
        kg = s_gnext;
        __syncthreads();
    }
    int r = 2;  // stamps r - 1 >= 1 mark vertices found taken
    bool stop = s_ndec >= m;
    while (!stop) {
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_gnext = 0;
        }
        __syncthreads();
        const Appender<uint16_t> A{nxt, &s_cnt, TL_LCAP, gout, &s_gnext, off};
        const int klc = kl;
        // compact tiles: the round's first items go to wave r mod (waves), so
        // the wave that visited in the previous round, whose stores may still
        // be in flight, does not wait for them at its first memory access
        constexpr int NW = hem_nt<SIDE>() / kWave;
        const int first = COMPACT ? (int)((threadIdx.x + (unsigned)(NW - r % NW) * kWave) % hem_nt<SIDE>())
                                  : (int)threadIdx.x;
        for (int idx = first; idx < kl + kg; idx += hem_nt<SIDE>()) {
            const int u = idx < klc ? (int)cur[idx] + off : gin[idx - klc];
            if (COMPACT) tile_visit_lean(S, st, C, r, u, A, &s_ndec);
            else tile_visit<SIDE>(S, st, r, u, A, &s_ndec);
        }
        if (threadIdx.x == 0 && (r & 31) == 0 && (wall_clock64() - t_start > tmo || r >= kTileMaxRound))
            s_stop = 1;
        __syncthreads();
        kl = min(s_cnt, TL_LCAP);
        kg = s_gnext;
        stop = s_ndec >= m || s_stop != 0;
        __syncthreads();  // every thread has read the counts before the next reset
        uint16_t* t = cur;
        cur = nxt;
        nxt = t;
        int* tg = gin;
        gin = gout;
        gout = tg;
        ++r;
    }
    if (threadIdx.x == 0) {
        atomicMax(&cnt[6], r - 2);
        if (s_ndec < m) atomicOr(&cnt[7], 1);
    }
}

// ---------------------------------------------------------------------------
// Edge-based matching (Algorithm 3): the greedy matching over undirected
// edges {u, v} in increasing key (-W_uv, min(u,v), max(u,v)), where W_uv is
// the heavier of |a_uv| and |a_vu| (the first occurrence of the pair in the
// sorted edge list).  Same rounds of locally dominant edges, for this key:
// every undecided vertex points to its best edge to an undecided neighbour;
// mutual pointers match; a vertex with no undecided neighbour is a
// singleton.  A pointer changes only when a neighbour is decided, so each
// round recomputes the pointers of the vertices next to the previous round's
// decisions ("dirty"), then (after a launch boundary) matches mutual pairs.
// ---------------------------------------------------------------------------
namespace {
struct EdgeKey {
    double w;
    int lo, hi;
    __device__ __forceinline__ bool better(const EdgeKey& o) const {  // smaller key
        if (w != o.w) return w > o.w;
        if (lo != o.lo) return lo < o.lo;
        return hi < o.hi;
    }
};
}  // namespace

__global__ __launch_bounds__(BS) void k_ehem_init(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double* __restrict__ v, double* __restrict__ wsym,
                                                  int* __restrict__ dec, int* __restrict__ mate,
                                                  int* __restrict__ ptr, int* __restrict__ stamp,
                                                  int* __restrict__ wl0, int* cnt, int* err) {
    const int u = blockIdx.x * BS + threadIdx.x;
    if (u >= n) return;
    dec[u] = kUndecided;
    mate[u] = -1;
    ptr[u] = -1;
    stamp[u] = -1;
    wl0[u] = u;  // every vertex starts dirty
    if (u == 0) cnt[0] = n;
    bool bad = false;
    for (int e = rp[u]; e < rp[u + 1]; ++e) {
        const int x = ci[e];
        double w = 0.0;
        if (x != u) {
            const int pos = find_col(ci, rp[x], rp[x + 1], u);
            if (pos < 0) bad = true;
            const double back = pos >= 0 ? fabs(v[pos]) : 0.0;
            const double fwd = fabs(v[e]);
            w = fwd > back ? fwd : back;
        }
        wsym[e] = w;
    }
    if (bad) atomicOr(err, ERR_NONSYM);
}

// pointer of each dirty undecided vertex (state at the start of the round)
__global__ __launch_bounds__(BS) void k_ehem_point(int r, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ wsym, const int* __restrict__ dec,
                                                   int* __restrict__ ptr, const int* __restrict__ win, int* cnt,
                                                   int slot_in, int zero_w) {
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[zero_w] = 0;
    const int m = cnt[slot_in];
    if (m > 0 && blockIdx.x == 0 && threadIdx.x == 0) cnt[6] = r + 1;  // rounds with work
    for (int idx = blockIdx.x * BS + threadIdx.x; idx < m; idx += gridDim.x * BS) {
        const int u = win[idx];
        if (dec[u] != kUndecided) continue;
        EdgeKey best{-1.0, 0, 0};
        int bv = -1;
        for (int e = rp[u]; e < rp[u + 1]; ++e) {
            const int x = ci[e];
            const double w = wsym[e];
            if (x == u || w == 0.0 || dec[x] != kUndecided) continue;
            const EdgeKey k{w, min(u, x), max(u, x)};
            if (bv < 0 || k.better(best)) {
                best = k;
                bv = x;
            }
        }
        ptr[u] = bv;
    }
}

// mutual pointers match; the undecided neighbours of each decision are the
// next round's dirty vertices (marked once per round through the stamps)
__global__ __launch_bounds__(BS) void k_ehem_match(int r, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ wsym, int* __restrict__ dec,
                                                   int* __restrict__ mate, const int* __restrict__ ptr,
                                                   int* __restrict__ stamp, const int* __restrict__ win,
                                                   int* __restrict__ wout, int* cnt, int slot_in, int slot_out) {
    const int m = cnt[slot_in];
    for (int idx = blockIdx.x * BS + threadIdx.x; idx < m; idx += gridDim.x * BS) {
        const int u = win[idx];
        if (dec[u] != kUndecided) continue;
        const int v = ptr[u];
        if (v < 0) {  // no undecided neighbour: unaggregated singleton
            dec[u] = r;
            mate[u] = -1;
            continue;
        }
        if (ptr[v] != u) continue;
        // matched (found by u, and by v too if v is dirty: identical writes)
        dec[u] = r;
        dec[v] = r;
        mate[u] = v;
        mate[v] = u;
        for (int q = 0; q < 2; ++q) {
            const int x = q == 0 ? u : v;
            for (int e = rp[x]; e < rp[x + 1]; ++e) {
                const int y = ci[e];
                if (y == x || wsym[e] == 0.0) continue;
                if (atomicExch(&stamp[y], r) != r) wout[atomicAdd(&cnt[slot_out], 1)] = y;
            }
        }
    }
}

void launch_ehem_init(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
    hipLaunchKernelGGL(k_ehem_init, dim3(blocks_for(n)), dim3(BS), 0, s, n, rp, ci, v, w.wsym, w.dec, w.mate,
                       w.ptr, w.lcnt, w.wl[0], w.cnt, w.err);
}

void launch_ehem_round(int r, int n, const int* rp, const int* ci, HemWork& w, hipStream_t s) {
    const int g = blocks_for(n, BS, 4 * w.round_grid);
    hipLaunchKernelGGL(k_ehem_point, dim3(g), dim3(BS), 0, s, r, rp, ci, w.wsym, w.dec, w.ptr, w.wl[r & 1], w.cnt,
                       r % 3, (r + 2) % 3);
    hipLaunchKernelGGL(k_ehem_match, dim3(g), dim3(BS), 0, s, r, rp, ci, w.wsym, w.dec, w.mate, w.ptr, w.lcnt,
                       w.wl[r & 1], w.wl[(r + 1) & 1], w.cnt, r % 3, (r + 1) % 3);
}

// ---------------------------------------------------------------------------
// Matching from the last index (Section 2.1.1): vertices visited downward and
// row entries scanned downward, ties to the highest index.  Renumbering
// i -> n-1-i turns this into the upward pass, so it runs the kernels above on
// the mirrored matrix and maps the pairs back.  Mirroring reverses the order
// of the rows and, with it, of the entries inside each row: the column and
// value arrays are read backwards as a whole and the columns stay ascending.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_mirror_csr(int n, int64_t nnz, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const double* __restrict__ v,
                                                   int* __restrict__ mrp, int* __restrict__ mci,
                                                   double* __restrict__ mv) {
    const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (e < nnz) {
        mci[e] = n - 1 - ci[nnz - 1 - e];
        mv[e] = v[nnz - 1 - e];
    }
    if (e <= n) mrp[e] = (int)(nnz - rp[n - e]);
}

__global__ __launch_bounds__(BS) void k_unmirror_mate(int n, const int* __restrict__ mr, int* __restrict__ mate) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const int m = mr[n - 1 - i];
    mate[i] = m < 0 ? -1 : n - 1 - m;
}

void launch_mirror_csr(int n, int64_t nnz, const int* rp, const int* ci, const double* v, int* mrp, int* mci,
                       double* mv, hipStream_t s) {
    const int64_t work = nnz > (int64_t)n + 1 ? nnz : (int64_t)n + 1;
    hipLaunchKernelGGL(k_mirror_csr, dim3(blocks_for(work)), dim3(BS), 0, s, n, nnz, rp, ci, v, mrp, mci, mv);
}

void launch_unmirror_mate(int n, const int* mr, int* mate, hipStream_t s) {
    hipLaunchKernelGGL(k_unmirror_mate, dim3(blocks_for(n)), dim3(BS), 0, s, n, mr, mate);
}

#define AMG_HEM_SIDE(side, CALL) \
    switch (side) {                \
        case 7: CALL(7); break;    \
        case 15: CALL(15); break;  \
        default: CALL(31); break;  \
    }

void launch_hem_init(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
#define CALL(SD)                                                                                  \
    hipLaunchKernelGGL(k_hem_init<SD>, dim3(blocks_for(n)), dim3(BS), 0, s, n, rp, ci, v, w.lowok, \
                       static_cast<HemRecT<SD>*>(w.rec), w.lcnt, w.dec, w.mate, w.wl[0], w.cnt, w.err)
    AMG_HEM_SIDE(w.side, CALL)
#undef CALL
}

int hem_next_count_slot(int round) { return round % 3; }

void launch_hem_round(int r, int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
    const int g = blocks_for(n, HEM_BS, w.round_grid);
    const HemState S{rp, ci, v, w.lowok, w.rec, w.mate};
#define CALL(SD)                                                                                            \
    hipLaunchKernelGGL(k_hem_round<SD>, dim3(g), dim3(HEM_BS), 0, s, r, n, S, w.dec, w.lcnt, w.wl[r & 1],    \
                       w.wl[(r + 1) & 1], w.cnt, r % 3, (r + 1) % 3, (r + 2) % 3)
    AMG_HEM_SIDE(w.side, CALL)
#undef CALL
}

void launch_hem_lds_seg(int nseg, const int2* seg, const int* rp, const int* ci, const double* v, HemWork& w,
                        int* sl0, int* sl1, hipStream_t s) {
    if (nseg <= 0) return;
    const HemState S{rp, ci, v, w.lowok, w.rec, w.mate};
#define CALL(SD)                                                                                                 \
    hipLaunchKernelGGL(k_hem_lds_seg<SD>, dim3(nseg), dim3(hem_nt<SD>()), 0, s, seg, S, w.lcnt, w.dec, sl0, sl1, \
                       w.cnt, w.lds_rows < kHemLdsRows ? w.lds_rows : kHemLdsRows)
    AMG_HEM_SIDE(w.side, CALL)
#undef CALL
}

// Rows of system j of a pass from the previous pass's aggregate map: the
// systems start at rows off[j] of the previous operator, so in this one at
// agg[off[j]]; with mirror the operator is numbered backwards (n rows).
__global__ __launch_bounds__(BS) void k_seg_table(int m, const int* __restrict__ off, const int* __restrict__ agg,
                                                  int n, int mirror, int2* __restrict__ seg) {
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= m) return;
    const int a = off[j] >= 0 ? agg[off[j]] : 0;
    const int b = j + 1 < m ? agg[off[j + 1]] : n;
    seg[j] = mirror ? make_int2(n - b, b - a) : make_int2(a, b - a);
}

void launch_seg_table(int m, const int* off, const int* agg, int n, bool mirror, int2* seg, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_table, dim3(blocks_for(m)), dim3(BS), 0, s, m, off, agg, n, mirror ? 1 : 0, seg);
}

void launch_hem_tile(int n, int64_t nnz, const int* rp, const int* ci, const double* v, HemWork& w, long long tmo,
                     hipStream_t s) {
    // Small tiles with LDS copies of the records cut the cost of a round but
    // multiply the vertices whose lower neighbours lie in other tiles, and a
    // step across tiles costs several rounds.  As measured on MI355X they pay
    // for passes of short rows (at most 8 entries on average, so nearly every
    // record fits) of at most 512 tiles; more tiles cannot all be resident at
    // once (one workgroup per compute unit), so a tile would wait for a lower
    // one to finish, and on the long chains of such passes that loses.
    const int Tc = w.tile_c_rows < kTileCRows ? w.tile_c_rows : kTileCRows;
    const int64_t ntc = Tc > 0 ? ((int64_t)n + Tc - 1) / Tc : 0;
    const bool compact = w.side == 7 && Tc > 0 && nnz <= 8 * (int64_t)n &&
                         (w.tile_c_rows < kTileCRows || ntc <= kCompactMaxTiles);
    const int T = compact ? Tc : w.tile_rows;
    const int nt = (n + T - 1) / T;
    hipLaunchKernelGGL(k_hem_tile_prep, dim3(blocks_for(n)), dim3(BS), 0, s, n, T, rp, ci, w.lowok, w.lcnt, w.cnt);
    const HemState S{rp, ci, v, w.lowok, w.rec, w.mate};
#define CALL(SD, CP)                                                                                              \
    hipLaunchKernelGGL((k_hem_tile<SD, CP>), dim3(nt), dim3(hem_nt<SD>()), 0, s, n, T, S, w.dec, w.lcnt, w.wl[0], \
                       w.wl[1], w.cnt, tmo)
    if (compact) CALL(7, true);
    else if (w.side == 7) CALL(7, false);
    else CALL(15, false);  // records of tiled passes hold at most 15 entries a side
#undef CALL
}

void launch_hem_all(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s) {
    const HemState S{rp, ci, v, w.lowok, w.rec, w.mate};
    if (n <= w.lds_rows) {
#define CALL(SD) \
    hipLaunchKernelGGL(k_hem_lds<SD>, dim3(1), dim3(hem_nt<SD>()), 0, s, n, S, w.lcnt, w.wl[0], w.wl[1], w.cnt)
        AMG_HEM_SIDE(w.side, CALL)
#undef CALL
    } else {
#define CALL(SD) \
    hipLaunchKernelGGL(k_hem_all<SD>, dim3(1), dim3(hem_nt<SD>()), 0, s, n, S, w.dec, w.lcnt, w.wl[0], w.wl[1], w.cnt)
        AMG_HEM_SIDE(w.side, CALL)
#undef CALL
    }
}
#undef AMG_HEM_SIDE

}  // namespace amg
