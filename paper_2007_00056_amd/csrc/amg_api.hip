// Host orchestration and C ABI (include/hemamg.h): the setup phase (Section 3)
// building the hierarchy level by level on the GPU, the V-cycle driver
// (Algorithm 1) and the Krylov drivers (Algorithms 4 and 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "amg_host.hpp"

namespace amg {

namespace {
// per-device free lists of streams and events
struct DeviceRes {
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events[2];  // [0] without timing, [1] timing
};
std::mutex g_res_mu;
std::map<int, DeviceRes> g_res;
}  // namespace

int current_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

// Pinned host blocks of 4 KiB for the Krylov scalar slots of a handle, kept
// in a free list for the process (pinned allocation and release are slow).
namespace {
std::mutex g_pinned_mu;
std::vector<void*> g_pinned_free;
}  // namespace

void* pinned_get() {
    {
        std::lock_guard<std::mutex> g(g_pinned_mu);
        if (!g_pinned_free.empty()) {
            void* p = g_pinned_free.back();
            g_pinned_free.pop_back();
            return p;
        }
    }
    // mapped into the device and coherent: kernels may write slots straight
    // into it, and the host reads them once the stream has finished
    void* p = nullptr;
    HIPCHK(hipHostMalloc(&p, kPinnedBlock, hipHostMallocMapped | hipHostMallocCoherent));
    return p;
}

void pinned_put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(g_pinned_mu);
    g_pinned_free.push_back(p);
}

hipStream_t stream_get() {
    {
        std::lock_guard<std::mutex> g(g_res_mu);
        auto& v = g_res[current_device()].streams;
        if (!v.empty()) {
            hipStream_t s = v.back();
            v.pop_back();
            return s;
        }
    }
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
}

void stream_put(hipStream_t s) {
    if (!s) return;
    std::lock_guard<std::mutex> g(g_res_mu);
    g_res[current_device()].streams.push_back(s);
}

namespace {
struct KeptChunk {
    void* p;
    size_t bytes;
    hipEvent_t ev;  // recorded on the stream that last used the chunk
};
std::mutex g_chunk_mu;
std::map<int, std::vector<KeptChunk>> g_chunks;  // per device, oldest first
std::map<int, size_t> g_chunk_bytes;
}  // namespace

size_t chunk_cache_cap() {
    static std::mutex mu;
    static std::map<int, size_t> caps;
    const int d = current_device();
    std::lock_guard<std::mutex> g(mu);
    auto it = caps.find(d);
    if (it != caps.end()) return it->second;
    size_t total = 0;
    if (hipDeviceTotalMem(&total, d) != hipSuccess) {
        (void)hipGetLastError();
        total = 0;
    }
    const size_t cap = std::min(total / 4, size_t(64) << 30);
    caps[d] = cap;
    return cap;
}

bool chunk_keep(void* p, size_t bytes, hipStream_t s) {
    const int d = current_device();
    const size_t cap = chunk_cache_cap();
    if (bytes > cap) return false;
    hipEvent_t ev = event_get(false);
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipGetLastError();
        event_put(ev, false);
        return false;
    }
    std::vector<KeptChunk> evict;
    {
        std::lock_guard<std::mutex> g(g_chunk_mu);
        auto& v = g_chunks[d];
        size_t& tot = g_chunk_bytes[d];
        v.push_back(KeptChunk{p, bytes, ev});
        tot += bytes;
        while (tot > cap) {  // the oldest go back to the pool
            evict.push_back(v.front());
            tot -= v.front().bytes;
            v.erase(v.begin());
        }
    }
    for (KeptChunk& k : evict) {
        (void)hipStreamWaitEvent(s, k.ev, 0);
        (void)hipFreeAsync(k.p, s);
        event_put(k.ev, false);
    }
    return true;
}

void* chunk_take(size_t bytes, hipStream_t s) {
    const int d = current_device();
    KeptChunk k{nullptr, 0, nullptr};
    {
        std::lock_guard<std::mutex> g(g_chunk_mu);
        auto& v = g_chunks[d];
        for (size_t i = v.size(); i-- > 0;)
            if (v[i].bytes == bytes) {
                k = v[i];
                v.erase(v.begin() + (std::ptrdiff_t)i);
                g_chunk_bytes[d] -= bytes;
                break;
            }
    }
    if (!k.p) return nullptr;
    HIPCHK(hipStreamWaitEvent(s, k.ev, 0));
    event_put(k.ev, false);
    return k.p;
}

size_t chunk_kept_bytes() {
    const int d = current_device();
    std::lock_guard<std::mutex> g(g_chunk_mu);
    auto it = g_chunk_bytes.find(d);
    return it == g_chunk_bytes.end() ? 0 : it->second;
}

void chunk_flush() {
    const int d = current_device();
    std::vector<KeptChunk> all;
    {
        std::lock_guard<std::mutex> g(g_chunk_mu);
        all.swap(g_chunks[d]);
        g_chunk_bytes[d] = 0;
    }
    for (KeptChunk& k : all) {
        (void)hipEventSynchronize(k.ev);
        (void)hipFreeAsync(k.p, nullptr);
        event_put(k.ev, false);
    }
    if (!all.empty()) (void)hipStreamSynchronize(nullptr);
}

hipEvent_t event_get(bool timing) {
    {
        std::lock_guard<std::mutex> g(g_res_mu);
        auto& v = g_res[current_device()].events[timing ? 1 : 0];
        if (!v.empty()) {
            hipEvent_t e = v.back();
            v.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, timing ? hipEventDisableSystemFence : hipEventDisableTiming));
    return e;
}

void event_put(hipEvent_t e, bool timing) {
    if (!e) return;
    std::lock_guard<std::mutex> g(g_res_mu);
    g_res[current_device()].events[timing ? 1 : 0].push_back(e);
}

// Pinned host words for small read-backs (per thread, kept for the process).
int* pinned_words(int** dev) {
    thread_local int* p = nullptr;
    thread_local int* d = nullptr;
    if (!p) {
        HIPCHK(hipHostMalloc((void**)&p, 64 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&d), p, 0));
    }
    if (dev) *dev = d;
    return p;
}

int read_int(const int* d, hipStream_t s) {
    int* h = pinned_words();
    HIPCHK(hipMemcpyAsync(h, d, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return h[0];
}

void raise_err_word(int e, const char* where) {
    if (e & ERR_NONFINITE) raise(AMG_ENOTFINITE, "%s: matrix has a NaN or Inf value", where);
    if (e & ERR_STRUCT) raise(AMG_EINVAL, "%s: invalid CSR structure (row_ptr, column range or order)", where);
    if (e & ERR_DIAG) raise(AMG_EINVAL, "%s: a diagonal entry is missing or zero", where);
    if (e & ERR_NONSYM) raise(AMG_EINVAL, "%s: sparsity pattern is not structurally symmetric", where);
    if (e & ERR_SINGULAR) raise(AMG_ESINGULAR, "%s: coarsest matrix is singular", where);
}

void check_err_word(const int* err, hipStream_t s, const char* where) { raise_err_word(read_int(err, s), where); }

void validate_params(const amg_params& p) {
    if (p.passes_per_level < 1 || p.passes_per_level > 2) raise(AMG_EINVAL, "passes_per_level must be 1 or 2");
    if (p.max_coarse_rows < 1 || p.max_coarse_rows > kDenseMaxRows)
        raise(AMG_EINVAL, "max_coarse_rows must be in 1..%d", kDenseMaxRows);
    if (p.max_dense_rows < 1 || p.max_dense_rows > kDenseMaxRows)
        raise(AMG_EINVAL, "max_dense_rows must be in 1..%d", kDenseMaxRows);
    if (p.max_levels < 1 || p.max_levels > 64) raise(AMG_EINVAL, "max_levels must be in 1..64");
    if (p.pre < 0 || p.pre > 8 || p.post < 0 || p.post > 8) raise(AMG_EINVAL, "pre/post sweeps must be in 0..8");
    if (!std::isfinite(p.omega)) raise(AMG_EINVAL, "omega must be finite");
    if (p.true_res_period < 0) raise(AMG_EINVAL, "true_res_period must be >= 0");
    if (p.precond_fp32 != 0 && p.precond_fp32 != 1) raise(AMG_EINVAL, "precond_fp32 must be 0 or 1");
    if (!(p.stall_ratio > 0.0 && p.stall_ratio <= 1.0)) raise(AMG_EINVAL, "stall_ratio must be in (0, 1]");
    if (p.hem != 0 && p.hem != 1) raise(AMG_EINVAL, "hem must be 0 (node-based) or 1 (edge-based)");
    if (p.alternate != 0 && p.alternate != 1) raise(AMG_EINVAL, "alternate must be 0 or 1");
    if (p.alternate && p.hem != 0) raise(AMG_EINVAL, "alternate applies to node-based matching (hem = 0)");
    if (p.precond_fp32 && !(p.pre == 1 && p.post == 1))
        raise(AMG_EINVAL, "a float preconditioner needs one pre- and one post-sweep");
}

}  // namespace amg

namespace {

using namespace amg;

struct Csr {
    int n = 0;
    int64_t nnz = 0;
    int* rp = nullptr;
    int* ci = nullptr;
    double* v = nullptr;
};

// Buffers reused by every matching pass and Galerkin product of a setup,
// sized for level 0 (every later pass is smaller).
struct SetupWork {
    HemWork hw{};
    int* mate[2]{};
    int* agg[2]{};
    int* lead[2]{};
    int* flag = nullptr;
    int* ids = nullptr;
    int* stmp = nullptr;
    int* rowcnt = nullptr;
    int* ovf = nullptr;
    int* novf = nullptr;
    int* hc = nullptr;  // pinned: worklist sizes read back between batches
    hipEvent_t ev[2]{};
    int hem_small = 65536;  // passes on at most this many rows run in one workgroup
    bool tile_strict = false;  // a tiled pass past its time limit is an error (tests), not repeated

    bool edge = false;  // edge-based matching (Algorithm 3)
    int* mrp = nullptr;  // mirrored matrix of a pass from the last index
    int* mci = nullptr;
    double* mv = nullptr;

    void init(int n, int64_t nnz, DevPool& P, int* err, bool edge_based, bool alternate) {
        edge = edge_based;
        if (edge) {
            hw.wsym = P.get<double>((size_t)nnz);
            hw.ptr = P.get<int>(n);
        }
        if (alternate) {  // every later pass has at most n rows and nnz entries
            mrp = P.get<int>((size_t)n + 1);
            mci = P.get<int>((size_t)nnz);
            mv = P.get<double>((size_t)nnz);
        }
        hw.lowok = P.get<uint8_t>((size_t)nnz);
        hw.rec_bytes = sizeof(HemRecT<7>) * (size_t)n;
        hw.rec = P.get<char>(hw.rec_bytes);
        hw.side = 7;
        hw.lcnt = P.get<int>(n);
        hw.dec = P.get<int>(n);
        hw.wl[0] = P.get<int>(n);
        hw.wl[1] = P.get<int>(n);
        hw.cnt = P.get<int>(8);
        hw.err = err;
        for (int t = 0; t < 2; ++t) {
            mate[t] = P.get<int>(n);
            agg[t] = P.get<int>(n);
            lead[t] = P.get<int>(n);
        }
        flag = P.get<int>(n);
        ids = P.get<int>((size_t)n + 1);
        stmp = P.get<int>(scan_tmp_ints(n));
        rowcnt = P.get<int>(n);
        ovf = P.get<int>(n);
        novf = P.get<int>(1);
        hc = pinned_words() + 32;  // this thread's pinned words, past the read-back area
        ev[0] = event_get(false);
        ev[1] = event_get(false);
        if (const char* e = getenv("HEMAMG_HEM_SMALL")) hem_small = atoi(e);  // tuning sweeps
        if (const char* e = getenv("HEMAMG_HEM_GRID")) hw.round_grid = atoi(e) > 0 ? atoi(e) : 96;
        if (const char* e = getenv("HEMAMG_HEM_LDS")) hw.lds_rows = atoi(e) < kHemLdsRows ? atoi(e) : kHemLdsRows;
        if (const char* e = getenv("HEMAMG_TILE_STRICT")) tile_strict = atoi(e) != 0;
        if (const char* e = getenv("HEMAMG_HEM_TILE"))  // rows per tile; 0: no tiled passes
            hw.tile_rows = atoi(e) <= 0 ? 0 : (atoi(e) < kHemTileRows ? atoi(e) : kHemTileRows);
        if (const char* e = getenv("HEMAMG_HEM_TILE_C"))  // rows per LDS-record tile; 0: not used
            hw.tile_c_rows = atoi(e) <= 0 ? 0 : (atoi(e) < kHemTileCRows ? atoi(e) : kHemTileCRows);
    }
    ~SetupWork() {
        event_put(ev[0], false);
        event_put(ev[1], false);
    }
};

// One matching pass on B (Algorithm 2) into slot t: mate, aggregate map and
// the smaller vertex (leader) of each aggregate.
struct Pass {
    int* mate = nullptr;
    int* agg = nullptr;
    int* lead = nullptr;
    int* cnt = nullptr;  // matching counters (device)
    int n = 0;           // fine rows
    int nc = 0;          // coarse rows, known after the Galerkin count
    int rounds = 0;
};

// Matching rounds launched in batches; the size of the next worklist is
// copied back after each batch and checked one batch later, so the host
// check overlaps the GPU work.  Rounds with an empty worklist do nothing.
template <class Launch>
void run_rounds(SetupWork& W, HemWork& w, int n, hipStream_t s, Launch&& launch_round) {
    const int batch = 16;
    int r = 0;
    for (int j = 0;; ++j) {
        for (int b = 0; b < batch; ++b, ++r) launch_round(r);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&W.hc[j & 1], w.cnt + hem_next_count_slot(r), sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(W.ev[j & 1], s));
        if (j >= 1) {
            HIPCHK(hipEventSynchronize(W.ev[(j - 1) & 1]));
            if (W.hc[(j - 1) & 1] == 0) break;
        }
        if (r > n + 4 * batch) raise(AMG_EHIP, "matching did not terminate (internal error)");
    }
}

// Time limit of a tiled pass in wall-clock ticks (250 ms; a pass of a few
// million rows takes a few milliseconds).
long long tile_timeout_ticks() {
    thread_local int dev = -1;
    thread_local long long ticks = 0;
    int d = 0;
    HIPCHK(hipGetDevice(&d));
    if (d != dev) {
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d));
        ticks = (long long)(khz > 0 ? khz : 100000) * 250;
        dev = d;
    }
    return ticks;
}

bool tiled(const HemWork& w, int n) {
    return w.tile_rows > 0 && ((int64_t)n + w.tile_rows - 1) / w.tile_rows <= kHemMaxTiles;
}

// A tiled pass; false when it did not finish (the caller repeats the pass).
bool run_tiles(SetupWork& W, HemWork& w, const Csr& B, hipStream_t s) {
    launch_hem_tile(B.n, B.nnz, B.rp, B.ci, B.v, w, tile_timeout_ticks(), s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&W.hc[2], w.cnt + 7, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return W.hc[2] == 0;
}

// Systems of a batched setup inside the operator of a pass: seg = device table
// of (first row, rows) in the pass's numbering.  Systems up to the LDS limit
// are matched one workgroup each; the round kernels run only for larger ones.
struct SegPass {
    const int2* seg = nullptr;
    int nseg = 0;
    bool all_small = false;
    int* sl[2] = {nullptr, nullptr};  // list space, a row per vertex each
};

// from_last: the pass starts from the last index (run on the mirrored matrix,
// its pairs mapped back before numbering).
Pass hem_pass(const Csr& Bin, SetupWork& W, int t, hipStream_t s, int* err, bool from_last,
              const SegPass* sp = nullptr) {
    const int n = Bin.n;
    Csr B = Bin;
    HemWork w = W.hw;
    w.mate = W.mate[t];
    if (from_last) {
        launch_mirror_csr(n, Bin.nnz, Bin.rp, Bin.ci, Bin.v, W.mrp, W.mci, W.mv, s);
        B.rp = W.mrp;
        B.ci = W.mci;
        B.v = W.mv;
        w.mate = W.agg[t];  // free until numbering writes the aggregate map
    }
    // record side from the average row length, within the record buffer
    const double avg = n > 0 ? (double)B.nnz / n : 0.0;
    // workgroup-wide drivers (one workgroup, tiles) take records of at most 15
    w.side = avg <= 9.0 ? 7 : (avg <= 20.0 || n <= W.hem_small || tiled(w, n) ? 15 : 31);
    while (w.side > 7 && (size_t)(w.side + 1) * 8 * (size_t)n > w.rec_bytes) w.side = (w.side + 1) / 2 - 1;
    HIPCHK(hipMemsetAsync(w.cnt, 0, 8 * sizeof(int), s));
    if (W.edge) {
        launch_ehem_init(n, B.rp, B.ci, B.v, w, s);
        run_rounds(W, w, n, s, [&](int r) { launch_ehem_round(r, n, B.rp, B.ci, w, s); });
    } else {
        // small passes: one workgroup with LDS state; larger ones: tiles, else
        // one workgroup with global state or one launch per round
        auto start = [&] {
            launch_hem_init(n, B.rp, B.ci, B.v, w, s);
            if (sp) launch_hem_lds_seg(sp->nseg, sp->seg, B.rp, B.ci, B.v, w, sp->sl[0], sp->sl[1], s);
            HIPCHK(hipGetLastError());
        };
        auto rounds = [&] { run_rounds(W, w, n, s, [&](int r) { launch_hem_round(r, n, B.rp, B.ci, B.v, w, s); }); };
        start();
        if (sp ? sp->all_small : n <= W.hem_small && n <= w.lds_rows) {
            if (!sp) launch_hem_all(n, B.rp, B.ci, B.v, w, s);
        } else if (tiled(w, n)) {
            if (!run_tiles(W, w, B, s)) {  // past its time limit: repeat with the round kernels
                if (W.tile_strict) raise(AMG_EHIP, "tiled matching pass did not finish in time");
                HIPCHK(hipMemsetAsync(w.cnt, 0, 8 * sizeof(int), s));
                start();
                rounds();
            }
        } else if (!sp && n <= W.hem_small) {
            launch_hem_all(n, B.rp, B.ci, B.v, w, s);
        } else {
            rounds();
        }
        HIPCHK(hipGetLastError());
    }
    if (from_last) {
        launch_unmirror_mate(n, w.mate, W.mate[t], s);
        w.mate = W.mate[t];
    }
    Pass P;
    P.mate = w.mate;
    P.agg = W.agg[t];
    P.lead = W.lead[t];
    P.n = n;
    P.cnt = w.cnt;
    // coarse ids: rank of each aggregate's smaller vertex; the count stays on
    // the device until the Galerkin product reads it back with its own sizes
    launch_leader_flags(n, w.mate, W.flag, s);
    launch_scan(W.flag, n, W.ids, W.stmp, s);
    launch_assign_ids(n, w.mate, W.ids, P.agg, P.lead, s);
    HIPCHK(hipGetLastError());
    return P;
}

// Galerkin product of one pass; output buffers from `out`.  The row counts
// are formed over an upper bound of the coarse size (rows past it count 0),
// so one read-back returns the coarse size, its nonzero count, the matching
// counters and the error word together.
Csr galerkin(const Csr& B, Pass& P, SetupWork& W, DevPool& out, hipStream_t s, const int* err) {
    const int nmax = P.n;  // coarse rows <= fine rows
    const int* ncp = W.ids + P.n;
    HIPCHK(hipMemsetAsync(W.novf, 0, sizeof(int), s));
    launch_rap_count(nmax, ncp, P.lead, P.mate, B.rp, B.ci, P.agg, W.rowcnt, W.ovf, W.novf, s);
    launch_rap_count_slow(nmax, W.ovf, W.novf, P.lead, P.mate, B.rp, B.ci, P.agg, W.rowcnt, s);
    Csr C;
    C.rp = out.get<int>((size_t)nmax + 1);
    launch_scan(W.rowcnt, nmax, C.rp, W.stmp, s);
    HIPCHK(hipGetLastError());
    int* dw = nullptr;
    int* hw = pinned_words(&dw);
    launch_pass_words(dw, P.cnt, ncp, C.rp + nmax, err, s);  // one launch in place of four copies
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    raise_err_word(hw[10], "amg_setup");
    if (hw[5] != 0) raise(AMG_EINVAL, "matching: sparsity pattern is not structurally symmetric");
    if (hw[7] != 0) raise(AMG_EHIP, "matching did not terminate (internal error)");
    P.rounds = hw[6];
    P.nc = hw[8];
    C.n = P.nc;
    C.nnz = hw[9];
    C.ci = out.get<int>((size_t)C.nnz);
    C.v = out.get<double>((size_t)C.nnz);
    launch_rap_fill(P.nc, P.lead, P.mate, B.rp, B.ci, B.v, P.agg, C.rp, C.ci, C.v, s);
    launch_rap_fill_slow(P.nc, W.ovf, W.novf, P.lead, P.mate, B.rp, B.ci, B.v, P.agg, C.rp, C.ci, C.v, s);
    HIPCHK(hipGetLastError());
    return C;
}

void alloc_workspace(amg_hier* h) {
    if (h->r) return;
    const int n = h->lev[0].n;
    DevPool& P = h->pool;
    double* v[10];
    for (double*& p : v) p = P.get<double>(n);  // all or none: an allocation failure leaves h->r unset
    h->z = v[1];
    h->pv[0] = v[2];
    h->pv[1] = v[3];
    h->q = v[4];
    h->rb = v[5];
    h->pt = v[6];
    h->sv = v[7];
    h->st = v[8];
    h->t = v[9];
    h->r = v[0];
}

void timer_reserve(Timer& T) {
    if (T.used + 2 > T.ev.size())
        for (int k = 0; k < 64; ++k) T.ev.push_back(event_get(true));
}

void timed_begin(amg_hier* h, int cls, hipStream_t s) {
    Timer& T = h->tim[cls];
    if (!T.on) return;
    timer_reserve(T);
    HIPCHK(hipEventRecord(T.ev[T.used], s));
}

// The next start/stop pair of class cls for a launch that records them
// itself (nullptr when timing is off); timed_end then commits the pair
// without recording.
void timed_pair(amg_hier* h, int cls, hipEvent_t& a, hipEvent_t& b) {
    Timer& T = h->tim[cls];
    a = b = nullptr;
    if (!T.on) return;
    timer_reserve(T);
    a = T.ev[T.used];
    b = T.ev[T.used + 1];
}

void timed_end(amg_hier* h, int cls, hipStream_t s, bool recorded = false) {
    Timer& T = h->tim[cls];
    if (!T.on) return;
    if (!recorded) HIPCHK(hipEventRecord(T.ev[T.used + 1], s));
    T.used += 2;
    if (T.used >= 4096) {  // fold completed pairs to bound the pool
        HIPCHK(hipEventSynchronize(T.ev[T.used - 1]));
        for (size_t k = 0; k < T.used; k += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, T.ev[k], T.ev[k + 1]));
            T.total_ms += ms;
            T.launches += 1;
        }
        T.used = 0;
    }
}

// Whether level L runs the CSR-stream kernels (else the lane-group kernels).
inline bool streamed(const amg_hier* h, const Level& L) { return L.sched < 0 ? L.n >= h->stream_min : L.sched == 0; }

// Whether the level-0 postsmoothing can run as a separate step (part 2).
bool vcycle_splits(const amg_hier* h) { return h->lev.size() > 1 && h->p.pre == 1 && h->p.post == 1; }

template <class T>
VLevel<T> vlevel(const Level& L);
template <>
VLevel<double> vlevel<double>(const Level& L) {
    return VLevel<double>{L.n, L.rp, L.ci, L.v, L.dinv, L.mem, L.sched > 0 ? L.sched : L.lpr, L.rb};
}
template <>
VLevel<float> vlevel<float>(const Level& L) {
    return VLevel<float>{L.n, L.rp, L.ci, L.v32, L.dinv32, L.mem, L.sched > 0 ? L.sched : L.lpr, L.rb};
}
template <class T>
const T* dinv_of(const Level& L);
template <>
const double* dinv_of<double>(const Level& L) {
    return L.dinv;
}
template <>
const float* dinv_of<float>(const Level& L) {
    return L.dinv32;
}

// Algorithm 1 with one pre- and one post-sweep, in value type T.  r and z are
// double; g0 (T), if given, already holds D^{-1} r.  dot_slot >= 0 also stores
// (r, z) there.  part 0 runs the whole cycle; part 1 everything but the
// level-0 postsmoothing (and the dot); part 2 only those.
template <class T>
void run_vcycle_t(amg_hier* h, const double* r, double* z, hipStream_t s, const T* g0, int dot_slot, int part) {
    const int L = (int)h->lev.size() - 1;
    const T w = T(h->p.omega);
    const Reducer R = h->reducer();
    const Level& L0 = h->lev[0];
    if (L == 0) {  // a single level is solved directly
        if (part == 2) return;
        vc_dense_apply<double, double, double>(h->n_coarse, h->ainv_t, r, z, nullptr, s);
        if (dot_slot >= 0) launch_dot(L0.n, r, z, R, dot_slot, s);
        return;
    }
    auto vec = [](void* p) { return static_cast<T*>(p); };
    if (!g0) {
        if (part != 2) vc_scale_dinv<T>(L0.n, L0.dinv, r, vec(h->g0), s);
        g0 = vec(h->g0);
    }
    auto gk = [&](int k) { return k == 0 ? g0 : vec(h->lev[k].g); };
    auto scatter_to = [&](int k) {  // into level k from level k+1
        return ScatterT<T>{h->lev[k].mem, gk(k), vec(h->lev[k].xp), w};
    };
    if (part == 2) {  // level-0 postsmoothing (+ (r, z)) only
        const VLevel<T> V = vlevel<T>(L0);
        h->rz_np = 0;
        if (streamed(h, L0)) {
            hipEvent_t t0, t1;
            timed_pair(h, 0, t0, t1);
            if (dot_slot >= 0 && h->fuse_dots) {  // (r, z) partials for the direction kernel to add
                const Reducer Rz{R.part + kPartRZ, R.S};
                h->rz_np = vc_stream_post<T, double>(V, vec(L0.xp), g0, w, z, r, &Rz, kPartialsOnly, nullptr, s, t0,
                                                     t1);
            } else {
                vc_stream_post<T, double>(V, vec(L0.xp), g0, w, z, r, dot_slot >= 0 ? &R : nullptr, dot_slot, nullptr,
                                          s, t0, t1);
            }
            timed_end(h, 0, s, true);
        } else {
            timed_begin(h, 0, s);
            vc_prolong_post<T, double>(V, vec(L0.xp), g0, w, z, nullptr, s);
            timed_end(h, 0, s);
            if (dot_slot >= 0) launch_dot(L0.n, r, z, R, dot_slot, s);
        }
        return;
    }
    // down-sweep
    for (int k = 0; k < L; ++k) {
        const Level& Lk = h->lev[k];
        const Level& Lc = h->lev[k + 1];
        const VLevel<T> V = vlevel<T>(Lk);
        T* fc = vec(Lc.f);
        T* gc = vec(Lc.g);
        if (k == 0) timed_begin(h, 1, s);
        if (streamed(h, Lk)) {
            if (k == 0) vc_stream_resid<T, double>(V, r, g0, w, vec(Lk.t), s);
            else vc_stream_resid<T, T>(V, vec(Lk.f), gk(k), w, vec(Lk.t), s);
            if (k == 0) timed_end(h, 1, s);
            vc_restrict<T>(Lc.n, Lk.mem, vec(Lk.t), dinv_of<T>(Lc), fc, gc, s);
        } else {
            if (k == 0) vc_resid_restrict<T, double>(V, Lc.n, r, g0, w, dinv_of<T>(Lc), fc, gc, s);
            else vc_resid_restrict<T, T>(V, Lc.n, vec(Lk.f), gk(k), w, dinv_of<T>(Lc), fc, gc, s);
            if (k == 0) timed_end(h, 1, s);
        }
    }
    // coarsest, then the up-sweep: each level's result is scattered to the
    // finer level's prolongated iterate, which that level's postsmoothing reads
    {
        const ScatterT<T> sc = scatter_to(L - 1);
        vc_dense_apply<T, T, T>(h->n_coarse, h->ainv_t, vec(h->lev[L].f), vec(h->lev[L].x), &sc, s);
    }
    bool dot_done = false;
    for (int k = L - 1; k >= (part == 1 ? 1 : 0); --k) {
        const Level& Lk = h->lev[k];
        const VLevel<T> V = vlevel<T>(Lk);
        if (k > 0) {
            const ScatterT<T> sc = scatter_to(k - 1);
            if (streamed(h, Lk))
                vc_stream_post<T, T>(V, vec(Lk.xp), gk(k), w, vec(Lk.x), nullptr, nullptr, -1, &sc, s);
            else
                vc_prolong_post<T, T>(V, vec(Lk.xp), gk(k), w, vec(Lk.x), &sc, s);
            continue;
        }
        if (streamed(h, Lk)) {
            hipEvent_t t0, t1;
            timed_pair(h, 0, t0, t1);
            vc_stream_post<T, double>(V, vec(Lk.xp), g0, w, z, r, dot_slot >= 0 ? &R : nullptr, dot_slot, nullptr, s,
                                      t0, t1);
            timed_end(h, 0, s, true);
            dot_done = dot_slot >= 0;
        } else {
            timed_begin(h, 0, s);
            vc_prolong_post<T, double>(V, vec(Lk.xp), g0, w, z, nullptr, s);
            timed_end(h, 0, s);
        }
    }
    if (part == 1) return;
    if (dot_slot >= 0 && !dot_done) launch_dot(L0.n, r, z, R, dot_slot, s);
}

// General path (any sweep counts, double only): damped Jacobi sweeps with
// explicit iterates, residual + restriction, prolongation, postsmoothing.
void run_vcycle_general(amg_hier* h, const double* r, double* z, hipStream_t s, int dot_slot) {
    const int L = (int)h->lev.size() - 1;
    const double w = h->p.omega;
    const Reducer R = h->reducer();
    auto dv = [](void* p) { return static_cast<double*>(p); };
    std::vector<const double*> f(L + 1);
    std::vector<double*> x(L + 1);
    f[0] = r;
    x[0] = z;
    for (int k = 1; k <= L; ++k) {
        f[k] = dv(h->lev[k].f);
        x[k] = dv(h->lev[k].x);
    }
    for (int k = 0; k < L; ++k) {
        const Level& Lk = h->lev[k];
        const LevelView V = Lk.view();
        const double* xs = nullptr;
        if (h->p.pre > 0) {
            double* a = x[k];
            double* b = dv(Lk.t);
            launch_jacobi_zero(Lk.n, Lk.dinv, f[k], w, a, s);
            for (int it = 1; it < h->p.pre; ++it) {
                launch_jacobi(V, f[k], a, w, b, s);
                std::swap(a, b);
            }
            if (a != x[k]) HIPCHK(hipMemcpyAsync(x[k], a, sizeof(double) * Lk.n, hipMemcpyDeviceToDevice, s));
            xs = x[k];
        } else {
            launch_scale_zero(Lk.n, x[k], s);
        }
        launch_resid_restrict_x(V, h->lev[k + 1].n, f[k], xs, const_cast<double*>(f[k + 1]), s);
    }
    vc_dense_apply<double, double, double>(h->n_coarse, h->ainv_t, f[L], x[L], nullptr, s);
    for (int k = L - 1; k >= 0; --k) {
        const Level& Lk = h->lev[k];
        const LevelView V = Lk.view();
        launch_prolong_add(Lk.n, Lk.agg, x[k + 1], x[k], s);
        double* a = x[k];
        double* b = dv(Lk.t);
        for (int it = 0; it < h->p.post; ++it) {
            launch_jacobi(V, f[k], a, w, b, s);
            std::swap(a, b);
        }
        if (a != x[k]) HIPCHK(hipMemcpyAsync(x[k], a, sizeof(double) * Lk.n, hipMemcpyDeviceToDevice, s));
    }
    if (dot_slot >= 0) launch_dot(h->lev[0].n, r, z, R, dot_slot, s);
}

// z = V(r) (Algorithm 1).  g0, if given, already holds D^{-1} r in the
// preconditioner's value type.
void run_vcycle(amg_hier* h, const double* r, double* z, hipStream_t s, const void* g0 = nullptr, int dot_slot = -1,
                int part = 0) {
    if (part != 0 && !vcycle_splits(h)) {
        if (part == 2) return;
        part = 0;
    }
    if (!(h->p.pre == 1 && h->p.post == 1)) {
        if (h->lev.size() == 1) {
            vc_dense_apply<double, double, double>(h->n_coarse, h->ainv_t, r, z, nullptr, s);
            if (dot_slot >= 0) launch_dot(h->lev[0].n, r, z, h->reducer(), dot_slot, s);
            return;
        }
        run_vcycle_general(h, r, z, s, dot_slot);
        return;
    }
    if (h->prec32)
        run_vcycle_t<float>(h, r, z, s, static_cast<const float*>(g0), dot_slot, part);
    else
        run_vcycle_t<double>(h, r, z, s, static_cast<const double*>(g0), dot_slot, part);
}

void read_slots(amg_hier* h, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(h->S_host, h->S, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

inline bool usable(double d) { return std::isfinite(d) && d != 0.0; }

void spmv_dot_timed(amg_hier* h, const LevelView& A, const double* p, double* q, const double* d, int slot,
                    hipStream_t s) {
    timed_begin(h, 2, s);
    launch_spmv_dot(A, p, q, d, h->reducer(), slot, s);
    timed_end(h, 2, s);
}

// One PCG iteration of parity pc (ping-pong of the direction vectors and of
// the (r,z) slots): steps [A] q = A p, (p,q); x, r update, (r,r); V-cycle up
// to level 1.  [P] level-0 postsmoothing and (r, z).  [B] next direction and
// the hand-over of the scalar slots (mapped host memory).  The reductions of
// the iteration are added by their consumer kernels from the producers' block
// partials (the update adds (p, q), the direction kernel (r, z) and (r, r)),
// so no separate finish kernel runs.
// [A] is enqueued in two parts: the SpMV (q = A p and the (p, q) partials,
// both scratch that nothing else reads, so it may run ahead of the decision
// whether the iteration is needed), then the update and the V-cycle to level 1.
void pcg_iter_q(amg_hier* h, int pc, hipStream_t s) {
    const Level& A0 = h->lev[0];
    const Reducer R = h->reducer();
    double* p = h->pv[pc];
    if (h->fuse_dots) {
        timed_begin(h, 2, s);
        h->pq_np = launch_spmv_dot_parts(A0.view(), p, h->q, p, R.part + kPartPQ, s);
        timed_end(h, 2, s);
    } else {
        spmv_dot_timed(h, A0.view(), p, h->q, p, S_PQ, s);
        h->pq_np = 0;
    }
}

void pcg_iter_u(amg_hier* h, double* x, int pc, hipStream_t s) {
    const Level& A0 = h->lev[0];
    const Reducer R = h->reducer();
    const int cur = pc ? S_RHO1 : S_RHO0, nxt = pc ? S_RHO0 : S_RHO1;
    double* p = h->pv[pc];
    if (h->fuse_dots) {
        launch_cg_update(A0.n, x, h->r, p, h->q, A0.dinv, h->g0, h->prec32, R, cur, S_PQ, S_RR, s, R.part + kPartPQ,
                         h->pq_np, R.part + kPartRR, &h->rr_np);
    } else {
        launch_cg_update(A0.n, x, h->r, p, h->q, A0.dinv, h->g0, h->prec32, R, cur, S_PQ, S_RR, s);
        h->rr_np = 0;
    }
    run_vcycle(h, h->r, h->z, s, h->g0, nxt, 1);
}

void pcg_iter_a(amg_hier* h, double* x, int pc, hipStream_t s) {
    pcg_iter_q(h, pc, s);
    pcg_iter_u(h, x, pc, s);
}

void pcg_iter_p(amg_hier* h, int pc, hipStream_t s) {
    run_vcycle(h, h->r, h->z, s, h->g0, pc ? S_RHO0 : S_RHO1, 2);
}

// seq != 0: the direction kernel also publishes seq after the slots (eager
// launches only: a captured graph would replay one value).
void pcg_iter_b(amg_hier* h, int pc, hipStream_t s, unsigned long long seq = 0) {
    const int cur = pc ? S_RHO1 : S_RHO0, nxt = pc ? S_RHO0 : S_RHO1;
    double* part = h->part;
    // the direction kernel also writes the slots into the mapped host block
    unsigned long long* hseq = seq ? reinterpret_cast<unsigned long long*>(h->S_dev + kSeqSlot) : nullptr;
    launch_cg_dir(h->lev[0].n, h->z, h->pv[pc], h->pv[1 - pc], h->S, nxt, cur, s, h->S_dev, S_COUNT,
                  h->rz_np ? part + kPartRZ : nullptr, h->rz_np, h->rr_np ? part + kPartRR : nullptr, h->rr_np, S_RR,
                  hseq, seq);
}

// Waits for the eager iteration that publishes sequence number h->seq: the
// host watches that word of the mapped slot block instead of blocking on the
// stream (the next iteration is launched sooner).  After one second it falls
// back to a blocking synchronisation, which also reports a failed kernel.
void wait_slots(amg_hier* h, hipStream_t s) {
    volatile unsigned long long* w = reinterpret_cast<volatile unsigned long long*>(h->S_host + kSeqSlot);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned k = 1; *w != h->seq; ++k) {
        if ((k & 4095) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
            HIPCHK(hipStreamSynchronize(s));
            if (*w != h->seq) raise(AMG_EHIP, "krylov_solve: the iteration's scalars did not arrive");
            break;
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

template <class F>
hipGraphExec_t capture(hipStream_t s, F&& body) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    body();
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        raise(AMG_EHIP, "graph capture failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) raise(AMG_EHIP, "graph instantiation failed: %s", hipGetErrorString(e3));
    return ex;
}

// Enqueue PCG iteration `pc` and its slot read-back on s (graph replay when
// possible); the caller waits for the slots (wait_slots for eager launches,
// a stream synchronisation for graphs) and reads them.  Eager launches:
// q_done says the iteration's SpMV is already enqueued, and ahead (for the
// iteration after this one, parity 1 - pc) enqueues the next SpMV behind it.
void pcg_iteration(amg_hier* h, const double* b, double* x, int pc, bool graphs, hipStream_t s, bool q_done = false,
                   bool ahead = false) {
    const bool timed = h->tim[0].on && vcycle_splits(h);
    if (!graphs) {
        if (!q_done) pcg_iter_q(h, pc, s);
        pcg_iter_u(h, x, pc, s);
        pcg_iter_p(h, pc, s);
        pcg_iter_b(h, pc, s, ++h->seq);
        if (ahead) pcg_iter_q(h, 1 - pc, s);
        HIPCHK(hipGetLastError());
        return;
    }
    if (h->g_key_b != b || h->g_key_x != x) h->drop_graphs();
    h->g_key_b = b;
    h->g_key_x = x;
    if (!timed) {
        if (!h->g_full[pc])
            h->g_full[pc] = capture(s, [&] {
                pcg_iter_a(h, x, pc, s);
                pcg_iter_p(h, pc, s);
                pcg_iter_b(h, pc, s);
            });
        HIPCHK(hipGraphLaunch(h->g_full[pc], s));
        return;
    }
    // timed: the level-0 postsmoothing runs between two graphs, bracketed by
    // events.  The second graph is captured after the postsmoothing has been
    // enqueued once: the direction kernel takes the number of (r, z) partials
    // the postsmoothing leaves (h->rz_np), which that enqueue sets.
    if (!h->g_a[pc]) h->g_a[pc] = capture(s, [&] { pcg_iter_a(h, x, pc, s); });
    HIPCHK(hipGraphLaunch(h->g_a[pc], s));
    pcg_iter_p(h, pc, s);
    if (!h->g_b[pc]) h->g_b[pc] = capture(s, [&] { pcg_iter_b(h, pc, s); });
    HIPCHK(hipGraphLaunch(h->g_b[pc], s));
}

// Algorithm 4 with the readings documented in the header.
amg_status pcg(amg_hier* h, const double* b, double* x, double rtol, int maxit, hipStream_t s, amg_info& info) {
    const Level& A0 = h->lev[0];
    const LevelView A = A0.view();
    const int n = A0.n;
    const Reducer R = h->reducer();
    const int period = h->p.true_res_period;
    const bool graphs = h->use_graphs && !h->tim[1].on && !h->tim[2].on;
    double* S = h->S_host;
    launch_dot(n, b, b, R, S_BB, s);
    launch_residual(A, b, x, h->r, h->g0, h->prec32, R, S_RR, s);
    read_slots(h, s);
    const double nb = std::sqrt(S[S_BB]);
    info.iters = 0;
    if (nb == 0.0) {
        launch_scale_zero(n, x, s);
        HIPCHK(hipStreamSynchronize(s));
        info.rel_res = info.true_rel_res = 0.0;
        return AMG_OK;
    }
    double rel = std::sqrt(S[S_RR]) / nb;
    info.rel_res = info.true_rel_res = rel;
    if (rel <= rtol) return AMG_OK;
    int pc = 0;
    run_vcycle(h, h->r, h->z, s, h->g0, S_RHO0);
    HIPCHK(hipMemcpyAsync(h->pv[0], h->z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    bool q_done = false;  // eager launches: this iteration's SpMV was enqueued ahead
    double rel_prev = 0.0;  // relative residual one iteration earlier (0: none yet)
    for (int it = 1; it <= maxit; ++it) {
        const int cur = pc ? S_RHO1 : S_RHO0, nxt = pc ? S_RHO0 : S_RHO1;
        // the preconditioning, (r, z) and the next direction are speculative:
        // unused when this iteration stops; so is the next iteration's SpMV,
        // enqueued before the host reads this iteration's scalars (it writes
        // only q and its partials).  It is not enqueued when the iteration
        // ends in a residual replacement, or when the last two residuals
        // extrapolate to convergence in this iteration (a wrong guess only
        // delays the next SpMV).
        const bool ahead = !graphs && it < maxit && !(period > 0 && it % period == 0) &&
                           !(rel_prev > 0.0 && rel * (rel / rel_prev) <= rtol);
        pcg_iteration(h, b, x, pc, graphs, s, q_done, ahead);
        q_done = ahead;
        if (graphs) HIPCHK(hipStreamSynchronize(s));
        else wait_slots(h, s);
        if (!usable(S[S_PQ]) || !std::isfinite(S[cur])) return AMG_EBREAKDOWN;
        info.iters = it;
        rel_prev = rel;
        rel = std::sqrt(S[S_RR]) / nb;
        info.rel_res = rel;
        if (!std::isfinite(rel)) return AMG_EBREAKDOWN;
        if (rel <= rtol || (period > 0 && it % period == 0)) {
            launch_residual(A, b, x, h->r, h->g0, h->prec32, R, S_TRR, s);  // residual replacement
            read_slots(h, s);
            const double tr = std::sqrt(S[S_TRR]) / nb;
            info.true_rel_res = tr;
            if (tr <= rtol) return AMG_OK;
            run_vcycle(h, h->r, h->z, s, h->g0, nxt);
            launch_cg_dir(n, h->z, h->pv[pc], h->pv[1 - pc], h->S, nxt, cur, s);
            read_slots(h, s);
            q_done = false;  // the direction changed: the SpMV enqueued ahead is stale
        }
        if (!usable(S[nxt])) return AMG_EBREAKDOWN;
        pc = 1 - pc;
    }
    return AMG_ENOTCONV;
}

// AMG as a stationary solver: Algorithm 1 repeated, x <- x + V(b - A x),
// until the recomputed relative residual reaches rtol.
amg_status stationary(amg_hier* h, const double* b, double* x, double rtol, int maxit, hipStream_t s,
                      amg_info& info) {
    const Level& A0 = h->lev[0];
    const LevelView A = A0.view();
    const int n = A0.n;
    const Reducer R = h->reducer();
    double* S = h->S_host;
    launch_dot(n, b, b, R, S_BB, s);
    launch_residual(A, b, x, h->r, h->g0, h->prec32, R, S_RR, s);
    read_slots(h, s);
    const double nb = std::sqrt(S[S_BB]);
    info.iters = 0;
    if (nb == 0.0) {
        launch_scale_zero(n, x, s);
        HIPCHK(hipStreamSynchronize(s));
        info.rel_res = info.true_rel_res = 0.0;
        return AMG_OK;
    }
    double rel = std::sqrt(S[S_RR]) / nb;
    info.rel_res = info.true_rel_res = rel;
    for (int it = 1; rel > rtol; ++it) {
        if (it > maxit) return AMG_ENOTCONV;
        run_vcycle(h, h->r, h->z, s, h->g0);  // D^{-1} r came with the residual
        launch_add(n, x, h->z, s);
        launch_residual(A, b, x, h->r, h->g0, h->prec32, R, S_RR, s);
        read_slots(h, s);
        info.iters = it;
        rel = std::sqrt(S[S_RR]) / nb;
        info.rel_res = info.true_rel_res = rel;
        if (!std::isfinite(rel)) return AMG_EBREAKDOWN;
    }
    return AMG_OK;
}

// Algorithm 5 (right-preconditioned BiCGStab) with p_0 = r_0 = shadow residual.
amg_status bicgstab(amg_hier* h, const double* b, double* x, double rtol, int maxit, hipStream_t s, amg_info& info) {
    const Level& A0 = h->lev[0];
    const LevelView A = A0.view();
    const int n = A0.n;
    const Reducer R = h->reducer();
    const int period = h->p.true_res_period;
    double* S = h->S_host;
    launch_dot(n, b, b, R, S_BB, s);
    launch_residual(A, b, x, h->r, nullptr, false, R, S_RR, s);
    read_slots(h, s);
    const double nb = std::sqrt(S[S_BB]);
    info.iters = 0;
    if (nb == 0.0) {
        launch_scale_zero(n, x, s);
        HIPCHK(hipStreamSynchronize(s));
        info.rel_res = info.true_rel_res = 0.0;
        return AMG_OK;
    }
    double rel = std::sqrt(S[S_RR]) / nb;
    info.rel_res = info.true_rel_res = rel;
    if (rel <= rtol) return AMG_OK;
    HIPCHK(hipMemcpyAsync(h->rb, h->r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->pv[0], h->r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    int cur = S_RHO0, nxt = S_RHO1, pc = 0;
    launch_dot(n, h->r, h->rb, R, cur, s);
    double* v = h->q;
    unsigned long long* hseq = reinterpret_cast<unsigned long long*>(h->S_dev + kSeqSlot);
    // The direction kernel hands the slots over through the mapped block and
    // the host waits on its sequence word.  Before that wait, the next
    // iteration's first V-cycle (pt = M^{-1} p_next, scratch until the next
    // iteration reads it) is enqueued, so the device works while the host
    // decides; v_done says it was.
    bool v_done = false;
    double rel_prev = 0.0;  // relative residual one iteration earlier (0: none yet)
    for (int it = 1; it <= maxit; ++it) {
        double* p = h->pv[pc];
        double* pn = h->pv[1 - pc];
        if (!v_done) run_vcycle(h, p, h->pt, s);
        spmv_dot_timed(h, A, h->pt, v, h->rb, S_RV, s);
        launch_bicg_s(n, h->r, v, h->sv, h->S, cur, S_RV, s);
        run_vcycle(h, h->sv, h->st, s);
        launch_spmv_dot2(A, h->st, h->t, h->sv, R, S_TT, S_TS, s);
        launch_bicg_update(n, x, h->r, h->pt, h->st, h->sv, h->t, h->rb, R, cur, S_RV, S_TT, S_TS, S_RR, nxt, s);
        launch_bicg_dir(n, h->r, p, v, pn, h->S, cur, S_RV, S_TT, S_TS, nxt, s, h->S_dev, S_COUNT, hseq, ++h->seq);
        // not ahead when this iteration ends in a residual replacement, or is
        // extrapolated to converge (as in PCG)
        v_done = it < maxit && !(period > 0 && it % period == 0) &&
                 !(rel_prev > 0.0 && rel * (rel / rel_prev) <= rtol);
        if (v_done) run_vcycle(h, pn, h->pt, s);
        HIPCHK(hipGetLastError());
        wait_slots(h, s);
        if (!usable(S[S_RV]) || !usable(S[cur])) return AMG_EBREAKDOWN;
        if (!std::isfinite(S[S_TT]) || !std::isfinite(S[S_TS]) || S[S_TT] == 0.0) return AMG_EBREAKDOWN;
        const double omega = S[S_TS] / S[S_TT];
        info.iters = it;
        rel_prev = rel;
        rel = std::sqrt(S[S_RR]) / nb;
        info.rel_res = rel;
        if (!std::isfinite(rel)) return AMG_EBREAKDOWN;
        if (rel <= rtol || (period > 0 && it % period == 0)) {
            launch_residual(A, b, x, h->r, nullptr, false, R, S_TRR, s);
            read_slots(h, s);
            const double tr = std::sqrt(S[S_TRR]) / nb;
            info.true_rel_res = tr;
            if (tr <= rtol) return AMG_OK;
            launch_dot(n, h->r, h->rb, R, nxt, s);
            launch_bicg_dir(n, h->r, p, v, pn, h->S, cur, S_RV, S_TT, S_TS, nxt, s);
            read_slots(h, s);
            v_done = false;  // the direction changed: the V-cycle enqueued ahead is stale
        }
        if (omega == 0.0 || !usable(S[nxt])) return AMG_EBREAKDOWN;
        std::swap(cur, nxt);
        pc = 1 - pc;
    }
    return AMG_ENOTCONV;
}

void setup_impl(const amg_csr* Ain, const amg_params* pin, const amg_allocator* alloc, hipStream_t s,
                amg_hier** out) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!Ain || !out) raise(AMG_EINVAL, "amg_setup: NULL argument");
    *out = nullptr;
    const amg_allocator al = checked_allocator(alloc);
    amg_params p;
    amg_params_default(&p);
    if (pin) p = *pin;
    validate_params(p);
    const amg_csr& A = *Ain;
    if (A.n <= 0) raise(AMG_EINVAL, "n must be positive");
    if (A.nnz < A.n || A.nnz >= (int64_t(1) << 31)) raise(AMG_EINVAL, "nnz must be in [n, 2^31)");
    if (!A.row_ptr || !A.col_idx || !A.val) raise(AMG_EINVAL, "NULL CSR array");

    std::unique_ptr<amg_hier> h(new amg_hier());
    h->p = p;
    h->stream = s;
    h->pool.s = s;
    h->pool.al = al;
    DevPool& P = h->pool;
    P.hint(6 * (size_t)A.nnz + 96 * (size_t)A.n + (size_t(1) << 20));  // most of the hierarchy in one chunk
    h->err = P.get<int>(1);
    HIPCHK(hipMemsetAsync(h->err, 0, sizeof(int), s));

    Level L0;
    L0.n = A.n;
    L0.nnz = A.nnz;
    L0.rp = A.row_ptr;
    L0.ci = A.col_idx;
    L0.v = A.val;
    L0.dinv = P.get<double>(A.n);
    L0.lpr = pick_lanes_per_row((double)A.nnz / A.n);
    launch_validate(A.n, A.nnz, A.row_ptr, A.col_idx, A.val, L0.dinv, h->err, s);
    HIPCHK(hipGetLastError());
    check_err_word(h->err, s, "amg_setup");
    h->lev.push_back(L0);

    DevPool wpool;
    wpool.s = s;
    wpool.al = al;
    wpool.hint((size_t)A.nnz * (p.hem == 1 ? 9 : 1) + 168 * (size_t)A.n + 4096 +
               (p.alternate ? 12 * (size_t)A.nnz + 4 * (size_t)A.n : 0));
    struct WpoolGuard {
        DevPool& t;
        ~WpoolGuard() { t.release(); }
    } wg{wpool};
    SetupWork SW;
    if (A.n > p.max_coarse_rows && p.max_levels > 1)
        SW.init(A.n, A.nnz, wpool, h->err, p.hem == 1, p.alternate == 1);
    // timing events around every matching pass (start/end pairs), read once
    // the setup has synchronised
    std::vector<hipEvent_t> pev;
    struct EvGuard {
        std::vector<hipEvent_t>& v;
        ~EvGuard() {
            for (hipEvent_t e : v) event_put(e, true);
        }
    } evg{pev};
    auto mark_pass = [&](hipStream_t st) {
        pev.push_back(event_get(true));
        HIPCHK(hipEventRecord(pev.back(), st));
    };
    for (int k = 0;; ++k) {
        Level& F = h->lev[k];
        if (F.n <= p.max_coarse_rows) break;
        if (k + 1 >= p.max_levels) {
            if (F.n > p.max_dense_rows)
                raise(AMG_ESTALL, "max_levels reached with %d rows on the coarsest level", F.n);
            break;
        }
        DevPool tmp;
        tmp.s = s;
        tmp.al = al;
        tmp.hint(4 * (size_t)F.n + 12 * (size_t)F.nnz + 4096);  // the intermediate operator of pass 1
        struct TmpGuard {
            DevPool& t;
            ~TmpGuard() { t.release(); }
        } tg{tmp};
        Csr B{F.n, F.nnz, const_cast<int*>(F.rp), const_cast<int*>(F.ci), const_cast<double*>(F.v)};
        // setup-wide pass index: with alternate, odd passes start from the last index
        const int g0 = k * p.passes_per_level;
        mark_pass(s);
        Pass p1 = hem_pass(B, SW, 0, s, h->err, p.alternate && (g0 & 1));
        mark_pass(s);
        h->pass_n.push_back(B.n);
        h->pass_nnz.push_back(B.nnz);
        DevPool& out1 = (p.passes_per_level == 1) ? P : tmp;
        Csr C1 = galerkin(B, p1, SW, out1, s, h->err);
        h->rounds.push_back(p1.rounds);
        Csr Cf = C1;
        int* agg = nullptr;
        int4* mem = nullptr;
        if (p.passes_per_level == 2) {
            mark_pass(s);
            Pass p2 = hem_pass(C1, SW, 1, s, h->err, p.alternate && ((g0 + 1) & 1));
            mark_pass(s);
            h->pass_n.push_back(C1.n);
            h->pass_nnz.push_back(C1.nnz);
            Cf = galerkin(C1, p2, SW, P, s, h->err);
            h->rounds.push_back(p2.rounds);
            agg = P.get<int>(F.n);
            launch_compose(F.n, p1.agg, p2.agg, agg, s);
            mem = P.get<int4>(Cf.n);
            launch_members(Cf.n, p2.lead, p2.mate, p1.lead, p1.mate, mem, s);
        } else {
            agg = P.get<int>(F.n);
            HIPCHK(hipMemcpyAsync(agg, p1.agg, sizeof(int) * F.n, hipMemcpyDeviceToDevice, s));
            mem = P.get<int4>(Cf.n);
            launch_members(Cf.n, nullptr, nullptr, p1.lead, p1.mate, mem, s);
        }
        HIPCHK(hipGetLastError());
        if (Cf.n == F.n) {  // no progress: this level becomes the coarsest
            if (F.n > p.max_dense_rows)
                raise(AMG_ESTALL, "coarsening stalled at %d rows (above max_dense_rows)", F.n);
            HIPCHK(hipStreamSynchronize(s));
            break;
        }
        if ((double)Cf.n >= p.stall_ratio * (double)F.n && F.n <= p.max_dense_rows) {
            HIPCHK(hipStreamSynchronize(s));  // poor progress on a level the dense solve takes
            break;
        }
        F.agg = agg;
        F.mem = mem;
        Level C;
        C.n = Cf.n;
        C.nnz = Cf.nnz;
        C.rp = Cf.rp;
        C.ci = Cf.ci;
        C.v = Cf.v;
        C.dinv = P.get<double>(C.n);
        C.lpr = pick_lanes_per_row((double)C.nnz / C.n);
        launch_dinv(C.n, C.rp, C.ci, C.v, C.dinv, h->err, s);
        HIPCHK(hipGetLastError());  // its error bit is read back with the next level's sizes
        h->lev.push_back(C);
    }
    // coarsest level: dense LU and inverse
    Level& Lc = h->lev.back();
    const int m = Lc.n;
    h->n_coarse = m;
    {
        if (m > kDenseMaxRows) raise(AMG_EHIP, "coarsest level of %d rows exceeds the dense limit (internal error)", m);
        DevPool tmp;
        tmp.s = s;
        tmp.al = al;
        tmp.hint(8 * (size_t)m * m + 8 * (size_t)m + 4096);
        struct TmpGuard {
            DevPool& t;
            ~TmpGuard() { t.release(); }
        } tg{tmp};
        double* a = tmp.get<double>((size_t)m * m);
        int* piv = tmp.get<int>(2 * (size_t)m);  // permutation and pivot rows
        h->ainv_t = P.get<double>((size_t)m * m);
        HIPCHK(hipMemsetAsync(a, 0, sizeof(double) * (size_t)m * m, s));
        launch_dense_assemble(m, Lc.rp, Lc.ci, Lc.v, a, s);
        launch_dense_lu_inverse(m, a, piv, h->ainv_t, h->err, s);
        HIPCHK(hipGetLastError());
        check_err_word(h->err, s, "coarsest level");
    }
    // per-level work vectors, float copies of the values for a float V-cycle
    const bool fused = p.pre == 1 && p.post == 1;
    h->prec32 = p.precond_fp32 != 0;
    const size_t esz = h->prec32 ? sizeof(float) : sizeof(double);
    if (const char* e = getenv("HEMAMG_STREAM_MIN")) h->stream_min = atoi(e);  // tuning sweeps
    if (const char* e = getenv("HEMAMG_RB"))
        for (Level& L : h->lev) L.rb = atoi(e);
    if (const char* e = getenv("HEMAMG_GRAPHS")) h->use_graphs = atoi(e) != 0;
    if (const char* e = getenv("HEMAMG_FUSE_DOTS")) h->fuse_dots = atoi(e) != 0;
    for (size_t k = 0; k < h->lev.size(); ++k) {
        Level& L = h->lev[k];
        if (k > 0) {
            L.f = P.get<char>(esz * L.n);
            L.g = P.get<char>(esz * L.n);
            L.x = P.get<char>(esz * L.n);
        }
        if (fused && k + 1 < h->lev.size()) L.xp = P.get<char>(esz * L.n);
        if (k + 1 < h->lev.size()) L.t = P.get<char>(esz * L.n);  // any level may be tuned to CSR-stream
        if (h->prec32) {
            L.v32 = P.get<float>((size_t)L.nnz);
            L.dinv32 = P.get<float>(L.n);
            launch_cast_f32(L.nnz, L.v, L.v32, s);
            launch_cast_f32(L.n, L.dinv, L.dinv32, s);
        }
    }
    h->g0 = P.get<char>(esz * h->lev[0].n);
    h->S = P.get<double>(S_COUNT);
    h->part = P.get<double>(2 * (size_t)kRedBlocks);
    HIPCHK(hipMemsetAsync(h->S, 0, S_COUNT * sizeof(double), s));
    static_assert((kSeqSlot + 1) * sizeof(double) <= kPinnedBlock, "slots, a read-back word and the sequence word");
    h->S_host = static_cast<double*>(pinned_get());
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->S_dev), h->S_host, 0));
    // the block may come from an earlier handle (whose work has finished):
    // its sequence word restarts with this handle's counter
    *reinterpret_cast<volatile unsigned long long*>(h->S_host + kSeqSlot) = 0;
    h->seq = 0;
    HIPCHK(hipStreamSynchronize(s));
    for (size_t k = 0; k + 1 < pev.size(); k += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pev[k], pev[k + 1]));
        h->match_ms.push_back(ms);
    }
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
}


// ---------------------------------------------------------------------------
// Autotuner: each level's V-cycle schedule is chosen by timing it on this
// hierarchy (both steps of the level, several repetitions after a warm-up):
// CSR-stream kernels with 128, 256 or 512 rows per block, or lane-group
// kernels with 2, 4 or 8 lanes per row.  The schedules differ only in the
// order of a row's additions.
// ---------------------------------------------------------------------------
template <class T>
void tune_level_steps(amg_hier* h, int k, hipStream_t s) {
    const T w = T(h->p.omega);
    auto vec = [](void* p) { return static_cast<T*>(p); };
    Level& Lk = h->lev[k];
    const Level& Lc = h->lev[k + 1];
    const VLevel<T> V = vlevel<T>(Lk);
    const T* g = k == 0 ? vec(h->g0) : vec(Lk.g);
    T* fk = k == 0 ? nullptr : vec(Lk.f);
    if (streamed(h, Lk)) {
        if (k == 0) vc_stream_resid<T, double>(V, h->r, g, w, vec(Lk.t), s);
        else vc_stream_resid<T, T>(V, fk, g, w, vec(Lk.t), s);
        vc_restrict<T>(Lc.n, Lk.mem, vec(Lk.t), dinv_of<T>(Lc), vec(Lc.f), vec(Lc.g), s);
    } else {
        if (k == 0) vc_resid_restrict<T, double>(V, Lc.n, h->r, g, w, dinv_of<T>(Lc), vec(Lc.f), vec(Lc.g), s);
        else vc_resid_restrict<T, T>(V, Lc.n, fk, g, w, dinv_of<T>(Lc), vec(Lc.f), vec(Lc.g), s);
    }
    if (k == 0) {
        if (streamed(h, Lk))
            vc_stream_post<T, double>(V, vec(Lk.xp), g, w, h->z, nullptr, nullptr, -1, nullptr, s);
        else
            vc_prolong_post<T, double>(V, vec(Lk.xp), g, w, h->z, nullptr, s);
        return;
    }
    const Level& Lf = h->lev[k - 1];
    const ScatterT<T> sc{Lf.mem, k - 1 == 0 ? vec(h->g0) : vec(Lf.g), vec(Lf.xp), w};
    if (streamed(h, Lk))
        vc_stream_post<T, T>(V, vec(Lk.xp), g, w, vec(Lk.x), nullptr, nullptr, -1, &sc, s);
    else
        vc_prolong_post<T, T>(V, vec(Lk.xp), g, w, vec(Lk.x), &sc, s);
}

void autotune_impl(amg_hier* h, hipStream_t s, int32_t* out) {
    const int nl = (int)h->lev.size();
    if (out)
        for (int k = 0; k < nl; ++k) out[k] = 0;
    if (nl < 2 || !(h->p.pre == 1 && h->p.post == 1)) return;  // the general path has one schedule
    h->stream = s;
    h->pool.s = s;
    alloc_workspace(h);
    const size_t esz = h->prec32 ? 4 : 8;
    // finite contents for every vector the level steps touch
    HIPCHK(hipMemsetAsync(h->r, 0, sizeof(double) * h->lev[0].n, s));
    HIPCHK(hipMemsetAsync(h->z, 0, sizeof(double) * h->lev[0].n, s));
    HIPCHK(hipMemsetAsync(h->g0, 0, esz * h->lev[0].n, s));
    for (int k = 0; k < nl; ++k) {
        Level& L = h->lev[k];
        for (void* p : {L.f, L.g, L.x, L.xp, L.t})
            if (p) HIPCHK(hipMemsetAsync(p, 0, esz * L.n, s));
    }
    hipEvent_t e0 = event_get(true), e1 = event_get(true);
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            event_put(a, true);
            event_put(b, true);
        }
    } eg{e0, e1};
    struct Cand {
        int sched, rb;
    };
    const Cand cands[] = {{0, 128}, {0, 256}, {0, 512}, {2, 256}, {4, 256}, {8, 256}};
    const int reps = 5;
    for (int k = 0; k + 1 < nl; ++k) {
        Level& Lk = h->lev[k];
        float best = 1e30f;
        Cand pick{-1, 256};
        for (const Cand& c : cands) {
            Lk.sched = c.sched;
            Lk.rb = c.rb;
            auto step = [&] {
                if (h->prec32) tune_level_steps<float>(h, k, s);
                else tune_level_steps<double>(h, k, s);
            };
            step();  // warm-up
            HIPCHK(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) step();
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipGetLastError());
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                pick = c;
            }
        }
        Lk.sched = pick.sched;
        Lk.rb = pick.rb;
        if (out) out[k] = pick.sched == 0 ? pick.rb : -pick.sched;
    }
    h->drop_graphs();
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace

namespace amg {

// Batched setup (see amg_host.hpp).  Level 0 is the inputs concatenated with
// column offsets; a block-diagonal operator couples no two systems, so each
// matching pass and Galerkin product acts on every system exactly as on the
// system alone, and the coarse ids of a system stay contiguous (numbering by
// smallest fine index).  After each level the coarse size of every system is
// read back and the single-system stop rules decide, per system, whether it
// goes on; systems that stop are dropped from the next level's operator.
void batch_coarsen(const amg_csr* A, int count, const amg_params& p, hipStream_t s, DevPool& P,
                   std::vector<SegSrc>& out) {
    validate_params(p);
    if (!A || count < 1) raise(AMG_EINVAL, "amg_batch_setup: no systems");
    out.assign(count, SegSrc{});
    int* err = P.get<int>((size_t)count + 1);  // per-system words, then the shared one
    HIPCHK(hipMemsetAsync(err, 0, sizeof(int) * ((size_t)count + 1), s));
    int* gerr = err + count;
    // level 0: validate each system on its own (a column outside a system must
    // not become a coupling to its neighbour), writing D^{-1} in place
    int64_t N = 0, E = 0;
    std::vector<int> off(count, 0);
    std::vector<int64_t> eoff(count, 0);
    for (int i = 0; i < count; ++i) {
        const amg_csr& a = A[i];
        if (a.n <= 0 || a.nnz < a.n || a.nnz >= (int64_t(1) << 31) || !a.row_ptr || !a.col_idx || !a.val) {
            out[i].status = AMG_EINVAL;
            continue;
        }
        off[i] = (int)N;
        eoff[i] = E;
        N += a.n;
        E += a.nnz;
    }
    if (N >= (int64_t(1) << 31) || E >= (int64_t(1) << 31))
        raise(AMG_EINVAL, "amg_batch_setup: the systems exceed 2^31 rows or entries together");
    if (N == 0) raise(AMG_EINVAL, "amg_batch_setup: no valid system");
    Csr M{(int)N, E, P.get<int>((size_t)N + 1), P.get<int>((size_t)E), P.get<double>((size_t)E)};
    double* dinv = P.get<double>((size_t)N);
    for (int i = 0; i < count; ++i)
        if (out[i].status == AMG_OK)
            launch_validate(A[i].n, A[i].nnz, A[i].row_ptr, A[i].col_idx, A[i].val, dinv + off[i], err + i, s);
    HIPCHK(hipGetLastError());
    {
        std::vector<int> e(count);
        HIPCHK(hipMemcpyAsync(e.data(), err, sizeof(int) * count, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < count; ++i) {
            if (out[i].status != AMG_OK) continue;
            try {
                raise_err_word(e[i], "amg_batch_setup");
            } catch (const Failure& f) {
                out[i].status = f.st;
            }
        }
    }
    // concatenate the valid systems
    std::vector<GatherPiece> pcs;
    int last = -1;
    N = 0;
    E = 0;
    for (int i = 0; i < count; ++i) {
        if (out[i].status != AMG_OK) continue;
        off[i] = (int)N;  // rows of failed systems are left out
        eoff[i] = E;
        N += A[i].n;
        E += A[i].nnz;
        last = i;
    }
    if (last < 0) raise(AMG_EINVAL, "amg_batch_setup: no valid system");
    M.n = (int)N;
    M.nnz = E;
    {
        // D^{-1} of the valid systems moves with them
        double* d2 = P.get<double>((size_t)N);
        int64_t src = 0;
        for (int i = 0; i < count; ++i) {
            const int n = A[i].n > 0 ? A[i].n : 0;
            if (out[i].status == AMG_OK) {
                pcs.push_back(GatherPiece{A[i].row_ptr, M.rp + off[i], n + (i == last ? 1 : 0), (int)eoff[i], 0});
                pcs.push_back(GatherPiece{A[i].col_idx, M.ci + eoff[i], A[i].nnz, off[i], 0});
                pcs.push_back(GatherPiece{A[i].val, M.v + eoff[i], A[i].nnz, 0, 1});
                pcs.push_back(GatherPiece{dinv + src, d2 + off[i], n, 0, 1});
            }
            if (A[i].n > 0 && A[i].nnz >= A[i].n && A[i].nnz < (int64_t(1) << 31) && A[i].row_ptr && A[i].col_idx &&
                A[i].val)
                src += n;  // validated systems were written at their first-pass offsets
        }
        gather_run(pcs, P, s);
        dinv = d2;
    }
    // the systems present in the current level, in order
    struct Live {
        int seg, off, n;
        int64_t eoff, nnz;
    };
    std::vector<Live> live;
    for (int i = 0; i < count; ++i)
        if (out[i].status == AMG_OK) live.push_back(Live{i, off[i], A[i].n, eoff[i], A[i].nnz});
    auto level_src = [&](const Live& L, const Csr& C, const double* dv) {
        SegLevelSrc t;
        t.n = L.n;
        t.nnz = L.nnz;
        t.rp = C.rp + L.off;
        t.rp_add = -(int)L.eoff;
        t.ci = C.ci + L.eoff;
        t.ci_add = -L.off;
        t.v = C.v + L.eoff;
        t.dinv = dv + L.off;
        return t;
    };
    for (const Live& L : live) out[L.seg].lev.push_back(level_src(L, M, dinv));
    // coarsest blocks, factored at the end: (system, level operator, its rows)
    struct Coarsest {
        int seg;
        Csr C;
        Live L;
    };
    std::vector<Coarsest> fin;
    DevPool wpool;
    wpool.s = s;
    wpool.al = P.al;
    wpool.hint((size_t)E * (p.hem == 1 ? 9 : 1) + 168 * (size_t)N + 4096 +
               (p.alternate ? 12 * (size_t)E + 4 * (size_t)N : 0));
    struct WpoolGuard {
        DevPool& t;
        ~WpoolGuard() { t.release(); }
    } wg{wpool};
    SetupWork SW;
    SW.init((int)N, E, wpool, gerr, p.hem == 1, p.alternate == 1);
    int* starts = P.get<int>(2 * (size_t)count);
    int* offs_d = P.get<int>((size_t)count);
    std::vector<int> hs(2 * (size_t)count + 2), ho((size_t)count);
    // node-based passes match each system of at most the LDS limit in a
    // workgroup of its own (its rounds run concurrently with the others')
    const bool seg_ok = p.hem == 0;
    int2* seg_d[2] = {P.get<int2>((size_t)count), P.get<int2>((size_t)count)};
    int* sl0 = seg_ok ? wpool.get<int>((size_t)N) : nullptr;
    int* sl1 = seg_ok ? wpool.get<int>((size_t)N) : nullptr;
    std::vector<int2> hseg((size_t)count);
    for (int k = 0; !live.empty(); ++k) {
        std::vector<char> want(live.size(), 0);
        bool any = false;
        for (size_t j = 0; j < live.size(); ++j) {
            const Live& L = live[j];
            if (L.n <= p.max_coarse_rows) continue;
            if (k + 1 >= p.max_levels) {
                if (L.n > p.max_dense_rows) out[L.seg].status = AMG_ESTALL;
                continue;
            }
            want[j] = 1;
            any = true;
        }
        if (!any) {
            for (const Live& L : live)
                if (out[L.seg].status == AMG_OK) fin.push_back(Coarsest{L.seg, M, L});
            break;
        }
        const int g0 = k * p.passes_per_level;
        const int m = (int)live.size();
        for (int j = 0; j < m; ++j) ho[j] = live[j].off;
        HIPCHK(hipMemcpyAsync(offs_d, ho.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
        const bool fl1 = p.alternate && (g0 & 1), fl2 = p.alternate && ((g0 + 1) & 1);
        SegPass sp1, sp2;
        if (seg_ok) {
            int big = 0;
            for (int j = 0; j < m; ++j) {
                const Live& L = live[j];
                hseg[j] = fl1 ? make_int2(M.n - L.off - L.n, L.n) : make_int2(L.off, L.n);
                big = std::max(big, L.n);
            }
            HIPCHK(hipMemcpyAsync(seg_d[0], hseg.data(), sizeof(int2) * m, hipMemcpyHostToDevice, s));
            sp1.seg = seg_d[0];
            sp1.nseg = m;
            sp1.all_small = big <= SW.hw.lds_rows;  // a system's later passes are smaller
            sp1.sl[0] = sl0;
            sp1.sl[1] = sl1;
            sp2 = sp1;
            sp2.seg = seg_d[1];
        }
        Pass p1 = hem_pass(M, SW, 0, s, gerr, fl1, seg_ok ? &sp1 : nullptr);
        Csr C1 = galerkin(M, p1, SW, P, s, gerr);
        Csr Cf = C1;
        int* agg = P.get<int>((size_t)M.n);
        int4* mem = nullptr;
        if (p.passes_per_level == 2) {
            if (seg_ok) launch_seg_table(m, offs_d, p1.agg, C1.n, fl2, seg_d[1], s);
            Pass p2 = hem_pass(C1, SW, 1, s, gerr, fl2, seg_ok ? &sp2 : nullptr);
            Cf = galerkin(C1, p2, SW, P, s, gerr);
            launch_compose(M.n, p1.agg, p2.agg, agg, s);
            mem = P.get<int4>((size_t)Cf.n);
            launch_members(Cf.n, p2.lead, p2.mate, p1.lead, p1.mate, mem, s);
        } else {
            HIPCHK(hipMemcpyAsync(agg, p1.agg, sizeof(int) * M.n, hipMemcpyDeviceToDevice, s));
            mem = P.get<int4>((size_t)Cf.n);
            launch_members(Cf.n, nullptr, nullptr, p1.lead, p1.mate, mem, s);
        }
        // where each system starts in the coarse level
        launch_seg_starts(m, offs_d, agg, Cf.rp, starts, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hs.data(), starts, sizeof(int) * 2 * m, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<Live> next;
        for (int j = 0; j < m; ++j) {
            const Live& L = live[j];
            const int c0 = hs[2 * j], c1 = j + 1 < m ? hs[2 * (j + 1)] : Cf.n;
            const int64_t q0 = hs[2 * j + 1], q1 = j + 1 < m ? hs[2 * (j + 1) + 1] : Cf.nnz;
            const int nc = c1 - c0;
            bool stop = !want[j];
            if (!stop && nc == L.n) {  // no progress
                if (L.n > p.max_dense_rows) out[L.seg].status = AMG_ESTALL;
                stop = true;
            }
            if (!stop && (double)nc >= p.stall_ratio * (double)L.n && L.n <= p.max_dense_rows) stop = true;
            if (stop) {
                if (out[L.seg].status == AMG_OK) fin.push_back(Coarsest{L.seg, M, L});
                continue;
            }
            SegLevelSrc& cur = out[L.seg].lev.back();
            cur.mem = mem + c0;
            cur.mem_add = -L.off;
            next.push_back(Live{L.seg, c0, nc, q0, q1 - q0});
        }
        if (next.empty()) break;
        // the next level: the coarse operator, without the systems that stopped
        Csr Mn = Cf;
        bool compact = next.size() != live.size();
        if (compact) {
            int64_t n2 = 0, e2 = 0;
            for (const Live& L : next) {
                n2 += L.n;
                e2 += L.nnz;
            }
            Mn = Csr{(int)n2, e2, P.get<int>((size_t)n2 + 1), P.get<int>((size_t)e2), P.get<double>((size_t)e2)};
            std::vector<GatherPiece> cp;
            int r = 0;
            int64_t e = 0;
            for (size_t j = 0; j < next.size(); ++j) {
                Live& L = next[j];
                const bool lastp = j + 1 == next.size();
                cp.push_back(GatherPiece{Cf.rp + L.off, Mn.rp + r, L.n + (lastp ? 1 : 0), (int)(e - L.eoff), 0});
                cp.push_back(GatherPiece{Cf.ci + L.eoff, Mn.ci + e, L.nnz, r - L.off, 0});
                cp.push_back(GatherPiece{Cf.v + L.eoff, Mn.v + e, L.nnz, 0, 1});
                L.off = r;
                L.eoff = e;
                r += L.n;
                e += L.nnz;
            }
            gather_run(cp, P, s);
        }
        double* dn = P.get<double>((size_t)Mn.n);
        launch_dinv(Mn.n, Mn.rp, Mn.ci, Mn.v, dn, gerr, s);
        HIPCHK(hipGetLastError());
        for (const Live& L : next) out[L.seg].lev.push_back(level_src(L, Mn, dn));
        M = Mn;
        dinv = dn;
        live.swap(next);
    }
    check_err_word(gerr, s, "amg_batch_setup");
    // coarsest blocks: dense LU and inverse per system
    for (const Coarsest& c : fin) {
        SegSrc& S = out[c.seg];
        const int m = c.L.n;
        if (S.lev.size() < 2) {  // a single level is not batched
            S.status = AMG_EINVAL;
            continue;
        }
        if (m > kDenseMaxRows) raise(AMG_EHIP, "coarsest level of %d rows exceeds the dense limit (internal error)", m);
        double* a = P.get<double>((size_t)m * m);
        int* piv = P.get<int>(2 * (size_t)m);
        double* ainv = P.get<double>((size_t)m * m);
        HIPCHK(hipMemsetAsync(a, 0, sizeof(double) * (size_t)m * m, s));
        launch_dense_assemble(m, c.C.rp + c.L.off, c.C.ci, c.C.v, a, s, -c.L.off);
        launch_dense_lu_inverse(m, a, piv, ainv, err + c.seg, s);
        S.ainv_t = ainv;
        S.lev.back().mem = nullptr;
    }
    HIPCHK(hipGetLastError());
    std::vector<int> e(count);
    HIPCHK(hipMemcpyAsync(e.data(), err, sizeof(int) * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (const Coarsest& c : fin)
        if (out[c.seg].status == AMG_OK && (e[c.seg] & ERR_SINGULAR)) out[c.seg].status = AMG_ESINGULAR;
    for (SegSrc& S : out)
        if (S.status != AMG_OK) S.lev.clear();
}

// The Krylov solve behind krylov_solve.  ext (non-null): kKrylovVecs work
// vectors of at least n doubles each that the caller provides; the solve
// then draws nothing: no workspace from the handle's allocator, no stream of
// its own, no graph capture, read-backs through the handle's pinned slots.
amg_status krylov_run(amg_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                      void* stream, amg_info* info, double* const* ext) {
    amg_info local{};
    amg_info& I = info ? *info : local;
    I = amg_info{};
    const auto t0 = std::chrono::steady_clock::now();
    amg_status st = AMG_OK;
    amg_status g = guarded([&] {
        if (!h || !b || !x) raise(AMG_EINVAL, "krylov_solve: NULL argument");
        if (method < 0 || method > 2)
            raise(AMG_EINVAL, "krylov_solve: method must be 0 (PCG), 1 (BiCGStab) or 2 (stationary)");
        if (!(rtol >= 0.0) || maxit < 0) raise(AMG_EINVAL, "krylov_solve: rtol must be >= 0 and maxit >= 0");
        hipStream_t s = as_stream(stream);
        h->stream = s;
        h->pool.s = s;
        // the caller's vectors stand in for the handle's workspace for this
        // call only (graphs captured on the handle's own vectors stay valid)
        double* saved[kKrylovVecs];
        double** slot[kKrylovVecs] = {&h->r, &h->z, &h->pv[0], &h->pv[1], &h->q,
                                      &h->rb, &h->pt, &h->sv, &h->st, &h->t};
        const bool graphs_were = h->use_graphs;
        struct Restore {
            amg_hier* h;
            double** const* slot;
            double* const* saved;
            bool on, graphs;
            ~Restore() {
                if (!on) return;
                for (int k = 0; k < kKrylovVecs; ++k) *slot[k] = saved[k];
                h->use_graphs = graphs;
            }
        } restore{h, slot, saved, ext != nullptr, graphs_were};
        if (ext) {
            for (int k = 0; k < kKrylovVecs; ++k) {
                saved[k] = *slot[k];
                *slot[k] = ext[k];
            }
            h->use_graphs = false;
        } else {
            alloc_workspace(h);
        }
        // the solve runs on the caller's stream, or on the handle's own stream
        // (ordered after the caller's prior work) when that is the null
        // stream or graphs are replayed (they cannot be captured on it)
        const bool own = !ext && (s == nullptr || h->use_graphs);
        if (own && !h->gstream) {
            h->gstream = stream_get();
            h->gev[0] = event_get(false);
            h->gev[1] = event_get(false);
        }
        if (own) {
            HIPCHK(hipEventRecord(h->gev[0], s));
            HIPCHK(hipStreamWaitEvent(h->gstream, h->gev[0], 0));
        }
        hipStream_t ws = own ? h->gstream : s;
        h->pool.s = ws;
        HIPCHK(hipMemsetAsync(h->err, 0, sizeof(int), ws));
        launch_check_finite(h->lev[0].n, b, x, h->err, ws);
        HIPCHK(hipGetLastError());
        int e = 0;
        if (ext) {  // the handle's pinned block, past the scalar slots
            int* hw = reinterpret_cast<int*>(h->S_host + S_COUNT);
            HIPCHK(hipMemcpyAsync(hw, h->err, sizeof(int), hipMemcpyDeviceToHost, ws));
            HIPCHK(hipStreamSynchronize(ws));
            e = *hw;
        } else {
            e = read_int(h->err, ws);
        }
        if (e & ERR_NONFINITE) raise(AMG_ENOTFINITE, "krylov_solve: b or x0 has NaN or Inf");
        st = method == 0   ? pcg(h, b, x, rtol, maxit, ws, I)
             : method == 1 ? bicgstab(h, b, x, rtol, maxit, ws, I)
                           : stationary(h, b, x, rtol, maxit, ws, I);
        HIPCHK(hipStreamSynchronize(ws));
        if (own) {
            HIPCHK(hipEventRecord(h->gev[1], ws));
            HIPCHK(hipStreamWaitEvent(s, h->gev[1], 0));
        }
        h->pool.s = s;
        if (st == AMG_ENOTCONV) g_err = "krylov_solve: iteration limit reached";
        if (st == AMG_EBREAKDOWN) g_err = "krylov_solve: breakdown (zero or non-finite denominator)";
    });
    if (g != AMG_OK) st = g;
    I.status = st;
    I.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (h) {
        I.setup_ms = h->setup_ms;
        I.levels = (int32_t)h->lev.size();
    }
    return st;
}

}  // namespace amg

extern "C" {

amg_status amg_params_default(amg_params* p) {
    if (!p) {
        g_err = "amg_params_default: NULL argument";
        return AMG_EINVAL;
    }
    p->passes_per_level = 2;
    p->max_coarse_rows = 64;
    p->max_levels = 32;
    p->max_dense_rows = kDenseMaxRows;
    p->omega = 2.0 / 3.0;
    p->pre = 1;
    p->post = 1;
    p->true_res_period = 50;
    p->precond_fp32 = 0;
    p->stall_ratio = 0.9;
    p->hem = 0;
    p->alternate = 0;
    return AMG_OK;
}

amg_status amg_setup(const amg_csr* A, const amg_params* params, const amg_allocator* alloc, void* stream,
                     amg_hier** out) {
    if (out) *out = nullptr;
    return guarded([&] { setup_impl(A, params, alloc, as_stream(stream), out); });
}

amg_status amg_destroy(amg_hier* h) {
    return guarded([&] { delete h; });
}

amg_status amg_vcycle(amg_hier* h, const double* r, double* z, void* stream) {
    return guarded([&] {
        if (!h || !r || !z) raise(AMG_EINVAL, "amg_vcycle: NULL argument");
        hipStream_t s = as_stream(stream);
        h->stream = s;
        h->pool.s = s;
        run_vcycle(h, r, z, s);
        HIPCHK(hipGetLastError());
    });
}

amg_status krylov_solve(amg_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                        void* stream, amg_info* info) {
    return amg::krylov_run(h, method, b, x, rtol, maxit, stream, info, nullptr);
}

}  // extern "C"

// Work vectors of krylov_solve_noalloc: kKrylovVecs vectors of up to
// kNoAllocRows doubles each (80 MiB), one copy on every device the library
// runs on, held until the process ends.  Host code never uses the array's
// name as an address: each device's copy is reached through the pointer that
// hipGetSymbolAddress returns for it.
namespace {
constexpr int kNoAllocRows = 1 << 20;
static __device__ __align__(256) double scratch[(size_t)amg::kKrylovVecs * kNoAllocRows];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];  // device address of scratch, per device (nullptr: not resolved yet)

// The current device's copy of scratch, resolved once per device.
double* scratch_of_current_device() {
    const int d = amg::current_device();
    if (d < 0 || d >= kMaxDevices) raise(AMG_EHIP, "krylov_solve_noalloc: device %d out of range", d);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[d]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            raise(AMG_EHIP, "krylov_solve_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[d] = static_cast<double*>(p);
    }
    return g_scratch_dev[d];
}
}  // namespace

extern "C" {

amg_status krylov_solve_noalloc(amg_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                                void* stream, amg_info* info) {
    double* ext[amg::kKrylovVecs];
    const amg_status st = guarded([&] {
        if (!h) raise(AMG_EINVAL, "krylov_solve_noalloc: NULL argument");
        const int n = h->lev[0].n;
        if (n > kNoAllocRows)
            raise(AMG_EINVAL, "krylov_solve_noalloc: %d rows exceed the scratch limit of %d rows", n, kNoAllocRows);
        double* base = scratch_of_current_device();
        const size_t stride = ((size_t)n + 31) / 32 * 32;  // 256-byte aligned vectors
        for (int k = 0; k < amg::kKrylovVecs; ++k) ext[k] = base + (size_t)k * stride;
    });
    if (st != AMG_OK) {
        if (info) {
            *info = amg_info{};
            info->status = st;
        }
        return st;
    }
    return amg::krylov_run(h, method, b, x, rtol, maxit, stream, info, ext);
}

amg_status amg_num_levels(const amg_hier* h, int32_t* levels) {
    return guarded([&] {
        if (!h || !levels) raise(AMG_EINVAL, "amg_num_levels: NULL argument");
        *levels = (int32_t)h->lev.size();
    });
}

amg_status amg_level_size(const amg_hier* h, int32_t k, int32_t* n, int64_t* nnz) {
    return guarded([&] {
        if (!h || !n || !nnz) raise(AMG_EINVAL, "amg_level_size: NULL argument");
        if (k < 0 || k >= (int32_t)h->lev.size()) raise(AMG_EINVAL, "amg_level_size: level out of range");
        *n = h->lev[k].n;
        *nnz = h->lev[k].nnz;
    });
}

amg_status amg_export_level(const amg_hier* h, int32_t k, int32_t* row_ptr, int32_t* col_idx, double* val,
                            int32_t* agg, void* stream) {
    return guarded([&] {
        if (!h) raise(AMG_EINVAL, "amg_export_level: NULL handle");
        if (k < 0 || k >= (int32_t)h->lev.size()) raise(AMG_EINVAL, "amg_export_level: level out of range");
        const Level& L = h->lev[k];
        hipStream_t s = as_stream(stream);
        if (row_ptr)
            HIPCHK(hipMemcpyAsync(row_ptr, L.rp, sizeof(int) * ((size_t)L.n + 1), hipMemcpyDeviceToHost, s));
        if (col_idx) HIPCHK(hipMemcpyAsync(col_idx, L.ci, sizeof(int) * L.nnz, hipMemcpyDeviceToHost, s));
        if (val) HIPCHK(hipMemcpyAsync(val, L.v, sizeof(double) * L.nnz, hipMemcpyDeviceToHost, s));
        if (agg && L.agg) HIPCHK(hipMemcpyAsync(agg, L.agg, sizeof(int) * L.n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    });
}

amg_status amg_setup_stats(const amg_hier* h, int32_t cap, int32_t* rounds, double* match_ms, int32_t* pass_n,
                           int64_t* pass_nnz, int32_t* npasses, size_t* owned_bytes) {
    return guarded([&] {
        if (!h) raise(AMG_EINVAL, "amg_setup_stats: NULL handle");
        const int32_t np = (int32_t)h->rounds.size();
        if (npasses) *npasses = np;
        for (int32_t i = 0; i < cap && i < np; ++i) {
            if (rounds) rounds[i] = h->rounds[i];
            if (match_ms) match_ms[i] = i < (int32_t)h->match_ms.size() ? h->match_ms[i] : 0.0;
            if (pass_n) pass_n[i] = i < (int32_t)h->pass_n.size() ? h->pass_n[i] : 0;
            if (pass_nnz) pass_nnz[i] = i < (int32_t)h->pass_nnz.size() ? h->pass_nnz[i] : 0;
        }
        if (owned_bytes) *owned_bytes = h->pool.bytes;
    });
}

amg_status amg_timing_enable(amg_hier* h, int32_t kernel, int32_t on) {
    return guarded([&] {
        if (!h || kernel < 0 || kernel > 2) raise(AMG_EINVAL, "amg_timing_enable: bad argument");
        h->tim[kernel].on = on != 0;
    });
}

amg_status amg_autotune(amg_hier* h, void* stream, int32_t* schedule) {
    return guarded([&] {
        if (!h) raise(AMG_EINVAL, "amg_autotune: NULL handle");
        autotune_impl(h, as_stream(stream), schedule);
    });
}

amg_status amg_timing_read(amg_hier* h, int32_t kernel, int64_t* launches, double* total_ms) {
    return guarded([&] {
        if (!h || kernel < 0 || kernel > 2) raise(AMG_EINVAL, "amg_timing_read: bad argument");
        Timer& T = h->tim[kernel];
        if (T.used > 0) {
            HIPCHK(hipEventSynchronize(T.ev[T.used - 1]));
            for (size_t k = 0; k < T.used; k += 2) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, T.ev[k], T.ev[k + 1]));
                T.total_ms += ms;
                T.launches += 1;
            }
            T.used = 0;
        }
        if (launches) *launches = T.launches;
        if (total_ms) *total_ms = T.total_ms;
        T.launches = 0;
        T.total_ms = 0.0;
    });
}

const char* amg_last_error(void) { return g_err.c_str(); }

amg_status amg_cached_bytes(uint64_t* bytes) {
    return guarded([&] {
        if (!bytes) raise(AMG_EINVAL, "amg_cached_bytes: NULL argument");
        *bytes = (uint64_t)chunk_kept_bytes();
    });
}

amg_status amg_release_cached(void) {
    return guarded([&] {
        chunk_flush();  // waits for each chunk's last use, frees it and waits for the frees
        HIPCHK(hipMemPoolTrimTo(lib_pool(), 0));
    });
}

}  // extern "C"
