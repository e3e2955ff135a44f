// Host-side infrastructure shared by the library's host sources: error
// reporting, device memory arenas, pooled streams, events and pinned memory,
// and the hierarchy handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "amg_internal.hpp"
#include "hemamg.h"

namespace amg {
inline thread_local std::string g_err = "no error";

struct Failure {
    amg_status st;
    std::string msg;
};

[[noreturn]] inline void raise(amg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw Failure{st, buf};
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            if (e_ == hipErrorOutOfMemory) raise(AMG_ENOMEM, "%s: out of GPU memory", #call); \
            raise(AMG_EHIP, "%s: %s", #call, hipGetErrorString(e_));                          \
        }                                                                                     \
    } while (0)

// Streams and events are kept in process-wide free lists per device:
// creating and destroying them costs milliseconds per handle.  Streams are
// non-blocking at the default priority; timing events record times, the
// others do not.
int current_device();
hipStream_t stream_get();
void stream_put(hipStream_t s);
hipEvent_t event_get(bool timing);
void event_put(hipEvent_t e, bool timing);
// Pinned host blocks of kPinnedBlock bytes (scalar slots of a handle or a
// batch), mapped into the device and coherent, kept for reuse.
constexpr size_t kPinnedBlock = 4096;
void* pinned_get();
void pinned_put(void* p);
// Pinned host words for small read-backs (per thread, kept for the process).
// (mapped into the device and coherent: a kernel may write them, through the
// device address *dev, for the host to read once the stream has finished)
int* pinned_words(int** dev = nullptr);
int read_int(const int* d, hipStream_t s);
void raise_err_word(int e, const char* where);
void check_err_word(const int* err, hipStream_t s, const char* where);

// Device memory comes from a stream-ordered pool owned by the library (one
// per device) that keeps freed blocks for reuse instead of returning them to
// the driver, so building a hierarchy does not remap memory level by level.
inline hipMemPool_t lib_pool() {
    static std::mutex mu;
    static std::map<int, hipMemPool_t> pools;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto it = pools.find(dev);
    if (it != pools.end()) return it->second;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    HIPCHK(hipMemPoolCreate(&pool, &props));
    uint64_t keep = UINT64_MAX;
    HIPCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    pools[dev] = pool;
    return pool;
}

// The caller's allocator (amg_allocator), checked and copied: both
// functions set, or neither (then the library pool serves).
inline amg_allocator checked_allocator(const amg_allocator* a) {
    amg_allocator r{};
    if (!a || (!a->alloc && !a->free)) return r;
    if (!a->alloc || !a->free) raise(AMG_EINVAL, "amg_allocator: alloc and free must both be set");
    return *a;
}

// Library-pool chunks that an arena releases are kept per device instead of
// being handed back to the stream-ordered pool.  Returning a block costs about
// 0.3 ms of host time on MI355X, and once blocks have gone back, a later
// allocation that reuses them has been measured to block the host for 0.3 to
// 1.8 s while the device sits idle (concurrent setups of a served stream).
// Chunk sizes are rounded up to classes (below) so that released chunks fit
// later requests.  chunk_keep stores a chunk with an event recorded on the
// stream that last used it (false: larger than the cache, the caller frees
// it); the oldest kept chunks go back to the pool once the device's cache
// holds more than chunk_cache_cap().  chunk_take hands out a kept chunk of
// exactly `bytes` on the current device after `s` waits for that event
// (nullptr: none); chunk_flush frees every kept chunk of the current device
// (an allocation that finds the device out of memory calls it).
bool chunk_keep(void* p, size_t bytes, hipStream_t s);
void* chunk_take(size_t bytes, hipStream_t s);
void chunk_flush();
size_t chunk_kept_bytes();  // kept on the current device
// Kept bytes per device at most: a quarter of the device's memory, and no
// more than 64 GiB.
size_t chunk_cache_cap();

// Size class of a library-pool chunk of at least c bytes: c rounded up to a
// multiple of a quarter of the largest power of two not above it (classes
// 4, 5, 6, 7 and 8 times 2^(k-2) between 2^k and 2^(k+1): at most 25% over),
// and at least 1 MiB.
inline size_t chunk_class(size_t c) {
    if (c <= (size_t(1) << 20)) return size_t(1) << 20;
    const int k = 63 - __builtin_clzll((unsigned long long)c);
    const size_t q = size_t(1) << (k - 2);
    return (c + q - 1) / q * q;
}

// An arena over the pool (or the caller's allocator): pieces (256-byte
// aligned) are carved from a few chunks (sized from a hint, or by a larger
// request), so a handle makes a handful of allocation calls instead of one
// per array.  Chunks are released stream-ordered on the stream they were
// drawn on (library chunks into the chunk cache above).
struct DevPool {
    struct Chunk {
        void* p;
        hipStream_t s;
        size_t bytes;
    };
    hipStream_t s = nullptr;
    hipMemPool_t mp = nullptr;
    amg_allocator al{};                // al.alloc set: chunks come from the caller
    std::vector<Chunk> chunks;
    char* cur = nullptr;
    size_t left = 0;
    size_t bytes = 0;                 // device memory held (sum of chunks)
    size_t next_chunk = size_t(1) << 20;

    void hint(size_t b) {
        if (b > next_chunk) next_chunk = b;
    }

    template <class T>
    T* get(size_t count) {
        const size_t b = (((count > 0 ? count : 1) * sizeof(T)) + 255) & ~size_t(255);
        if (b > left) {
            size_t c = b > next_chunk ? b : next_chunk;
            void* p = nullptr;
            if (!al.alloc) c = chunk_class(c);
            if (al.alloc) {
                p = al.alloc(c, al.ctx, s);
                if (!p) raise(AMG_ENOMEM, "the caller's allocator returned NULL for %zu bytes", c);
            } else if (!(p = chunk_take(c, s))) {
                if (!mp) mp = lib_pool();
                hipError_t e = hipMallocFromPoolAsync(&p, c, mp, s);
                if (e == hipErrorOutOfMemory) {  // give the kept chunks back and try once more
                    (void)hipGetLastError();
                    chunk_flush();
                    e = hipMallocFromPoolAsync(&p, c, mp, s);
                }
                if (e == hipErrorOutOfMemory) raise(AMG_ENOMEM, "hipMallocFromPoolAsync: out of GPU memory");
                if (e != hipSuccess) raise(AMG_EHIP, "hipMallocFromPoolAsync: %s", hipGetErrorString(e));
            }
            chunks.push_back(Chunk{p, s, c});
            cur = static_cast<char*>(p);
            left = c;
            bytes += c;
            next_chunk = c;
        }
        T* r = reinterpret_cast<T*>(cur);
        cur += b;
        left -= b;
        return r;
    }
    void release() {
        for (auto& c : chunks) {
            if (al.alloc) al.free(c.p, al.ctx, c.s);
            else if (!chunk_keep(c.p, c.bytes, c.s)) (void)hipFreeAsync(c.p, c.s);
        }
        chunks.clear();
        cur = nullptr;
        left = 0;
        bytes = 0;
        next_chunk = size_t(1) << 20;
    }
};

struct Level {
    int n = 0;
    int64_t nnz = 0;
    const int* rp = nullptr;
    const int* ci = nullptr;
    const double* v = nullptr;
    double* dinv = nullptr;
    int* agg = nullptr;    // to level k+1
    int4* mem = nullptr;   // members of level k+1 rows
    float* v32 = nullptr;     // float copy of the values (single-precision preconditioner)
    float* dinv32 = nullptr;
    // V-cycle vectors, of the preconditioner's value type (double or float)
    void* f = nullptr;    // restricted right-hand side (k >= 1)
    void* g = nullptr;    // D^{-1} f (k >= 1)
    void* x = nullptr;    // correction (k >= 1)
    void* xp = nullptr;   // prolongated iterate w D^{-1} f + P e (k < coarsest)
    void* t = nullptr;    // residual scratch (CSR-stream levels) / general smoothing path
    int lpr = 4;
    // V-cycle schedule of this level: sched < 0 follows the size rule
    // (CSR-stream kernels from amg_hier::stream_min rows up), 0 forces the
    // CSR-stream kernels, > 0 the lane-group kernels with that many lanes per
    // row; rb = rows per block of the CSR-stream kernels.
    int sched = -1;
    int rb = 256;

    LevelView view() const {
        LevelView w;
        w.n = n;
        w.nnz = (int)nnz;
        w.rp = rp;
        w.ci = ci;
        w.v = v;
        w.dinv = dinv;
        w.agg = agg;
        w.mem = mem;
        w.lpr = lpr;
        return w;
    }
};

// Scalar slots of the Krylov recurrences.
enum Slot { S_BB = 0, S_RR, S_TRR, S_PQ, S_RHO0, S_RHO1, S_RV, S_TT, S_TS, S_COUNT = 16 };
// In a handle's mapped slot block: S_COUNT slots, an int read-back word at
// S_COUNT, and at kSeqSlot the sequence number of the last eager PCG
// iteration whose slots have arrived.
constexpr int kSeqSlot = S_COUNT + 1;

struct Timer {
    bool on = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t used = 0;
    int64_t launches = 0;
    double total_ms = 0.0;
};

template <class F>
amg_status guarded(F&& f) {
    try {
        f();
        return AMG_OK;
    } catch (const Failure& e) {
        g_err = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return AMG_ENOMEM;
    } catch (...) {
        g_err = "unexpected internal error";
        return AMG_EHIP;
    }
}

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// ---- batches ----------------------------------------------------------------
// One system's level k inside source arrays (a hierarchy, or the concatenated
// operators of a batched setup).  Adding rp_add to the row pointers, ci_add to
// the columns and mem_add to the members gives the system's own numbering.
struct SegLevelSrc {
    int n = 0;
    int64_t nnz = 0;
    const int* rp = nullptr;  // [n + 1]
    int rp_add = 0;
    const int* ci = nullptr;  // [nnz]
    int ci_add = 0;
    const double* v = nullptr;
    const float* v32 = nullptr;     // null: rounded from v
    const double* dinv = nullptr;   // [n]
    const float* dinv32 = nullptr;  // null: rounded from dinv
    const int4* mem = nullptr;      // [rows of level k+1]; null on the coarsest level
    int mem_add = 0;
};
struct SegSrc {
    amg_status status = AMG_OK;      // a failed system takes no rows in a batch
    std::vector<SegLevelSrc> lev;    // levels 0 .. coarsest
    const double* ainv_t = nullptr;  // coarsest inverse, column-major
};

void validate_params(const amg_params& p);
// Copies every piece with one launch (blocks the host until done).
void gather_run(const std::vector<GatherPiece>& pcs, DevPool& P, hipStream_t s);
// Work vectors of a Krylov solve (PCG, BiCGStab, stationary), n doubles each.
constexpr int kKrylovVecs = 10;
amg_status krylov_run(amg_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                      void* stream, amg_info* info, double* const* ext);
// Batched PCG advanced one iteration at a time (the solve of amg_batch_solve
// with method 0, step by step): start runs the prologue on the batch's stream
// from the right-hand sides and initial guesses already in the batch
// (batch_load), enqueue queues one iteration, collect waits for it and
// applies the per-system rules.  `done` receives the systems that left the
// iteration (their iterate is final from then on).  Blocks the host in start
// and collect only.
struct PcgRun;
PcgRun* pcg_run_start(amg_batch* B, double rtol, int maxit, std::vector<int>& done);
void pcg_run_enqueue(PcgRun* R);
void pcg_run_collect(PcgRun* R, std::vector<int>& done);
int pcg_run_live(const PcgRun* R);
const amg_info& pcg_run_info(const PcgRun* R, int i);
void pcg_run_end(PcgRun* R);
// System i's right-hand side and initial guess into the batch (device to
// device, on the batch's stream, ordered after `after` when given).
void batch_load(amg_batch* B, int i, const double* b, const double* x0, hipStream_t after);
// Device address and rows of system i's iterate inside the batch, and the
// batch's stream.
const double* batch_x(const amg_batch* B, int i, int* n);
// Device memory the batch holds (levels, coarsest blocks, Krylov vectors).
size_t batch_bytes(const amg_batch* B);
hipStream_t batch_stream(const amg_batch* B);
// setup_ms and levels of system i (what amg_batch_solve reports).
void batch_fill_info(const amg_batch* B, int i, amg_info& I);
// Batched setup: the systems' levels are built together on concatenated
// operators (one matching round and one Galerkin launch per step for all of
// them) with each system's stop rule applied to it alone.  The device arrays
// the sources point to live in P.
void batch_coarsen(const amg_csr* A, int count, const amg_params& p, hipStream_t s, DevPool& P,
                   std::vector<SegSrc>& out);

}  // namespace amg

struct amg_hier {
    using Level = amg::Level;
    using DevPool = amg::DevPool;
    using Timer = amg::Timer;
    using Reducer = amg::Reducer;
    amg_params p{};
    std::vector<Level> lev;
    int n_coarse = 0;
    double* ainv_t = nullptr;
    DevPool pool;
    double setup_ms = 0.0;  // host wall time of the setup call
    hipStream_t stream = nullptr;
    std::vector<int> rounds;
    std::vector<double> match_ms;  // GPU time of each matching pass (with its numbering)
    std::vector<int> pass_n;       // rows and entries of the operator each pass matched
    std::vector<int64_t> pass_nnz;
    // Krylov workspace (allocated on first solve)
    double *r = nullptr, *z = nullptr, *pv[2] = {nullptr, nullptr}, *q = nullptr, *rb = nullptr, *pt = nullptr,
           *sv = nullptr, *st = nullptr, *t = nullptr;
    void* g0 = nullptr;  // D^{-1} times the level-0 right-hand side of the V-cycle
    bool prec32 = false;  // V-cycle in float (values, vectors, accumulation)
    double* S = nullptr;
    double* part = nullptr;
    int* err = nullptr;
    int stream_min = 262144;  // levels with at least this many rows use CSR-stream kernels
    // the PCG iteration's reductions are added by their consumer kernels
    // (HEMAMG_FUSE_DOTS=0: separate finish kernels); partial counts pending
    bool fuse_dots = true;
    int rz_np = 0, rr_np = 0, pq_np = 0;
    double* S_host = nullptr;  // pinned, mapped and coherent host block of the slots
    double* S_dev = nullptr;   // the same block's device address
    unsigned long long seq = 0;  // sequence number of the last eager PCG iteration enqueued
    Timer tim[3];
    // PCG iteration graphs (one per ping-pong parity), replayed on gstream
    bool use_graphs = false;  // HEMAMG_GRAPHS=1: replay PCG iterations from HIP graphs
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipGraphExec_t g_full[2] = {nullptr, nullptr};  // whole iteration
    hipGraphExec_t g_a[2] = {nullptr, nullptr};     // up to the level-0 postsmoothing (timed mode)
    hipGraphExec_t g_b[2] = {nullptr, nullptr};     // after it (timed mode)
    const double* g_key_b = nullptr;
    double* g_key_x = nullptr;

    Reducer reducer() const { return Reducer{part, S}; }

    void drop_graphs() {
        for (int t = 0; t < 2; ++t) {
            for (hipGraphExec_t* e : {&g_full[t], &g_a[t], &g_b[t]})
                if (*e) {
                    (void)hipGraphExecDestroy(*e);
                    *e = nullptr;
                }
        }
        g_key_b = nullptr;
        g_key_x = nullptr;
    }

    ~amg_hier() {
        drop_graphs();
        if (gstream) (void)hipStreamSynchronize(gstream);
        if (stream) (void)hipStreamSynchronize(stream);
        pool.release();
        if (stream) (void)hipStreamSynchronize(stream);
        amg::pinned_put(S_host);
        for (auto& T : tim)
            for (hipEvent_t e : T.ev) amg::event_put(e, true);
        for (hipEvent_t e : gev)
            if (e) amg::event_put(e, false);
        if (gstream) amg::stream_put(gstream);
    }
};
