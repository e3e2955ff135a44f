// Batched solves: many independent systems of different sizes advanced
// together, each kernel launch covering every system of the batch.
//
// A batch is assembled from hierarchies built by amg_setup.  Level k of the
// batch stores, one after another, the level-k operators of the systems for
// which level k is not yet the coarsest ("smoothing rows"); the level-k
// vectors hold those rows followed by the coarsest rows of the systems whose
// coarsest level is k.  Aggregate member lists are renumbered into these
// layouts, so the V-cycle of Algorithm 1 runs the ordinary level kernels on
// the concatenated levels (one launch per level and step for the whole batch)
// and one launch solves every coarsest system.  The CSR-stream kernels add a
// row's products in entry order, so each row's result is the same whatever
// else shares the batch.  The preconditioned CG iteration (Algorithm 4) keeps
// one set of scalars per system (segmented reductions in k_batch.hip), and a
// system that has converged or broken down is masked off while the others
// continue.  Each iteration is replayed from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "amg_host.hpp"

namespace {

using namespace amg;

enum BSlot { B_BB = 0, B_RR, B_TRR, B_PQ, B_RHO0, B_RHO1, B_TT, B_TS };  // B_PQ is (rbar, v) in BiCGStab
static_assert(B_TS < kBatchSlots, "slots per system");

struct BLev {
    int n = 0;        // smoothing rows
    int V = 0;        // vector rows: smoothing rows, then coarsest rows
    int64_t nnz = 0;  // entries of the smoothing rows
    int* rp = nullptr;
    int* ci = nullptr;
    double* v = nullptr;
    float* v32 = nullptr;
    double* dinv = nullptr;  // [V]
    float* dinv32 = nullptr;
    int4* mem = nullptr;  // [V of level k+1] members of each coarse row
    void* f = nullptr;    // [V] (k >= 1)
    void* g = nullptr;    // [V] (k >= 1)
    void* x = nullptr;    // [V] (k >= 1)
    void* xp = nullptr;   // [n]
    void* t = nullptr;    // [n]
    int rb = 256;         // rows per block of the level's CSR-stream kernels
};

struct BSeg {
    amg_status status = AMG_OK;  // a system whose setup failed takes no rows
    int nlev = 0;
    int n0 = 0;     // level-0 rows
    int off0 = 0;   // first level-0 row
    int m = 0;      // coarsest rows
    int cl = 0;     // coarsest level
    int crow0 = 0;  // first coarsest row in the level-cl vectors
};

template <class F>
hipGraphExec_t capture_graph(hipStream_t s, F&& body) {
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

}  // namespace

struct amg_batch {
    int nseg = 0;
    bool prec32 = false;
    double omega = 0.0;
    int period = 50;
    std::vector<BLev> lev;
    std::vector<BSeg> seg;
    int n0 = 0;    // rows of the level-0 vectors
    int nblk = 0;  // reduction blocks over level 0
    int ndblk = 0; // blocks of the coarsest solves
    // device tables
    int2* btab = nullptr;
    int* seg_end = nullptr;
    int* seg_blk = nullptr;
    int* act = nullptr;   // systems still iterating
    int* mark = nullptr;  // systems whose residual is recomputed
    int* all = nullptr;   // every system
    void* dd = nullptr;   // BDense<T>[nseg]
    int2* dtab = nullptr;
    double* ainv = nullptr;
    double* S = nullptr;
    double* part = nullptr;
    // Krylov vectors over level 0
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *pv[2] = {nullptr, nullptr}, *q = nullptr;
    void* g0 = nullptr;
    double *rb = nullptr, *pt = nullptr, *sv = nullptr, *st = nullptr, *t = nullptr;  // BiCGStab, on first use
    hipGraphExec_t bgraph[2] = {nullptr, nullptr};                                   // BiCGStab iterations
    int* err = nullptr;
    // host side
    double* S_host = nullptr;  // pinned [nseg * kBatchSlots]
    int* mask_host = nullptr;  // pinned [nseg]
    void* pinned = nullptr;
    bool pinned_pooled = false;  // a block of the process-wide pinned pool
    bool use_graphs = true;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    amg::DevPool pool;
    double setup_ms = 0.0;  // amg_batch_setup: host wall time of the call

    BatchTab tab(const int* mask) const { return BatchTab{btab, seg_end, mask}; }

    ~amg_batch() {
        for (hipGraphExec_t& g : graph)
            if (g) (void)hipGraphExecDestroy(g);
        for (hipGraphExec_t& g : bgraph)
            if (g) (void)hipGraphExecDestroy(g);
        if (stream) (void)hipStreamSynchronize(stream);
        pool.release();
        if (stream) (void)hipStreamSynchronize(stream);
        if (pinned) {
            if (pinned_pooled) amg::pinned_put(pinned);
            else (void)hipHostFree(pinned);
        }
        for (hipEvent_t e : ev)
            if (e) amg::event_put(e, false);
        if (stream) amg::stream_put(stream);
    }
};

namespace {

template <class T>
const T* vals(const BLev& L);
template <>
const double* vals<double>(const BLev& L) {
    return L.v;
}
template <>
const float* vals<float>(const BLev& L) {
    return L.v32;
}
template <class T>
const T* dinvs(const BLev& L);
template <>
const double* dinvs<double>(const BLev& L) {
    return L.dinv;
}
template <>
const float* dinvs<float>(const BLev& L) {
    return L.dinv32;
}

// Algorithm 1 over the whole batch: z = V(r), g0 = D^{-1} r on level 0.
template <class T>
void batch_vcycle(const amg_batch* B, const double* r, double* z, hipStream_t s) {
    const int K = (int)B->lev.size();
    const T w = T(B->omega);
    auto vec = [](void* p) { return static_cast<T*>(p); };
    const T* g0 = static_cast<const T*>(B->g0);
    auto gk = [&](int k) { return k == 0 ? g0 : static_cast<const T*>(B->lev[k].g); };
    auto view = [&](int k) {
        const BLev& L = B->lev[k];
        return VLevel<T>{L.n, L.rp, L.ci, vals<T>(L), dinvs<T>(L), L.mem, 4, L.rb};
    };
    for (int k = 0; k + 1 < K; ++k) {
        const BLev& L = B->lev[k];
        const BLev& C = B->lev[k + 1];
        if (k == 0) vc_stream_resid<T, double>(view(0), r, g0, w, vec(L.t), s);
        else vc_stream_resid<T, T>(view(k), vec(L.f), gk(k), w, vec(L.t), s);
        vc_restrict<T>(C.V, L.mem, vec(L.t), dinvs<T>(C), vec(C.f), vec(C.g), s);
    }
    launch_bdense<T>(B->ndblk, static_cast<const BDense<T>*>(B->dd), B->dtab, s);
    for (int k = K - 2; k >= 1; --k) {
        const BLev& L = B->lev[k];
        const ScatterT<T> sc{B->lev[k - 1].mem, gk(k - 1), vec(B->lev[k - 1].xp), w};
        vc_stream_post<T, T>(view(k), vec(L.xp), gk(k), w, vec(L.x), nullptr, nullptr, -1, &sc, s);
    }
    vc_stream_post<T, double>(view(0), vec(B->lev[0].xp), g0, w, z, nullptr, nullptr, -1, nullptr, s);
}

// Level k's two steps of the batched V-cycle (for the autotuner).
template <class T>
void batch_level_steps(const amg_batch* B, int k, hipStream_t s) {
    const T w = T(B->omega);
    auto vec = [](void* p) { return static_cast<T*>(p); };
    const BLev& L = B->lev[k];
    const BLev& C = B->lev[k + 1];
    const VLevel<T> V{L.n, L.rp, L.ci, vals<T>(L), dinvs<T>(L), L.mem, 4, L.rb};
    const T* g = k == 0 ? static_cast<const T*>(B->g0) : static_cast<const T*>(L.g);
    if (k == 0) vc_stream_resid<T, double>(V, B->r, g, w, vec(L.t), s);
    else vc_stream_resid<T, T>(V, vec(L.f), g, w, vec(L.t), s);
    vc_restrict<T>(C.V, L.mem, vec(L.t), dinvs<T>(C), vec(C.f), vec(C.g), s);
    if (k == 0) {
        vc_stream_post<T, double>(V, vec(L.xp), g, w, B->z, nullptr, nullptr, -1, nullptr, s);
        return;
    }
    const BLev& F = B->lev[k - 1];
    const ScatterT<T> sc{F.mem, k - 1 == 0 ? static_cast<const T*>(B->g0) : static_cast<const T*>(F.g),
                         vec(F.xp), w};
    vc_stream_post<T, T>(V, vec(L.xp), g, w, vec(L.x), nullptr, nullptr, -1, &sc, s);
}

void vcycle(const amg_batch* B, const double* r, double* z, hipStream_t s) {
    if (B->prec32) batch_vcycle<float>(B, r, z, s);
    else batch_vcycle<double>(B, r, z, s);
}

void finish(const amg_batch* B, const int* mask, int slot_k, hipStream_t s) {
    launch_bfinish(B->nseg, B->seg_blk, mask, B->part, B->S, slot_k, s);
}

// One CG iteration of parity pc for the systems in `act`: q = A p, (p, q);
// x, r update, (r, r), g0; z = V(r); (r, z); next direction.
void iteration(const amg_batch* B, int pc, hipStream_t s) {
    const int cur = pc ? B_RHO1 : B_RHO0, nxt = pc ? B_RHO0 : B_RHO1;
    const BLev& L0 = B->lev[0];
    const BatchTab T = B->tab(B->act);
    double* p = B->pv[pc];
    launch_bspmv_dot(B->nblk, T, L0.rp, L0.ci, L0.v, p, B->q, p, B->part, s);
    finish(B, B->act, B_PQ, s);
    launch_bcg_update(B->nblk, T, B->x, B->r, p, B->q, L0.dinv, B->g0, B->prec32, B->part, B->S, cur, B_PQ, s);
    finish(B, B->act, B_RR, s);
    vcycle(B, B->r, B->z, s);
    launch_bdot(B->nblk, T, B->r, B->z, B->part, s);
    finish(B, B->act, nxt, s);
    launch_bcg_dir(B->nblk, T, B->z, p, B->pv[1 - pc], B->S, nxt, cur, s);
}

void read_slots(amg_batch* B, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(B->S_host, B->S, sizeof(double) * kBatchSlots * B->nseg, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

void upload_mask(amg_batch* B, const std::vector<char>& on, int* dst, hipStream_t s) {
    for (int i = 0; i < B->nseg; ++i) B->mask_host[i] = on[i] ? 1 : 0;
    HIPCHK(hipMemcpyAsync(dst, B->mask_host, sizeof(int) * B->nseg, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // the pinned words are reused by the next upload
}

inline bool usable(double d) { return std::isfinite(d) && d != 0.0; }

}  // namespace

namespace amg {

// Algorithm 4 for every system of a batch, advanced one iteration at a time,
// with the stop rule, residual replacement and breakdown checks of the
// single-system solver applied per system.  A system leaves the iteration as
// soon as it is done; its iterate then no longer changes.
struct PcgRun {
    amg_batch* B = nullptr;
    double rtol = 0.0;
    int maxit = 0;
    hipStream_t s = nullptr;
    std::vector<amg_info> info;
    std::vector<double> nb;
    std::vector<char> act, mark, zero;
    int it = 0, pc = 0, live = 0;
    bool pending = false;  // an iteration was enqueued and not collected
};

namespace {
double slot(const PcgRun& R, int i, int k) { return R.B->S_host[(size_t)i * kBatchSlots + k]; }
}  // namespace

PcgRun* pcg_run_start(amg_batch* B, double rtol, int maxit, std::vector<int>& done) {
    std::unique_ptr<PcgRun> R(new PcgRun());
    R->B = B;
    R->rtol = rtol;
    R->maxit = maxit;
    R->s = B->stream;
    hipStream_t s = R->s;
    const int ns = B->nseg;
    const BLev& L0 = B->lev[0];
    R->info.assign(ns, amg_info{});
    R->nb.assign(ns, 0.0);
    R->act.assign(ns, 1);
    R->mark.assign(ns, 0);
    R->zero.assign(ns, 0);
    // (b, b) and r = b - A x, g0 = D^{-1} r
    launch_bdot(B->nblk, B->tab(B->all), B->b, B->b, B->part, s);
    finish(B, B->all, B_BB, s);
    launch_bresidual(B->nblk, B->tab(B->all), L0.rp, L0.ci, L0.v, B->x, B->b, B->r, L0.dinv, B->g0, B->prec32,
                     B->part, s);
    finish(B, B->all, B_RR, s);
    read_slots(B, s);
    bool any_zero = false;
    for (int i = 0; i < ns; ++i) {
        if (B->seg[i].status != AMG_OK) {  // its setup failed: nothing to solve
            R->info[i].status = B->seg[i].status;
            R->act[i] = 0;
            done.push_back(i);
            continue;
        }
        R->nb[i] = std::sqrt(slot(*R, i, B_BB));
        if (R->nb[i] == 0.0) {  // x = 0 is the solution
            R->zero[i] = 1;
            any_zero = true;
            R->act[i] = 0;
            done.push_back(i);
            continue;
        }
        const double rel = std::sqrt(slot(*R, i, B_RR)) / R->nb[i];
        R->info[i].rel_res = R->info[i].true_rel_res = rel;
        if (rel <= rtol) {
            R->act[i] = 0;
            done.push_back(i);
        }
        R->live += R->act[i];
    }
    if (any_zero) {
        upload_mask(B, R->zero, B->mark, s);
        launch_bzero(B->nblk, B->tab(B->mark), B->x, s);
    }
    if (R->live > 0 && maxit <= 0) {  // no iteration allowed
        for (int i = 0; i < ns; ++i)
            if (R->act[i]) {
                R->info[i].status = AMG_ENOTCONV;
                R->act[i] = 0;
                done.push_back(i);
            }
        R->live = 0;
    }
    upload_mask(B, R->act, B->act, s);
    if (R->live == 0) {
        HIPCHK(hipStreamSynchronize(s));
        return R.release();
    }
    vcycle(B, B->r, B->z, s);
    launch_bdot(B->nblk, B->tab(B->act), B->r, B->z, B->part, s);
    finish(B, B->act, B_RHO0, s);
    HIPCHK(hipMemcpyAsync(B->pv[0], B->z, sizeof(double) * B->n0, hipMemcpyDeviceToDevice, s));
    if (B->use_graphs && !B->graph[0]) {
        for (int pc = 0; pc < 2; ++pc) B->graph[pc] = capture_graph(s, [&] { iteration(B, pc, s); });
    }
    HIPCHK(hipGetLastError());
    return R.release();
}

void pcg_run_enqueue(PcgRun* R) {
    if (R->live == 0 || R->pending) return;
    amg_batch* B = R->B;
    if (B->use_graphs) HIPCHK(hipGraphLaunch(B->graph[R->pc], R->s));
    else iteration(B, R->pc, R->s);
    HIPCHK(hipMemcpyAsync(B->S_host, B->S, sizeof(double) * kBatchSlots * B->nseg, hipMemcpyDeviceToHost, R->s));
    HIPCHK(hipGetLastError());
    R->pending = true;
}

void pcg_run_collect(PcgRun* R, std::vector<int>& done) {
    if (!R->pending) return;
    R->pending = false;
    amg_batch* B = R->B;
    hipStream_t s = R->s;
    const int ns = B->nseg;
    const BLev& L0 = B->lev[0];
    HIPCHK(hipStreamSynchronize(s));
    const int it = ++R->it;
    const int pc = R->pc;
    const int cur = pc ? B_RHO1 : B_RHO0, nxt = pc ? B_RHO0 : B_RHO1;
    std::vector<char>& act = R->act;
    std::vector<char>& mark = R->mark;
    bool any_mark = false, changed = false;
    auto leave = [&](int i) {
        act[i] = 0;
        changed = true;
        done.push_back(i);
    };
    for (int i = 0; i < ns; ++i) {
        if (!act[i]) continue;
        if (!usable(slot(*R, i, B_PQ)) || !std::isfinite(slot(*R, i, cur))) {
            R->info[i].status = AMG_EBREAKDOWN;
            leave(i);
            continue;
        }
        R->info[i].iters = it;
        const double rel = std::sqrt(slot(*R, i, B_RR)) / R->nb[i];
        R->info[i].rel_res = rel;
        if (!std::isfinite(rel)) {
            R->info[i].status = AMG_EBREAKDOWN;
            leave(i);
            continue;
        }
        mark[i] = rel <= R->rtol || (B->period > 0 && it % B->period == 0);
        any_mark |= mark[i] != 0;
    }
    if (any_mark) {  // recompute b - A x (residual replacement) for the marked systems
        upload_mask(B, mark, B->mark, s);
        launch_bresidual(B->nblk, B->tab(B->mark), L0.rp, L0.ci, L0.v, B->x, B->b, B->r, L0.dinv, B->g0,
                         B->prec32, B->part, s);
        finish(B, B->mark, B_TRR, s);
        read_slots(B, s);
        bool again = false;
        for (int i = 0; i < ns; ++i) {
            if (!mark[i]) continue;
            const double tr = std::sqrt(slot(*R, i, B_TRR)) / R->nb[i];
            R->info[i].true_rel_res = tr;
            if (tr <= R->rtol) {
                mark[i] = 0;
                leave(i);
            } else {
                again = true;
            }
        }
        if (again) {  // restart the direction from the recomputed residual
            upload_mask(B, mark, B->mark, s);
            vcycle(B, B->r, B->z, s);
            launch_bdot(B->nblk, B->tab(B->mark), B->r, B->z, B->part, s);
            finish(B, B->mark, nxt, s);
            launch_bcg_dir(B->nblk, B->tab(B->mark), B->z, B->pv[pc], B->pv[1 - pc], B->S, nxt, cur, s);
            read_slots(B, s);
        }
        std::fill(mark.begin(), mark.end(), 0);
    }
    for (int i = 0; i < ns; ++i) {
        if (act[i] && !usable(slot(*R, i, nxt))) {
            R->info[i].status = AMG_EBREAKDOWN;
            leave(i);
        }
    }
    R->live = 0;
    for (int i = 0; i < ns; ++i) R->live += act[i];
    if (R->live > 0 && it >= R->maxit) {  // iteration limit
        for (int i = 0; i < ns; ++i)
            if (act[i]) {
                R->info[i].status = AMG_ENOTCONV;
                act[i] = 0;
                done.push_back(i);
            }
        R->live = 0;
    } else if (changed && R->live > 0) {
        upload_mask(B, act, B->act, s);
    }
    R->pc = 1 - pc;
}

int pcg_run_live(const PcgRun* R) { return R->live; }
const amg_info& pcg_run_info(const PcgRun* R, int i) { return R->info[i]; }
void pcg_run_end(PcgRun* R) { delete R; }

}  // namespace amg

namespace {

void batch_pcg(amg_batch* B, double rtol, int maxit, hipStream_t s, amg_info* info) {
    (void)s;  // the run uses the batch's own stream
    std::vector<int> done;
    std::unique_ptr<PcgRun> R(pcg_run_start(B, rtol, maxit, done));
    while (R->live > 0 && R->it < maxit) {
        pcg_run_enqueue(R.get());
        pcg_run_collect(R.get(), done);
    }
    for (int i = 0; i < B->nseg; ++i) info[i] = R->info[i];
}

// D^{-1} v into the level-0 slot the V-cycle reads (a preconditioner input
// other than the CG residual).
void scale_dinv(const amg_batch* B, const double* v, hipStream_t s) {
    const BLev& L0 = B->lev[0];
    if (B->prec32) vc_scale_dinv<float>(B->n0, L0.dinv, v, static_cast<float*>(B->g0), s);
    else vc_scale_dinv<double>(B->n0, L0.dinv, v, static_cast<double*>(B->g0), s);
}

// One BiCGStab iteration for the systems in `act`; pc selects the direction
// pair and the (r, rbar) slots (they alternate together).
void bicg_iteration(const amg_batch* B, int pc, hipStream_t s) {
    const int cur = pc ? B_RHO1 : B_RHO0, nxt = pc ? B_RHO0 : B_RHO1;
    const BLev& L0 = B->lev[0];
    const BatchTab T = B->tab(B->act);
    const double* p = B->pv[pc];
    double* pn = B->pv[1 - pc];
    scale_dinv(B, p, s);
    vcycle(B, p, B->pt, s);
    launch_bspmv_dot(B->nblk, T, L0.rp, L0.ci, L0.v, B->pt, B->q, B->rb, B->part, s);
    finish(B, B->act, B_PQ, s);
    launch_bbicg_s(B->nblk, T, B->r, B->q, B->sv, B->S, cur, B_PQ, s);
    scale_dinv(B, B->sv, s);
    vcycle(B, B->sv, B->st, s);
    launch_bspmv_dot2(B->nblk, T, L0.rp, L0.ci, L0.v, B->st, B->t, B->sv, B->part, s);
    launch_bfinish(B->nseg, B->seg_blk, B->act, B->part, B->S, B_TT, s);
    launch_bfinish(B->nseg, B->seg_blk, B->act, B->part + B->nblk, B->S, B_TS, s);
    launch_bbicg_update(B->nblk, T, B->x, B->r, B->pt, B->st, B->sv, B->t, B->rb, B->part, B->S, cur, B_PQ, B_TT,
                        B_TS, s);
    launch_bfinish(B->nseg, B->seg_blk, B->act, B->part, B->S, B_RR, s);
    launch_bfinish(B->nseg, B->seg_blk, B->act, B->part + B->nblk, B->S, nxt, s);
    launch_bbicg_dir(B->nblk, T, B->r, p, B->q, pn, B->S, cur, B_PQ, B_TT, B_TS, nxt, s);
}

// Algorithm 5 (right preconditioned, p_0 = r_0 = shadow residual) for every
// system, with the stop rule, residual replacement and breakdown checks of
// the single-system solver applied per system.
void batch_bicgstab(amg_batch* B, double rtol, int maxit, hipStream_t s, amg_info* info) {
    const int ns = B->nseg;
    const BLev& L0 = B->lev[0];
    if (!B->rb) {
        const int n0 = B->n0;
        B->rb = B->pool.get<double>(n0);
        B->pt = B->pool.get<double>(n0);
        B->sv = B->pool.get<double>(n0);
        B->st = B->pool.get<double>(n0);
        B->t = B->pool.get<double>(n0);
    }
    const double* S = B->S_host;
    auto sv = [&](int i, int k) { return S[(size_t)i * kBatchSlots + k]; };
    std::vector<double> nb(ns, 0.0);
    std::vector<char> act(ns, 1), mark(ns, 0), zero(ns, 0);
    for (int i = 0; i < ns; ++i) info[i] = amg_info{};
    launch_bdot(B->nblk, B->tab(B->all), B->b, B->b, B->part, s);
    finish(B, B->all, B_BB, s);
    launch_bresidual(B->nblk, B->tab(B->all), L0.rp, L0.ci, L0.v, B->x, B->b, B->r, L0.dinv, B->g0, B->prec32,
                     B->part, s);
    finish(B, B->all, B_RR, s);
    read_slots(B, s);
    bool any_zero = false;
    int live = 0;
    for (int i = 0; i < ns; ++i) {
        if (B->seg[i].status != AMG_OK) {
            info[i].status = B->seg[i].status;
            act[i] = 0;
            continue;
        }
        nb[i] = std::sqrt(sv(i, B_BB));
        if (nb[i] == 0.0) {
            zero[i] = 1;
            any_zero = true;
            act[i] = 0;
            continue;
        }
        const double rel = std::sqrt(sv(i, B_RR)) / nb[i];
        info[i].rel_res = info[i].true_rel_res = rel;
        if (rel <= rtol) act[i] = 0;
        live += act[i];
    }
    if (any_zero) {
        upload_mask(B, zero, B->mark, s);
        launch_bzero(B->nblk, B->tab(B->mark), B->x, s);
    }
    upload_mask(B, act, B->act, s);
    if (live == 0) return;
    HIPCHK(hipMemcpyAsync(B->rb, B->r, sizeof(double) * B->n0, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(B->pv[0], B->r, sizeof(double) * B->n0, hipMemcpyDeviceToDevice, s));
    launch_bdot(B->nblk, B->tab(B->act), B->r, B->rb, B->part, s);
    finish(B, B->act, B_RHO0, s);
    if (B->use_graphs && !B->bgraph[0]) {
        for (int pc = 0; pc < 2; ++pc) B->bgraph[pc] = capture_graph(s, [&] { bicg_iteration(B, pc, s); });
    }
    int pc = 0;
    for (int it = 1; it <= maxit && live > 0; ++it) {
        const int cur = pc ? B_RHO1 : B_RHO0, nxt = pc ? B_RHO0 : B_RHO1;
        if (B->use_graphs) HIPCHK(hipGraphLaunch(B->bgraph[pc], s));
        else bicg_iteration(B, pc, s);
        read_slots(B, s);
        bool any_mark = false, changed = false;
        std::vector<double> omega(ns, 0.0);
        for (int i = 0; i < ns; ++i) {
            if (!act[i]) continue;
            const bool bad = !usable(sv(i, B_PQ)) || !usable(sv(i, cur)) || !std::isfinite(sv(i, B_TT)) ||
                             !std::isfinite(sv(i, B_TS)) || sv(i, B_TT) == 0.0;
            if (bad) {
                info[i].status = AMG_EBREAKDOWN;
                act[i] = 0;
                changed = true;
                continue;
            }
            omega[i] = sv(i, B_TS) / sv(i, B_TT);
            info[i].iters = it;
            const double rel = std::sqrt(sv(i, B_RR)) / nb[i];
            info[i].rel_res = rel;
            if (!std::isfinite(rel)) {
                info[i].status = AMG_EBREAKDOWN;
                act[i] = 0;
                changed = true;
                continue;
            }
            mark[i] = rel <= rtol || (B->period > 0 && it % B->period == 0);
            any_mark |= mark[i] != 0;
        }
        if (any_mark) {  // recompute b - A x (residual replacement) for the marked systems
            upload_mask(B, mark, B->mark, s);
            launch_bresidual(B->nblk, B->tab(B->mark), L0.rp, L0.ci, L0.v, B->x, B->b, B->r, L0.dinv, B->g0,
                             B->prec32, B->part, s);
            finish(B, B->mark, B_TRR, s);
            read_slots(B, s);
            bool again = false;
            for (int i = 0; i < ns; ++i) {
                if (!mark[i]) continue;
                const double tr = std::sqrt(sv(i, B_TRR)) / nb[i];
                info[i].true_rel_res = tr;
                if (tr <= rtol) {
                    act[i] = 0;
                    mark[i] = 0;
                    changed = true;
                } else {
                    again = true;
                }
            }
            if (again) {  // the next direction from the recomputed residual
                upload_mask(B, mark, B->mark, s);
                launch_bdot(B->nblk, B->tab(B->mark), B->r, B->rb, B->part, s);
                finish(B, B->mark, nxt, s);
                launch_bbicg_dir(B->nblk, B->tab(B->mark), B->r, B->pv[pc], B->q, B->pv[1 - pc], B->S, cur, B_PQ,
                                 B_TT, B_TS, nxt, s);
                read_slots(B, s);
            }
            std::fill(mark.begin(), mark.end(), 0);
        }
        for (int i = 0; i < ns; ++i) {
            if (act[i] && (omega[i] == 0.0 || !usable(sv(i, nxt)))) {
                info[i].status = AMG_EBREAKDOWN;
                act[i] = 0;
                changed = true;
            }
        }
        live = 0;
        for (int i = 0; i < ns; ++i) live += act[i];
        if (changed && live > 0) upload_mask(B, act, B->act, s);
        pc = 1 - pc;
    }
    for (int i = 0; i < ns; ++i)
        if (act[i]) info[i].status = AMG_ENOTCONV;
}

template <class T>
void build_dense(amg_batch* B, std::vector<char>& host, size_t at_dd, size_t at_dtab, const std::vector<size_t>& aoff) {
    BDense<T>* dd = reinterpret_cast<BDense<T>*>(host.data() + at_dd);
    int2* dtab = reinterpret_cast<int2*>(host.data() + at_dtab);
    const T w = T(B->omega);
    int nb = 0;
    for (int i = 0; i < B->nseg; ++i) {
        const BSeg& g = B->seg[i];
        if (g.status != AMG_OK) {
            dd[i] = BDense<T>{};
            continue;
        }
        const BLev& C = B->lev[g.cl];
        const BLev& F = B->lev[g.cl - 1];
        const T* gf = g.cl - 1 == 0 ? static_cast<const T*>(B->g0) : static_cast<const T*>(F.g);
        dd[i] = BDense<T>{g.m,
                          g.crow0,
                          B->ainv + aoff[i],
                          static_cast<const T*>(C.f) + g.crow0,
                          static_cast<T*>(C.x) + g.crow0,
                          ScatterT<T>{F.mem, gf, static_cast<T*>(F.xp), w}};
        for (int c = 0; c * 64 < g.m; ++c) dtab[nb++] = make_int2(i, c);
    }
}

// Lays out a batch from the systems' levels wherever they are stored (see
// SegSrc); blocks the host until the copies are done.
void create_impl(const std::vector<SegSrc>& src, bool prec32, double omega, int period, const amg_allocator& al,
                 hipStream_t caller, amg_batch** out) {
    const int count = (int)src.size();
    std::unique_ptr<amg_batch> B(new amg_batch());
    B->nseg = count;
    B->prec32 = prec32;
    B->omega = omega;
    B->period = period;
    B->stream = stream_get();
    B->ev[0] = event_get(false);
    B->ev[1] = event_get(false);
    hipStream_t s = B->stream;
    HIPCHK(hipEventRecord(B->ev[0], caller));
    HIPCHK(hipStreamWaitEvent(s, B->ev[0], 0));
    B->pool.s = s;
    B->pool.al = al;
    const int ns = count;
    int K = 0;
    for (int i = 0; i < ns; ++i) K = std::max(K, (int)src[i].lev.size());
    if (K < 2) raise(AMG_EINVAL, "amg_batch: no system with two or more levels");
    B->lev.resize(K);
    B->seg.resize(ns);
    // layouts: pos[k][i] = first row of system i in the level-k vectors
    std::vector<std::vector<int>> pos(K, std::vector<int>(ns, -1));
    std::vector<std::vector<int64_t>> epos(K, std::vector<int64_t>(ns, 0));
    for (int k = 0; k < K; ++k) {
        BLev& L = B->lev[k];
        for (int i = 0; i < ns; ++i) {
            const int nl = (int)src[i].lev.size();
            if (k == 0) pos[k][i] = L.n;  // a failed system sits empty at its place
            if (k <= nl - 2) {
                pos[k][i] = L.n;
                epos[k][i] = L.nnz;
                L.n += src[i].lev[k].n;
                L.nnz += src[i].lev[k].nnz;
            }
        }
        L.V = L.n;
        for (int i = 0; i < ns; ++i) {
            if ((int)src[i].lev.size() - 1 == k) {
                pos[k][i] = L.V;
                L.V += src[i].lev[k].n;
            }
        }
        if ((int64_t)L.V >= (int64_t)1 << 31 || L.nnz >= (int64_t)1 << 31)
            raise(AMG_EINVAL, "amg_batch_create: the batch exceeds 2^31 rows or entries on a level");
    }
    for (int i = 0; i < ns; ++i) {
        BSeg& g = B->seg[i];
        g.status = src[i].lev.size() >= 2 ? src[i].status : (src[i].status != AMG_OK ? src[i].status : AMG_EINVAL);
        g.off0 = pos[0][i];
        if (g.status != AMG_OK) continue;  // no rows, no levels
        g.nlev = (int)src[i].lev.size();
        g.n0 = src[i].lev[0].n;
        g.cl = g.nlev - 1;
        g.m = src[i].lev[g.cl].n;
        g.crow0 = pos[g.cl][i];
    }
    B->n0 = B->lev[0].n;
    const size_t esz = B->prec32 ? 4 : 8;
    // device memory
    DevPool& P = B->pool;
    size_t bytes = 0;
    for (const BLev& L : B->lev) bytes += 4 * (size_t)L.n + 12 * (size_t)L.nnz + 40 * (size_t)L.V + 2 * esz * L.n;
    P.hint(bytes + 80 * (size_t)B->n0 + (1u << 20));
    for (int k = 0; k < K; ++k) {
        BLev& L = B->lev[k];
        if (L.n > 0) {
            L.rp = P.get<int>((size_t)L.n + 1);
            L.ci = P.get<int>((size_t)L.nnz);
            L.v = P.get<double>((size_t)L.nnz);
            if (B->prec32) L.v32 = P.get<float>((size_t)L.nnz);
            L.mem = P.get<int4>((size_t)B->lev[k + 1].V);
            L.xp = P.get<char>(esz * L.n);
            L.t = P.get<char>(esz * L.n);
        }
        L.dinv = P.get<double>((size_t)L.V);
        if (B->prec32) L.dinv32 = P.get<float>((size_t)L.V);
        if (k > 0) {
            L.f = P.get<char>(esz * L.V);
            L.g = P.get<char>(esz * L.V);
            L.x = P.get<char>(esz * L.V);
        }
    }
    const int n0 = B->n0;
    B->b = P.get<double>(n0);
    B->x = P.get<double>(n0);
    B->r = P.get<double>(n0);
    B->z = P.get<double>(n0);
    B->pv[0] = P.get<double>(n0);
    B->pv[1] = P.get<double>(n0);
    B->q = P.get<double>(n0);
    B->g0 = P.get<char>(esz * n0);
    B->err = P.get<int>(1);
    std::vector<size_t> aoff(ns);
    size_t asz = 0;
    for (int i = 0; i < ns; ++i) {
        aoff[i] = asz;
        asz += (size_t)B->seg[i].m * B->seg[i].m;
    }
    B->ainv = P.get<double>(asz);
    // reduction blocks: 256 rows each from every system's first row
    std::vector<int> segblk(ns + 1, 0);
    for (int i = 0; i < ns; ++i) segblk[i + 1] = segblk[i] + (B->seg[i].n0 + 255) / 256;
    B->nblk = segblk[ns];
    int ndb = 0;
    for (int i = 0; i < ns; ++i) ndb += (B->seg[i].m + 63) / 64;
    B->ndblk = ndb;
    B->part = P.get<double>(2 * (size_t)B->nblk);
    B->S = P.get<double>((size_t)ns * kBatchSlots);
    // copies that assemble the levels
    std::vector<GatherPiece> pcs;
    auto piece = [&](const void* src, void* dst, int64_t cnt, int add, int kind) {
        if (cnt > 0) pcs.push_back(GatherPiece{src, dst, cnt, add, kind});
    };
    for (int k = 0; k < K; ++k) {
        BLev& L = B->lev[k];
        int last = -1;
        for (int i = 0; i < ns; ++i)
            if (k <= B->seg[i].nlev - 2) last = i;
        for (int i = 0; i < ns; ++i) {
            const BSeg& g = B->seg[i];
            if (k >= g.nlev) continue;
            const SegLevelSrc& H = src[i].lev[k];
            if (k <= g.nlev - 2) {
                const int o = pos[k][i];
                piece(H.rp, L.rp + o, (int64_t)H.n + (i == last ? 1 : 0), (int)epos[k][i] + H.rp_add, 0);
                piece(H.ci, L.ci + epos[k][i], H.nnz, o + H.ci_add, 0);
                piece(H.v, L.v + epos[k][i], H.nnz, 0, 1);
                if (B->prec32) {
                    if (H.v32) piece(H.v32, L.v32 + epos[k][i], H.nnz, 0, 2);
                    else piece(H.v, L.v32 + epos[k][i], H.nnz, 0, 4);
                }
                piece(H.mem, L.mem + pos[k + 1][i], src[i].lev[k + 1].n, o + H.mem_add, 3);
            }
            piece(H.dinv, L.dinv + pos[k][i], H.n, 0, 1);
            if (B->prec32) {
                if (H.dinv32) piece(H.dinv32, L.dinv32 + pos[k][i], H.n, 0, 2);
                else piece(H.dinv, L.dinv32 + pos[k][i], H.n, 0, 4);
            }
        }
    }
    for (int i = 0; i < ns; ++i)
        if (B->seg[i].status == AMG_OK)
            piece(src[i].ainv_t, B->ainv + aoff[i], (int64_t)B->seg[i].m * B->seg[i].m, 0, 1);
    const int CH = gather_chunk();
    std::vector<int2> gtab;
    for (size_t p = 0; p < pcs.size(); ++p)
        for (int64_t c = 0; c * CH < pcs[p].count; ++c) gtab.push_back(make_int2((int)p, (int)c));
    // host tables, uploaded in one copy
    auto align = [](size_t a) { return (a + 255) & ~size_t(255); };
    const size_t dsz = B->prec32 ? sizeof(BDense<float>) : sizeof(BDense<double>);
    size_t at = 0;
    const size_t at_pcs = at;
    at = align(at + sizeof(GatherPiece) * pcs.size());
    const size_t at_gtab = at;
    at = align(at + sizeof(int2) * gtab.size());
    const size_t at_btab = at;
    at = align(at + sizeof(int2) * B->nblk);
    const size_t at_end = at;
    at = align(at + sizeof(int) * ns);
    const size_t at_sblk = at;
    at = align(at + sizeof(int) * (ns + 1));
    const size_t at_masks = at;
    at = align(at + sizeof(int) * 3 * (size_t)ns);
    const size_t at_dd = at;
    at = align(at + dsz * ns);
    const size_t at_dtab = at;
    at = align(at + sizeof(int2) * ndb);
    std::vector<char> host(at, 0);
    std::memcpy(host.data() + at_pcs, pcs.data(), sizeof(GatherPiece) * pcs.size());
    std::memcpy(host.data() + at_gtab, gtab.data(), sizeof(int2) * gtab.size());
    {
        int2* bt = reinterpret_cast<int2*>(host.data() + at_btab);
        int* se = reinterpret_cast<int*>(host.data() + at_end);
        int* sb = reinterpret_cast<int*>(host.data() + at_sblk);
        int* mk = reinterpret_cast<int*>(host.data() + at_masks);
        for (int i = 0; i < ns; ++i) {
            const BSeg& g = B->seg[i];
            se[i] = g.off0 + g.n0;
            for (int b = segblk[i]; b < segblk[i + 1]; ++b) bt[b] = make_int2(i, g.off0 + 256 * (b - segblk[i]));
            mk[2 * ns + i] = 1;  // `all`
        }
        std::memcpy(sb, segblk.data(), sizeof(int) * (ns + 1));
    }
    char* dev = P.get<char>(at);
    B->btab = reinterpret_cast<int2*>(dev + at_btab);
    B->seg_end = reinterpret_cast<int*>(dev + at_end);
    B->seg_blk = reinterpret_cast<int*>(dev + at_sblk);
    B->act = reinterpret_cast<int*>(dev + at_masks);
    B->mark = B->act + ns;
    B->all = B->act + 2 * ns;
    B->dd = dev + at_dd;
    B->dtab = reinterpret_cast<int2*>(dev + at_dtab);
    if (B->prec32) build_dense<float>(B.get(), host, at_dd, at_dtab, aoff);
    else build_dense<double>(B.get(), host, at_dd, at_dtab, aoff);
    HIPCHK(hipMemcpyAsync(dev, host.data(), at, hipMemcpyHostToDevice, s));
    launch_gather((int)gtab.size(), reinterpret_cast<const GatherPiece*>(dev + at_pcs),
                  reinterpret_cast<const int2*>(dev + at_gtab), s);
    HIPCHK(hipGetLastError());
    // pinned host memory for the scalars and masks: a block of the pinned
    // pool when it fits (pinned allocation costs about a millisecond)
    const size_t pin = sizeof(double) * kBatchSlots * ns + sizeof(int) * ns;
    if (pin <= kPinnedBlock) {
        B->pinned = pinned_get();
        B->pinned_pooled = true;
    } else {
        HIPCHK(hipHostMalloc(&B->pinned, pin, hipHostMallocDefault));
    }
    B->S_host = static_cast<double*>(B->pinned);
    B->mask_host = reinterpret_cast<int*>(B->S_host + (size_t)kBatchSlots * ns);
    if (const char* e = getenv("HEMAMG_BATCH_GRAPHS")) B->use_graphs = atoi(e) != 0;
    HIPCHK(hipStreamSynchronize(s));  // the host tables are consumed
    *out = B.release();
}

// Rows per block of every level's CSR-stream kernels, chosen by timing the
// level's steps on this batch.  A row's sum is formed in entry order whatever
// the block size, so results do not change.
void batch_autotune(amg_batch* B, hipStream_t caller, int32_t* out) {
    hipStream_t s = B->stream;
    HIPCHK(hipEventRecord(B->ev[0], caller));
    HIPCHK(hipStreamWaitEvent(s, B->ev[0], 0));
    const size_t esz = B->prec32 ? 4 : 8;
    const int K = (int)B->lev.size();
    HIPCHK(hipMemsetAsync(B->r, 0, sizeof(double) * B->n0, s));
    HIPCHK(hipMemsetAsync(B->z, 0, sizeof(double) * B->n0, s));
    HIPCHK(hipMemsetAsync(B->g0, 0, esz * B->n0, s));
    for (BLev& L : B->lev) {
        for (void* p : {L.f, L.g, L.x}) if (p) HIPCHK(hipMemsetAsync(p, 0, esz * L.V, s));
        for (void* p : {L.xp, L.t}) if (p) HIPCHK(hipMemsetAsync(p, 0, esz * L.n, s));
    }
    hipEvent_t e0 = event_get(true), e1 = event_get(true);
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            event_put(a, true);
            event_put(b, true);
        }
    } eg{e0, e1};
    const int cand[] = {128, 256, 512};
    for (int k = 0; k < K; ++k) {
        if (out) out[k] = 0;
        if (k + 1 >= K) continue;
        BLev& L = B->lev[k];
        float best = 1e30f;
        int pick = 256;
        for (int rb : cand) {
            L.rb = rb;
            auto step = [&] {
                if (B->prec32) batch_level_steps<float>(B, k, s);
                else batch_level_steps<double>(B, k, s);
            };
            step();
            HIPCHK(hipEventRecord(e0, s));
            for (int r = 0; r < 5; ++r) step();
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipGetLastError());
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                pick = rb;
            }
        }
        L.rb = pick;
        if (out) out[k] = pick;
    }
    for (hipGraphExec_t* gs : {B->graph, B->bgraph})  // re-captured with the new launch shapes
        for (int k = 0; k < 2; ++k)
            if (gs[k]) {
                (void)hipGraphExecDestroy(gs[k]);
                gs[k] = nullptr;
            }
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace

namespace amg {

void gather_run(const std::vector<GatherPiece>& pcs, DevPool& P, hipStream_t s) {
    if (pcs.empty()) return;
    const int CH = gather_chunk();
    std::vector<int2> tab;
    for (size_t p = 0; p < pcs.size(); ++p)
        for (int64_t c = 0; c * CH < pcs[p].count; ++c) tab.push_back(make_int2((int)p, (int)c));
    const size_t a = (sizeof(GatherPiece) * pcs.size() + 255) & ~size_t(255);
    char* dev = P.get<char>(a + sizeof(int2) * tab.size());
    HIPCHK(hipMemcpyAsync(dev, pcs.data(), sizeof(GatherPiece) * pcs.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dev + a, tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice, s));
    launch_gather((int)tab.size(), reinterpret_cast<const GatherPiece*>(dev), reinterpret_cast<const int2*>(dev + a),
                  s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));  // the host tables are consumed
}

void batch_load(amg_batch* B, int i, const double* b, const double* x0, hipStream_t after) {
    const BSeg& g = B->seg[i];
    if (after) {
        HIPCHK(hipEventRecord(B->ev[0], after));
        HIPCHK(hipStreamWaitEvent(B->stream, B->ev[0], 0));
    }
    if (g.n0 == 0) return;
    HIPCHK(hipMemcpyAsync(B->b + g.off0, b, sizeof(double) * g.n0, hipMemcpyDeviceToDevice, B->stream));
    HIPCHK(hipMemcpyAsync(B->x + g.off0, x0, sizeof(double) * g.n0, hipMemcpyDeviceToDevice, B->stream));
}

const double* batch_x(const amg_batch* B, int i, int* n) {
    *n = B->seg[i].n0;
    return B->x + B->seg[i].off0;
}

hipStream_t batch_stream(const amg_batch* B) { return B->stream; }
size_t batch_bytes(const amg_batch* B) { return B->pool.bytes; }

void batch_fill_info(const amg_batch* B, int i, amg_info& I) {
    I.setup_ms = B->setup_ms;
    I.levels = B->seg[i].nlev;
}

}  // namespace amg

extern "C" {

amg_status amg_batch_create(const amg_hier* const* hiers, int32_t count, const amg_allocator* alloc, void* stream,
                            amg_batch** out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!hiers || !out || count < 1 || count > (1 << 20)) raise(AMG_EINVAL, "amg_batch_create: bad arguments");
        const amg_allocator al = checked_allocator(alloc);
        std::vector<SegSrc> src(count);
        for (int i = 0; i < count; ++i) {
            const amg_hier* h = hiers[i];
            if (!h) raise(AMG_EINVAL, "amg_batch_create: NULL hierarchy %d", i);
            if (h->lev.size() < 2) raise(AMG_EINVAL, "amg_batch_create: system %d has a single level", i);
            if (h->p.pre != 1 || h->p.post != 1) raise(AMG_EINVAL, "amg_batch_create: needs pre = post = 1");
            if (h->prec32 != hiers[0]->prec32 || h->p.omega != hiers[0]->p.omega ||
                h->p.true_res_period != hiers[0]->p.true_res_period)
                raise(AMG_EINVAL, "amg_batch_create: systems differ in precision, omega or true_res_period");
            for (size_t k = 0; k < h->lev.size(); ++k) {
                const Level& L = h->lev[k];
                SegLevelSrc t;
                t.n = L.n;
                t.nnz = L.nnz;
                t.rp = L.rp;
                t.ci = L.ci;
                t.v = L.v;
                t.v32 = L.v32;
                t.dinv = L.dinv;
                t.dinv32 = L.dinv32;
                t.mem = k + 1 < h->lev.size() ? L.mem : nullptr;
                src[i].lev.push_back(t);
            }
            src[i].ainv_t = h->ainv_t;
        }
        create_impl(src, hiers[0]->prec32, hiers[0]->p.omega, hiers[0]->p.true_res_period, al, as_stream(stream), out);
    });
}

amg_status amg_batch_setup(const amg_csr* A, int32_t count, const amg_params* params, const amg_allocator* alloc,
                           void* stream, amg_batch** out, amg_status* status) {
    if (out) *out = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    return guarded([&] {
        if (!A || !out || count < 1 || count > (1 << 20)) raise(AMG_EINVAL, "amg_batch_setup: bad arguments");
        const amg_allocator al = checked_allocator(alloc);
        amg_params p;
        amg_params_default(&p);
        if (params) p = *params;
        if (p.pre != 1 || p.post != 1) raise(AMG_EINVAL, "amg_batch_setup: needs pre = post = 1");
        hipStream_t caller = as_stream(stream);
        hipStream_t s = stream_get();
        hipEvent_t ev = event_get(false);
        DevPool P;
        P.s = s;
        P.al = al;
        struct Guard {
            DevPool& P;
            hipStream_t s;
            hipEvent_t ev;
            ~Guard() {
                (void)hipStreamSynchronize(s);
                P.release();
                (void)hipStreamSynchronize(s);
                event_put(ev, false);
                stream_put(s);
            }
        } guard{P, s, ev};
        HIPCHK(hipEventRecord(ev, caller));
        HIPCHK(hipStreamWaitEvent(s, ev, 0));
        std::vector<SegSrc> src;
        batch_coarsen(A, count, p, s, P, src);
        if (status)
            for (int i = 0; i < count; ++i) status[i] = src[i].status;
        create_impl(src, p.precond_fp32 != 0, p.omega, p.true_res_period, al, s, out);
        HIPCHK(hipEventRecord(ev, s));
        HIPCHK(hipStreamWaitEvent(caller, ev, 0));
        (*out)->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
}

amg_status amg_batch_rows(const amg_batch* b, int32_t* offsets) {
    return guarded([&] {
        if (!b || !offsets) raise(AMG_EINVAL, "amg_batch_rows: NULL argument");
        for (int i = 0; i < b->nseg; ++i) offsets[i] = b->seg[i].off0;
        offsets[b->nseg] = b->n0;
    });
}

amg_status amg_batch_solve(amg_batch* B, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                           void* stream, amg_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    amg_status st = AMG_OK;
    amg_status g = guarded([&] {
        if (!B || !b || !x || !info) raise(AMG_EINVAL, "amg_batch_solve: NULL argument");
        if (method != 0 && method != 1)
            raise(AMG_EINVAL, "amg_batch_solve: method must be 0 (PCG) or 1 (BiCGStab)");
        if (!(rtol >= 0.0) || maxit < 0) raise(AMG_EINVAL, "amg_batch_solve: rtol must be >= 0 and maxit >= 0");
        hipStream_t caller = as_stream(stream);
        hipStream_t s = B->stream;
        HIPCHK(hipEventRecord(B->ev[0], caller));
        HIPCHK(hipStreamWaitEvent(s, B->ev[0], 0));
        HIPCHK(hipMemcpyAsync(B->b, b, sizeof(double) * B->n0, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(B->x, x, sizeof(double) * B->n0, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemsetAsync(B->err, 0, sizeof(int), s));
        launch_check_finite(B->n0, B->b, B->x, B->err, s);
        HIPCHK(hipGetLastError());
        if (read_int(B->err, s) & ERR_NONFINITE) raise(AMG_ENOTFINITE, "amg_batch_solve: b or x0 has NaN or Inf");
        if (method == 0) batch_pcg(B, rtol, maxit, s, info);
        else batch_bicgstab(B, rtol, maxit, s, info);
        HIPCHK(hipMemcpyAsync(x, B->x, sizeof(double) * B->n0, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipEventRecord(B->ev[1], s));
        HIPCHK(hipStreamWaitEvent(caller, B->ev[1], 0));
        for (int i = 0; i < B->nseg; ++i)
            if (info[i].status != AMG_OK && st == AMG_OK) st = (amg_status)info[i].status;
        if (st == AMG_ENOTCONV) g_err = "amg_batch_solve: iteration limit reached for a system";
        if (st == AMG_EBREAKDOWN) g_err = "amg_batch_solve: breakdown for a system";
    });
    if (g != AMG_OK) {
        st = g;
        if (B && info)
            for (int i = 0; i < B->nseg; ++i) info[i].status = g;
    }
    if (B && info) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < B->nseg; ++i) {
            info[i].solve_ms = ms;
            info[i].setup_ms = B->setup_ms;
            info[i].levels = B->seg[i].nlev;
        }
    }
    return st;
}

amg_status amg_batch_autotune(amg_batch* b, void* stream, int32_t* schedule) {
    return guarded([&] {
        if (!b) raise(AMG_EINVAL, "amg_batch_autotune: NULL batch");
        batch_autotune(b, as_stream(stream), schedule);
    });
}

amg_status amg_batch_set_graphs(amg_batch* b, int32_t on) {
    return guarded([&] {
        if (!b) raise(AMG_EINVAL, "amg_batch_set_graphs: NULL batch");
        b->use_graphs = on != 0;
    });
}

amg_status amg_batch_levels(const amg_batch* b, int32_t* levels) {
    return guarded([&] {
        if (!b || !levels) raise(AMG_EINVAL, "amg_batch_levels: NULL argument");
        *levels = (int32_t)b->lev.size();
    });
}

amg_status amg_batch_destroy(amg_batch* b) {
    delete b;
    return AMG_OK;
}

}  // extern "C"
