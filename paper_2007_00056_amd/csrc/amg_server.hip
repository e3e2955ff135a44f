// Serving loop: independent solve requests run concurrently on one GPU.
//
// Requests are admitted in arrival order while the footprints of the
// requests in flight fit the budget; a request waits at the head of the
// queue until enough memory is released.
//
// Plain mode: each worker thread owns a HIP stream and runs whole requests
// (setup, Krylov solve, teardown) through the public entry points; kernels
// of different requests overlap on the device.
//
// Batched mode (batch >= 2): worker threads take the queued requests of one
// class (method, stop settings, small or large systems; up to `batch`,
// within the budget) and build their hierarchies together
// (amg_batch_setup).  The worker then advances its PCG group one iteration
// at a time on its own stream, so the groups of different workers overlap
// on the device and their launches come from several host threads, while
// idle workers form the next groups from whatever has arrived since.  A
// request is complete as soon as its own system leaves the iteration; the
// batch's memory, and the budget of its requests, is released when its last
// system is done.  BiCGStab groups are solved by their worker in one call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "amg_host.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    amg_csr A{};
    const double* b = nullptr;
    double* x = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the producer's stream at submission
    int32_t method = 0;
    double rtol = 0.0;
    int32_t maxit = 0;
    uint64_t foot = 0;
    Clock::time_point t_submit;
    Clock::time_point t_done;
    bool done = false;
    amg_status st = AMG_OK;
    amg_info info{};
};

constexpr int32_t kSmallRows = 32768;  // systems matched in one workgroup by a batched setup

uint64_t footprint(int32_t n, int64_t nnz, const amg_params& p) {
    const uint64_t N = (uint64_t)(n > 0 ? n : 0), Z = (uint64_t)(nnz > 0 ? nnz : 0);
    const uint64_t e = p.precond_fp32 ? 4 : 8;
    // coarsest inverse: at most max(max_coarse_rows, max_dense_rows) rows, and
    // never more than the system has
    uint64_t m = (uint64_t)(p.max_coarse_rows > p.max_dense_rows ? p.max_coarse_rows : p.max_dense_rows);
    if (m > N) m = N;
    const uint64_t dense = 8 * m * m + 4096;
    // persistent: level-0 D^{-1}; coarse CSR (row pointers sized by the finer
    // level), D^{-1}, maps and member lists over <= N rows and <= Z entries;
    // V-cycle vectors; float copies; Krylov vectors; reduction partials
    uint64_t b = 8 * N + (8 * N + 12 * Z + 8 * N + 8 * N + 16 * N) + dense;
    b += 5 * e * 2 * N + e * N;
    if (p.precond_fp32) b += 4 * 2 * Z + 4 * 2 * N;
    b += 10 * 8 * N + (1u << 20);
    // setup scratch at its peak: matching records and state, numbering,
    // Galerkin counts, the intermediate operator of a two-pass level, the
    // dense factorisation
    b += 256 * N + Z + 60 * N + (4 * N + 12 * Z) + dense;
    if (p.hem == 1) b += 8 * Z + 4 * N;            // symmetric weights, pointers
    if (p.alternate) b += 4 * N + 12 * Z + 4096;  // mirrored matrix of a pass from the last index
    return b;
}

// What a request adds inside a batch: its concatenated levels (level 0
// included), vectors and Krylov workspace, and its slices of the batch's
// right-hand side and solution.
uint64_t batch_extra(int32_t n, int64_t nnz, const amg_params& p) {
    const uint64_t N = (uint64_t)(n > 0 ? n : 0), Z = (uint64_t)(nnz > 0 ? nnz : 0);
    uint64_t m = (uint64_t)(p.max_coarse_rows > p.max_dense_rows ? p.max_coarse_rows : p.max_dense_rows);
    if (m > N) m = N;
    // also the batched setup's concatenated levels and its coarsest blocks
    // (matrix, factors and inverse)
    return 60 * Z + 256 * N + 16 * m * m + 8 * m + 4096;
}

}  // namespace

struct amg_server {
    amg_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request*> reqs;
    int64_t next_id = 1;
    uint64_t in_use = 0;
    int active = 0;
    bool stopping = false;
    std::vector<std::thread> threads;
    std::vector<hipStream_t> wstreams;  // one per worker, destroyed with the server

    // A set-up PCG group being solved by its worker.
    struct Flight {
        amg_batch* bt = nullptr;
        std::vector<Request*> grp;     // nullptr once the request is complete
        std::vector<uint64_t> feet;    // budget released with the batch
        std::vector<char> batched;     // system i is solved in the batch
        amg::PcgRun* run = nullptr;
        Clock::time_point t0;
    };

    void release_streams() {
        for (hipStream_t& st : wstreams)
            if (st) {
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
                st = nullptr;
            }
    }

    bool batched() const { return cfg.batch >= 2; }
    const amg_allocator* alloc() const { return cfg.alloc.alloc ? &cfg.alloc : nullptr; }

    // Workers drain the queue, finish their groups and exit.
    void stop_threads() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stopping = true;
        }
        cv_work.notify_all();
        for (auto& t : threads) t.join();
        threads.clear();
    }

    // The request's result is final: its waiter may proceed (and free it).
    void complete(Request* r) {
        {
            std::lock_guard<std::mutex> lk(mu);
            r->done = true;
            r->t_done = Clock::now();
        }
        cv_done.notify_all();
    }

    // Its memory is released: admission may take the next requests.
    void release(uint64_t foot) {
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= foot;
            --active;
        }
        cv_work.notify_all();
    }

    void finish(Request* r) {
        const uint64_t f = r->foot;
        complete(r);
        release(f);
    }

    // Once a setup is done, the memory its requests hold is known.  Their
    // admission estimates assume the worst (the largest coarsest block the
    // parameters allow, every setup buffer at its peak), while the coarsest
    // level normally has at most max_coarse_rows rows and the setup's scratch
    // is gone: the shares are cut to the `held` bytes, split in proportion to
    // the estimates, and admission may take further requests.  A share never
    // grows.
    void settle(const std::vector<uint64_t*>& feet, uint64_t held) {
        uint64_t sum = 0;
        for (const uint64_t* f : feet) sum += *f;
        if (feet.empty() || held >= sum) return;
        uint64_t cut = 0;
        {
            std::lock_guard<std::mutex> lk(mu);
            uint64_t left = held;
            for (size_t i = 0; i < feet.size(); ++i) {
                uint64_t f = i + 1 < feet.size() ? (uint64_t)((long double)*feet[i] * held / sum) : left;
                if (f > *feet[i]) f = *feet[i];
                cut += *feet[i] - f;
                left -= f;
                *feet[i] = f;
            }
            in_use -= cut;
        }
        if (cut) cv_work.notify_all();
    }

    // Requests that a group headed by h may hold: the same Krylov method (PCG
    // or BiCGStab) and stop settings, and the same size class (systems that
    // fit one workgroup's matching state are grouped apart from larger ones:
    // a group of small systems then needs no round kernels at all).
    static bool groups_with(const Request* h, const Request* r) {
        return (r->A.n <= kSmallRows) == (h->A.n <= kSmallRows) && r->method == h->method && r->rtol == h->rtol &&
               r->maxit == h->maxit;
    }

    // Budget the group a worker would take now needs: the head's footprint
    // and, in batched mode, those of the queued requests it groups with, up
    // to `batch` of them.  Called with mu held.
    uint64_t group_need() {
        const Request* h = reqs[pending.front()];
        uint64_t need = h->foot;
        if (!(batched() && h->method <= 1)) return need;
        int k = 1;
        for (auto it = pending.begin() + 1; it != pending.end() && k < cfg.batch; ++it) {
            const Request* r = reqs[*it];
            if (groups_with(h, r)) {
                need += r->foot;
                ++k;
            }
        }
        return need;
    }

    // Worker i runs on wstreams[i].  It takes the request at the head of the
    // queue, and in batched mode the queued requests that group with it, up to
    // `batch`, once that whole group fits the budget (or nothing else is in
    // flight): budget freed a little at a time would otherwise be taken by
    // ever smaller groups, whose iterations cost nearly as much as full ones.
    void worker(int i) {
        if (hipSetDevice(device) != hipSuccess) return;
        hipStream_t s = wstreams[i];
        for (;;) {
            std::vector<Request*> grp;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (pending.empty()) return stopping;
                    return active == 0 || in_use + group_need() <= cfg.hbm_budget_bytes;
                });
                if (pending.empty()) break;  // stopping and drained
                Request* head = reqs[pending.front()];
                pending.pop_front();
                grp.push_back(head);
                in_use += head->foot;
                ++active;
                if (batched() && head->method <= 1) {
                    for (auto it = pending.begin(); it != pending.end() && (int)grp.size() < cfg.batch;) {
                        Request* r = reqs[*it];
                        if (groups_with(head, r) && in_use + r->foot <= cfg.hbm_budget_bytes) {
                            grp.push_back(r);
                            in_use += r->foot;
                            ++active;
                            it = pending.erase(it);
                        } else {
                            ++it;
                        }
                    }
                }
            }
            // the worker reads b and x only after the producers' writes
            for (Request* r : grp)
                if (r->ready) {
                    (void)hipStreamWaitEvent(s, r->ready, 0);
                    amg::event_put(r->ready, false);
                    r->ready = nullptr;
                }
            if (!(batched() && grp[0]->method <= 1)) {
                run_one(grp[0], s);
                finish(grp[0]);
            } else if (grp[0]->method == 0) {
                pcg_group(grp, s);
            } else {
                run_group(grp, s);
                for (Request* r : grp) finish(r);
            }
        }
    }

    // Setup, solve and teardown of one request.
    void run_one(Request* r, hipStream_t s) {
        if (!s) {
            r->st = AMG_EHIP;
            r->info.status = AMG_EHIP;
            return;
        }
        amg_hier* h = nullptr;
        amg_status st = amg_setup(&r->A, &cfg.params, alloc(), s, &h);
        // no graph capture on a worker: it would make device-wide calls of the
        // other workers and of the caller's threads fail while it lasts
        if (h) h->use_graphs = false;
        if (st == AMG_OK) {
            // held: the hierarchy, the Krylov vectors still to come and the
            // reduction partials
            const uint64_t n0 = (uint64_t)h->lev[0].n;
            settle({&r->foot}, (uint64_t)h->pool.bytes + (h->r ? 0 : 10 * 8 * n0) + (1u << 20));
        }
        if (st == AMG_OK) st = krylov_solve(h, r->method, r->b, r->x, r->rtol, r->maxit, s, &r->info);
        else r->info.status = st;
        if (h) (void)amg_destroy(h);
        r->st = st;
    }

    static void fail(Request* r, amg_status st) {
        r->st = st;
        r->info.status = st;
    }

    // A PCG group: batched setup on the worker's stream, the systems' right-
    // hand sides and initial guesses loaded into the batch, then the solve,
    // one iteration at a time.  When the batched setup fails as a whole, or a
    // system cannot be batched (a single level), the requests concerned are
    // run one by one here.
    void pcg_group(std::vector<Request*>& grp, hipStream_t s) {
        const int n = (int)grp.size();
        std::vector<amg_csr> A(n);
        for (int i = 0; i < n; ++i) A[i] = grp[i]->A;
        std::vector<amg_status> st(n, AMG_OK);
        amg_batch* bt = nullptr;
        if (!s || amg_batch_setup(A.data(), n, &cfg.params, alloc(), s, &bt, st.data()) != AMG_OK) {
            for (Request* r : grp) {
                run_one(r, s);
                finish(r);
            }
            return;
        }
        (void)amg_batch_set_graphs(bt, 0);
        std::unique_ptr<Flight> F(new Flight());
        F->bt = bt;
        F->grp = grp;
        F->batched.assign(n, 1);
        for (Request* r : grp) F->feet.push_back(r->foot);
        std::vector<int32_t> off(n + 1);
        (void)amg_batch_rows(bt, off.data());
        std::vector<Request*> alone;
        const amg_status lst = amg::guarded([&] {
            for (int i = 0; i < n; ++i) {
                if (st[i] == AMG_EINVAL && off[i + 1] == off[i]) {  // invalid or a single level: the plain path
                    F->batched[i] = 0;
                    continue;
                }
                if (off[i + 1] > off[i]) amg::batch_load(bt, i, grp[i]->b, grp[i]->x, i == 0 ? s : nullptr);
            }
        });
        if (lst != AMG_OK) {
            (void)amg_batch_destroy(bt);
            for (Request* r : grp) {
                fail(r, lst);
                finish(r);
            }
            return;
        }
        F->feet.clear();
        for (int i = 0; i < n; ++i) {
            if (!F->batched[i]) {
                alone.push_back(grp[i]);
                F->grp[i] = nullptr;
            } else {
                F->feet.push_back(grp[i]->foot);
            }
        }
        {
            std::vector<uint64_t*> fp;
            for (uint64_t& f : F->feet) fp.push_back(&f);
            settle(fp, (uint64_t)amg::batch_bytes(bt) + (1u << 20));
        }
        for (Request* r : alone) {
            run_one(r, s);
            finish(r);
        }
        solve_flight(*F);
    }

    // BiCGStab groups: one batched setup and one batched solve.  When the
    // batched setup fails as a whole, or a system cannot be batched (a single
    // level), the requests concerned are run one by one.
    void run_group(std::vector<Request*>& grp, hipStream_t s) {
        const int n = (int)grp.size();
        if (!s) {
            for (Request* r : grp) fail(r, AMG_EHIP);
            return;
        }
        std::vector<amg_csr> A(n);
        for (int i = 0; i < n; ++i) A[i] = grp[i]->A;
        std::vector<amg_status> st(n, AMG_OK);
        amg_batch* bt = nullptr;
        if (amg_batch_setup(A.data(), n, &cfg.params, alloc(), s, &bt, st.data()) != AMG_OK) {
            for (Request* r : grp) run_one(r, s);
            return;
        }
        // no graph capture on a worker: it would make device-wide calls of the
        // other workers and of the caller's threads fail while it lasts
        (void)amg_batch_set_graphs(bt, 0);
        std::vector<int32_t> off(n + 1);
        (void)amg_batch_rows(bt, off.data());
        {
            // held: the batch, BiCGStab's vectors still to come and the
            // group's right-hand sides and solutions below
            std::vector<uint64_t*> fp;
            for (int i = 0; i < n; ++i)
                if (!(st[i] == AMG_EINVAL && off[i + 1] == off[i])) fp.push_back(&grp[i]->foot);
            settle(fp, (uint64_t)amg::batch_bytes(bt) + 7 * 8 * (uint64_t)off[n] + (1u << 20));
        }
        // right-hand sides and solutions of the group, drawn like every other
        // buffer of a request (so the allocator accounts for them) and released
        // with the group
        amg::DevPool io;
        io.s = s;
        io.al = cfg.alloc.alloc ? cfg.alloc : amg_allocator{};
        struct IoGuard {
            amg::DevPool& p;
            hipStream_t s;
            ~IoGuard() {
                (void)hipStreamSynchronize(s);
                p.release();
            }
        } iog{io, s};
        double* B = nullptr;
        try {
            B = io.get<double>(2 * (size_t)(off[n] > 0 ? off[n] : 1));
        } catch (const amg::Failure&) {
            (void)amg_batch_destroy(bt);
            for (Request* r : grp) fail(r, AMG_ENOMEM);
            return;
        }
        double* X = B + off[n];
        bool ok = true;
        for (int i = 0; i < n; ++i) {
            const size_t bytes = sizeof(double) * (size_t)(off[i + 1] - off[i]);
            if (bytes == 0) continue;
            ok &= hipMemcpyAsync(B + off[i], grp[i]->b, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess;
            ok &= hipMemcpyAsync(X + off[i], grp[i]->x, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess;
        }
        std::vector<amg_info> info(n);
        if (ok) (void)amg_batch_solve(bt, grp[0]->method, B, X, grp[0]->rtol, grp[0]->maxit, s, info.data());
        for (int i = 0; i < n && ok; ++i) {
            const size_t bytes = sizeof(double) * (size_t)(off[i + 1] - off[i]);
            if (bytes == 0) continue;
            ok &= hipMemcpyAsync(grp[i]->x, X + off[i], bytes, hipMemcpyDeviceToDevice, s) == hipSuccess;
        }
        ok &= hipStreamSynchronize(s) == hipSuccess;
        (void)amg_batch_destroy(bt);
        for (int i = 0; i < n; ++i) {
            if (!ok) {
                fail(grp[i], AMG_EHIP);
            } else if (st[i] == AMG_EINVAL && off[i + 1] == off[i]) {
                run_one(grp[i], s);  // invalid or a single level: the plain path decides
            } else {
                grp[i]->info = info[i];
                grp[i]->st = (amg_status)info[i].status;
            }
        }
    }

    // System i of flight F is done: its iterate goes to the request's x (on
    // the batch's stream, waited for), and the request completes.
    void deliver(Flight& F, int i, amg_status err = AMG_OK) {
        Request* r = F.grp[i];
        if (!r) return;
        F.grp[i] = nullptr;
        if (err != AMG_OK) {
            fail(r, err);
        } else {
            r->info = amg::pcg_run_info(F.run, i);
            amg::batch_fill_info(F.bt, i, r->info);
            r->st = (amg_status)r->info.status;
            int n = 0;
            const double* xs = amg::batch_x(F.bt, i, &n);
            hipStream_t bs = amg::batch_stream(F.bt);
            if (n > 0 && (hipMemcpyAsync(r->x, xs, sizeof(double) * n, hipMemcpyDeviceToDevice, bs) != hipSuccess ||
                          hipStreamSynchronize(bs) != hipSuccess))
                fail(r, AMG_EHIP);
        }
        r->info.solve_ms = std::chrono::duration<double, std::milli>(Clock::now() - F.t0).count();
        complete(r);
    }

    // The last system of F is done: the batch and the budget go.
    void retire(Flight& F) {
        for (size_t i = 0; i < F.grp.size(); ++i) deliver(F, (int)i, AMG_EHIP);  // none left normally
        if (F.run) amg::pcg_run_end(F.run);
        F.run = nullptr;
        (void)amg_batch_destroy(F.bt);
        F.bt = nullptr;
        for (uint64_t f : F.feet) release(f);
    }

    // The batched PCG of flight F, one iteration at a time: each system is
    // delivered as soon as it leaves the iteration; the batch goes with the
    // last one.
    void solve_flight(Flight& F) {
        F.t0 = Clock::now();
        std::vector<int> done;
        const Request* r0 = nullptr;
        for (Request* r : F.grp)
            if (r) {
                r0 = r;
                break;
            }
        if (!r0) {
            retire(F);
            return;
        }
        amg_status st = amg::guarded([&] { F.run = amg::pcg_run_start(F.bt, r0->rtol, r0->maxit, done); });
        for (int i : done) deliver(F, i);
        while (st == AMG_OK && F.run && amg::pcg_run_live(F.run) > 0) {
            done.clear();
            st = amg::guarded([&] {
                amg::pcg_run_enqueue(F.run);
                amg::pcg_run_collect(F.run, done);
            });
            for (int i : done) deliver(F, i);
        }
        if (st != AMG_OK)
            for (size_t i = 0; i < F.grp.size(); ++i) deliver(F, (int)i, st);
        retire(F);
    }
};

extern "C" {

amg_status amg_footprint_bytes(int32_t n, int64_t nnz, const amg_params* params, uint64_t* bytes) {
    if (!bytes || n < 0 || nnz < 0) return AMG_EINVAL;
    amg_params p;
    if (params) p = *params;
    else amg_params_default(&p);
    *bytes = footprint(n, nnz, p);
    return AMG_OK;
}

amg_status amg_server_config_default(amg_server_config* c) {
    if (!c) return AMG_EINVAL;
    c->workers = 4;
    c->batch = 0;
    c->hbm_budget_bytes = 64ull << 30;
    c->alloc = amg_allocator{};
    return amg_params_default(&c->params);
}

amg_status amg_server_create(const amg_server_config* c, amg_server** out) {
    if (out) *out = nullptr;
    if (!out) return AMG_EINVAL;
    amg_server_config cfg;
    if (c) cfg = *c;
    else amg_server_config_default(&cfg);
    if (cfg.workers < 1 || cfg.workers > 64 || cfg.hbm_budget_bytes == 0 || cfg.batch < 0) return AMG_EINVAL;
    if (!cfg.alloc.alloc != !cfg.alloc.free) return AMG_EINVAL;
    if (cfg.batch >= 2 && (cfg.params.pre != 1 || cfg.params.post != 1)) return AMG_EINVAL;
    amg_server* s = new (std::nothrow) amg_server();
    if (!s) return AMG_ENOMEM;
    s->cfg = cfg;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return AMG_EHIP;
    }
    try {
        s->wstreams.assign(cfg.workers, nullptr);
        for (int i = 0; i < cfg.workers; ++i)
            if (hipStreamCreateWithFlags(&s->wstreams[i], hipStreamNonBlocking) != hipSuccess) {
                s->release_streams();
                delete s;
                return AMG_EHIP;
            }
        for (int i = 0; i < cfg.workers; ++i) s->threads.emplace_back([s, i] { s->worker(i); });
    } catch (...) {
        s->stop_threads();
        s->release_streams();
        delete s;
        return AMG_ENOMEM;
    }
    *out = s;
    return AMG_OK;
}

amg_status amg_server_submit(amg_server* s, const amg_csr* A, const double* b, double* x, int32_t method,
                             double rtol, int32_t maxit, void* stream, int64_t* ticket) {
    if (!s || !A || !b || !x || !ticket) return AMG_EINVAL;
    Request* r = new (std::nothrow) Request();
    if (!r) return AMG_ENOMEM;
    r->A = *A;
    r->b = b;
    r->x = x;
    r->method = method;
    r->rtol = rtol;
    r->maxit = maxit;
    r->foot = footprint(A->n, A->nnz, s->cfg.params) + (s->batched() ? batch_extra(A->n, A->nnz, s->cfg.params) : 0);
    if (r->foot > s->cfg.hbm_budget_bytes) {
        delete r;
        return AMG_EINVAL;
    }
    // the request's inputs are ready once the work the producer enqueued on
    // `stream` so far has finished
    const amg_status est = amg::guarded([&] {
        using amg::raise;
        r->ready = amg::event_get(false);
        HIPCHK(hipEventRecord(r->ready, static_cast<hipStream_t>(stream)));
    });
    if (est != AMG_OK) {
        if (r->ready) amg::event_put(r->ready, false);
        delete r;
        return est;
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            amg::event_put(r->ready, false);
            delete r;
            return AMG_EINVAL;
        }
        const int64_t id = s->next_id++;
        s->reqs[id] = r;
        s->pending.push_back(id);
        *ticket = id;
    }
    s->cv_work.notify_one();
    return AMG_OK;
}

amg_status amg_server_wait(amg_server* s, int64_t ticket, amg_info* info, double* latency_ms) {
    if (!s) return AMG_EINVAL;
    Request* r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return AMG_EINVAL;
        r = it->second;
        s->cv_done.wait(lk, [&] { return r->done; });
        s->reqs.erase(ticket);  // the map may have changed while waiting
    }
    if (info) *info = r->info;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    const amg_status st = r->st;
    delete r;
    return st;
}

amg_status amg_server_destroy(amg_server* s) {
    if (!s) return AMG_OK;
    s->stop_threads();
    s->release_streams();
    for (auto& kv : s->reqs) {
        if (kv.second->ready) amg::event_put(kv.second->ready, false);
        delete kv.second;
    }
    delete s;
    return AMG_OK;
}

}  // extern "C"
