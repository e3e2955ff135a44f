// Internal interfaces between the host orchestration (amg_api.hip) and the
// kernel launchers (k_setup.hip, k_solve.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amg {

// Device error bits raised by validation and setup kernels.
enum : int {
    ERR_STRUCT = 1,      // bad row_ptr / column index / column order
    ERR_NONFINITE = 2,   // NaN or Inf value
    ERR_DIAG = 4,        // missing or zero diagonal
    ERR_NONSYM = 8,      // pattern not structurally symmetric
    ERR_SINGULAR = 16,   // dense coarsest LU met a zero pivot
};

constexpr int kUndecided = 0x3fffffff;  // round stamp of an undecided vertex
constexpr int kDenseMaxRows = 4096;     // largest coarsest level (dense LU, explicit inverse)

// Lanes per CSR row used by the level kernels (a power of two, 1..16).
int pick_lanes_per_row(double avg_row_len);

// ---- setup kernels (k_setup.hip) ------------------------------------------
void launch_validate(int n, int64_t nnz, const int* rp, const int* ci, const double* v, double* dinv, int* err,
                     hipStream_t s);
void launch_dinv(int n, const int* rp, const int* ci, const double* v, double* dinv, int* err, hipStream_t s);

// Per-vertex adjacency record of a matching pass (64, 128 or 256 bytes for
// SIDE = 7, 15, 31): the first SIDE higher neighbours j (a_uj non-zero) by
// |a_uj| descending, column ascending on ties, and the first SIDE lower
// edge-neighbours x (row x stores a non-zero a_xu) ascending.  kRecHiTrunc /
// kRecLoTrunc: the row has more of them (the first undecided entry of a list
// is still the vertex's choice when the list has one; otherwise the CSR row
// decides); kRecOverflow: either.
constexpr int kRecOverflow = 1 << 16;
constexpr int kRecHiTrunc = 1 << 17;
constexpr int kRecLoTrunc = 1 << 18;
constexpr int kHemLdsRows = 32768;  // passes up to this size keep their matching state in LDS
constexpr int kHemTileRows = 32768;  // largest tile of a tiled pass (its state in LDS)
constexpr int kHemMaxTiles = 4096;   // tiled passes up to this many tiles
constexpr int kHemTileCRows = 4096;  // largest tile whose records are kept in LDS
template <int SIDE>
struct alignas(4 * (SIDE + 1) * 2) HemRecT {
    int hdr;  // #higher | #lower << 8 | kRecOverflow | kRecHiTrunc | kRecLoTrunc
    int h[SIDE];
    int l[SIDE];
    int pad;
};
static_assert(sizeof(HemRecT<7>) == 64 && sizeof(HemRecT<15>) == 128 && sizeof(HemRecT<31>) == 256, "record");

struct HemWork {
    uint8_t* lowok;   // [nnz] entry (v,u), u < v, is an edge (row u stores a non-zero a_uv)
    void* rec;        // adjacency records, rec_bytes of room
    size_t rec_bytes;
    int side;         // record side of the current pass: 7, 15 or 31
    int* lcnt;        // [n] undecided lower neighbours
    int* dec;         // [n] round in which the vertex was decided
    int* mate;        // [n] partner or -1
    int* wl[2];       // [n] ready worklists (ping-pong)
    int* cnt;         // [8] worklist size ring, symmetry check, round count, guard
    int* err;
    int round_grid = 96;  // blocks of a one-launch-per-round pass
    int tile_rows = kHemTileRows;  // rows per tile of a tiled pass (0: no tiled passes)
    int tile_c_rows = kHemTileCRows;  // rows per LDS-record tile (0: not used; below kHemTileCRows: every
                                      // side-7 pass takes them, for tests)
    int lds_rows = kHemLdsRows;  // one-workgroup passes up to this size keep their state in LDS
    double* wsym = nullptr;  // edge-based matching: [nnz] heavier of |a_uv|, |a_vu| (0 on the diagonal)
    int* ptr = nullptr;      // edge-based matching: [n] best undecided neighbour
};
// w.cnt must be zeroed before the call.
void launch_hem_init(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s);
void launch_hem_round(int round, int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s);
// All rounds in one single-workgroup launch (small n).
void launch_hem_all(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s);
// Tiled pass: one workgroup per w.tile_rows rows, all rounds in one launch
// (after launch_hem_init and, for block-diagonal operators, launch_hem_lds_seg;
// w.side 7 or 15).
// cnt[7] != 0 afterwards: the pass did not finish within tmo wall-clock ticks
// (or a counter exceeded 16 bits) and must be repeated with the round kernels.
void launch_hem_tile(int n, int64_t nnz, const int* rp, const int* ci, const double* v, HemWork& w, long long tmo,
                     hipStream_t s);
// Block-diagonal operators: seg[j] = (first row, rows) of system j; systems of
// at most kHemLdsRows rows are matched one workgroup each and marked decided
// (stamp -1) for the round kernels.  sl0/sl1: global list space, n rows each.
void launch_hem_lds_seg(int nseg, const int2* seg, const int* rp, const int* ci, const double* v, HemWork& w,
                        int* sl0, int* sl1, hipStream_t s);
// seg[j] for the operator of the next pass: system j starts at agg[off[j]]
// (n rows in all; mirror numbers the operator backwards).
void launch_seg_table(int m, const int* off, const int* agg, int n, bool mirror, int2* seg, hipStream_t s);
// Edge-based matching (Algorithm 3): initialisation (every vertex dirty, the
// count in cnt[0]; w.lcnt serves as the per-round marks) and one round (two
// launches).  w.cnt must be zeroed before the initialisation.
void launch_ehem_init(int n, const int* rp, const int* ci, const double* v, HemWork& w, hipStream_t s);
void launch_ehem_round(int r, int n, const int* rp, const int* ci, HemWork& w, hipStream_t s);
int hem_next_count_slot(int round);  // counter slot that holds |worklist| before `round`

// Exclusive prefix sum: out[i] = sum in[0..i), out[n] = total.  tmp: scan_tmp_ints(n).
size_t scan_tmp_ints(int n);
// out[0..7] = cnt[0..7], out[8] = *ncp, out[9] = *nnzc, out[10] = *err (out: a
// device address of mapped host memory).
void launch_pass_words(int* out, const int* cnt, const int* ncp, const int* nnzc, const int* err, hipStream_t s);
void launch_scan(const int* in, int n, int* out, int* tmp, hipStream_t s);
void launch_leader_flags(int n, const int* mate, int* flag, hipStream_t s);
// agg[v] = id of v's aggregate; lead[id] = smaller vertex of the aggregate.
void launch_assign_ids(int n, const int* mate, const int* ids, int* agg, int* lead, hipStream_t s);

// Galerkin product of one matching pass (aggregates of size <= 2).
void launch_rap_count(int nmax, const int* ncp, const int* lead, const int* mate, const int* rp, const int* ci,
                      const int* agg, int* rowcnt, int* ovf, int* novf, hipStream_t s);
void launch_rap_count_slow(int nc, const int* ovf, const int* novf, const int* lead, const int* mate, const int* rp,
                           const int* ci, const int* agg, int* rowcnt, hipStream_t s);
void launch_rap_fill(int nc, const int* lead, const int* mate, const int* rp, const int* ci, const double* v,
                     const int* agg, const int* crp, int* cci, double* cv, hipStream_t s);
void launch_rap_fill_slow(int nc, const int* ovf, const int* novf, const int* lead, const int* mate, const int* rp,
                          const int* ci, const double* v, const int* agg, const int* crp, int* cci, double* cv,
                          hipStream_t s);

// Matching from the last index: the mirrored matrix (i -> n-1-i) and the map of
// its pairs back to the original numbering.
void launch_mirror_csr(int n, int64_t nnz, const int* rp, const int* ci, const double* v, int* mrp, int* mci,
                       double* mv, hipStream_t s);
void launch_unmirror_mate(int n, const int* mr, int* mate, hipStream_t s);

void launch_compose(int n, const int* agg1, const int* agg2, int* out, hipStream_t s);
// Member lists (ascending fine rows, -1 padded) of the level's coarse rows.
void launch_members(int nc, const int* lead2, const int* mate2, const int* lead1, const int* mate1, int4* mem,
                    hipStream_t s);

// a must be zeroed before the call.  col_add shifts the stored columns (a
// diagonal block of a larger matrix); entries outside the block are skipped.
void launch_dense_assemble(int n, const int* rp, const int* ci, const double* v, double* a, hipStream_t s,
                           int col_add = 0);
// Systems stored one after another in a level: out[2j] = agg[off[j]],
// out[2j+1] = crp[out[2j]] (coarse row and entry where system j starts).
void launch_seg_starts(int m, const int* off, const int* agg, const int* crp, int* out, hipStream_t s);
// piv: int32[2n] scratch.  n <= kDenseMaxRows.
void launch_dense_lu_inverse(int n, double* a, int* piv, double* ainv_t, int* err, hipStream_t s);

// ---- solve kernels (k_solve.hip) --------------------------------------------
struct LevelView {
    int n;
    int nnz;
    const int* rp;
    const int* ci;
    const double* v;
    const double* dinv;
    const int* agg;   // [n] aggregate on level k+1
    const int4* mem;  // [n_{k+1}] members of coarse rows (for k < L)
    int lpr;          // lanes per row
};

struct Reducer {
    double* part;     // [2 * kRedBlocks] per-block partial sums
    double* S;        // scalar slots
};

// A coarse level's finished value zc of row i becomes the finer level's
// prolongated iterate on i's members m: xpf[m] = w gf[m] + zc.
template <class T>
struct ScatterT {
    const int4* __restrict__ mem;
    const T* __restrict__ gf;
    T* __restrict__ xpf;
    T w;
    __device__ __forceinline__ void operator()(int i, T zc) const {
        const int4 m = mem[i];
        xpf[m.x] = w * gf[m.x] + zc;
        if (m.y >= 0) xpf[m.y] = w * gf[m.y] + zc;
        if (m.z >= 0) xpf[m.z] = w * gf[m.z] + zc;
        if (m.w >= 0) xpf[m.w] = w * gf[m.w] + zc;
    }
};

// V-cycle view of a level with values of type T (double, or the float copy).
template <class T>
struct VLevel {
    int n;
    const int* rp;
    const int* ci;
    const T* v;
    const T* dinv;
    const int4* mem;  // members of level k+1 rows
    int lpr;
    int rb = 256;     // rows per block of the CSR-stream kernels: 128, 256 or 512
};

// ---- V-cycle kernels (k_vcycle.hip), T = double or float -------------------
// Every level keeps g = D^{-1} f next to its right-hand side f; the kernel
// that produces f also writes g.  Large levels (CSR-stream): r = f - w A g,
// then f_c = P^T r and g_c; postsmoothing from the prolongated iterate xp:
// z = xp + w (g - D^{-1} A xp), with (f, z) reduced into `slot` when R is
// given and z scattered into the finer level's xp when sc is given.
template <class T, class TIN>
void vc_stream_resid(const VLevel<T>& L, const TIN* f, const T* g, T w, T* r, hipStream_t s);
template <class T>
void vc_restrict(int nc, const int4* mem, const T* r, const T* dinv_c, T* fc, T* gc, hipStream_t s);
// slot == kPartialsOnly: the (f, z) partials stay in R->part (at most
// kFusedParts blocks) for a consumer kernel to add; returns their number (0
// when no partials are left).
template <class T, class TOUT>
int vc_stream_post(const VLevel<T>& L, const T* xp, const T* g, T w, TOUT* z, const double* f, const Reducer* R,
                   int slot, const ScatterT<T>* sc, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);  // t0/t1: recorded at the start/end of the main kernel
// Small levels: the same operations with the restriction fused.
template <class T, class TIN>
void vc_resid_restrict(const VLevel<T>& L, int nc, const TIN* f, const T* g, T w, const T* dinv_c, T* fc, T* gc,
                       hipStream_t s);
template <class T, class TOUT>
void vc_prolong_post(const VLevel<T>& L, const T* xp, const T* g, T w, TOUT* z, const ScatterT<T>* sc,
                     hipStream_t s);
// g = D^{-1} f (computed in double, stored as T)
template <class T>
void vc_scale_dinv(int n, const double* dinv, const double* f, T* g, hipStream_t s);
// Coarsest level x = A_L^{-1} f in double (explicit inverse, column-major).
template <class T, class TIN, class TOUT>
void vc_dense_apply(int n, const double* ainv_t, const TIN* f, TOUT* x, const ScatterT<T>* sc, hipStream_t s);

// S[slot0] (and S[slot1] when nv = 2) = fixed-order sums of the partials.
void launch_cast_f32(int64_t n, const double* a, float* b, hipStream_t s);
void launch_finish(int nparts, int nv, const Reducer& R, int slot0, int slot1, hipStream_t s);

void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t s);
// General smoothing path.
void launch_jacobi_zero(int n, const double* dinv, const double* f, double w, double* x, hipStream_t s);
void launch_jacobi(const LevelView& L, const double* f, const double* x, double w, double* xo, hipStream_t s);
void launch_resid_restrict_x(const LevelView& L, int nc, const double* f, const double* x, double* fc,
                             hipStream_t s);
void launch_prolong_add(int n, const int* agg, const double* e, double* x, hipStream_t s);

// Krylov vector kernels.  Slots index Reducer::S.
// r = b - A x, (r, r); gout (may be null) receives D^{-1} r, as float when g32.
void launch_residual(const LevelView& A, const double* b, const double* x, double* r, void* gout, bool g32,
                     const Reducer& R, int slot_rr, hipStream_t s);
void launch_dot(int n, const double* a, const double* b, const Reducer& R, int slot, hipStream_t s);
void launch_spmv_dot(const LevelView& A, const double* p, double* q, const double* d, const Reducer& R, int slot,
                     hipStream_t s);
// q = A p with the block partials of (d, q) left in part (at most
// kFusedParts blocks); returns their number.
int launch_spmv_dot_parts(const LevelView& A, const double* p, double* q, const double* d, double* part,
                          hipStream_t s);
void launch_spmv_dot2(const LevelView& A, const double* p, double* t, const double* sv, const Reducer& R, int slot_tt,
                      int slot_ts, hipStream_t s);
// pq_part (non-null): the update adds the pq_np partials of (p, q) itself
// (block 0 stores the sum in slot_pq) and leaves the partials of (r, r) in
// rr_part (at most kFusedParts blocks; *rr_np receives their number) instead
// of finishing them into slot_rr.
void launch_cg_update(int n, double* x, double* r, const double* p, const double* q, const double* dinv, void* gout,
                      bool g32, const Reducer& R, int slot_rho, int slot_pq, int slot_rr, hipStream_t s,
                      const double* pq_part = nullptr, int pq_np = 0, double* rr_part = nullptr, int* rr_np = nullptr);
// Sh/nsh: optional host memory mapped into the device that receives the
// first nsh scalar slots (nsh <= 256).  new_part (non-null): the kernel adds
// the new_np partials of the new (r, z) itself (block 0 stores the sum in
// slot_new).  rr_part (non-null): block 0 adds the rr_np partials of (r, r)
// into slot_rr.  hseq (non-null, with Sh): after the slots, the word hseq
// (mapped host memory too) receives seq, so the host can wait for the slots
// by watching that word.
void launch_cg_dir(int n, const double* z, const double* p, double* pn, double* S, int slot_new, int slot_old,
                   hipStream_t s, double* Sh = nullptr, int nsh = 0, const double* new_part = nullptr, int new_np = 0,
                   const double* rr_part = nullptr, int rr_np = 0, int slot_rr = 0, unsigned long long* hseq = nullptr,
                   unsigned long long seq = 0);
void launch_bicg_s(int n, const double* r, const double* v, double* sv, const double* S, int slot_rho, int slot_rv,
                   hipStream_t s);
void launch_bicg_update(int n, double* x, double* r, const double* pt, const double* st, const double* sv,
                        const double* t, const double* rb, const Reducer& R, int slot_rho, int slot_rv, int slot_tt,
                        int slot_ts, int slot_rr, int slot_rhonew, hipStream_t s);
// Sh/nsh/hseq/seq: the slot hand-over into mapped host memory (see the PCG
// direction kernel); null leaves it out.
void launch_bicg_dir(int n, const double* r, const double* p, const double* v, double* pn, const double* S,
                     int slot_rho, int slot_rv, int slot_tt, int slot_ts, int slot_rhonew, hipStream_t s,
                     double* Sh = nullptr, int nsh = 0, unsigned long long* hseq = nullptr,
                     unsigned long long seq = 0);
void launch_scale_zero(int n, double* x, hipStream_t s);
void launch_add(int n, double* x, const double* z, hipStream_t s);
// err |= ERR_NONFINITE if any entry of a or b is NaN or Inf.
void launch_check_finite(int n, const double* a, const double* b, int* err, hipStream_t s);

constexpr int kRedBlocks = 65536;  // max blocks (partials) of a reduction kernel
// Reductions whose consumer kernel adds the partials itself use at most this
// many blocks (each consumer block reads them all).
constexpr int kFusedParts = 2048;
// Partial regions of the PCG iteration inside Reducer::part (each holds up to
// kFusedParts): (p, q) of the SpMV, (r, r) of the update, (r, z) of the
// level-0 postsmoothing.
constexpr int kPartPQ = 0, kPartRR = 4096, kPartRZ = 8192;
constexpr int kPartialsOnly = -2;  // slot value: leave the block partials, no finish kernel

// ---- batched solves (k_batch.hip) -------------------------------------------
// Systems ("segments") stored one after another.  blk[b] = (segment, first
// row) of reduction block b (256 rows, never crossing a segment end);
// seg_end[s] = one past the segment's last row; mask[s] != 0 selects the
// segments a launch works on.  Scalars: S[s * kBatchSlots + slot].
constexpr int kBatchSlots = 8;
struct BatchTab {
    const int2* blk;
    const int* seg_end;
    const int* mask;
};
// Coarsest solve of one segment: x = A_L^{-1} f on n rows (f, x already
// offset to the segment), each result scattered to the finer level's rows
// through sc at index row0 + i.
template <class T>
struct BDense {
    int n;
    int row0;
    const double* ainv_t;
    const T* f;
    T* x;
    ScatterT<T> sc;
};
// One copy of a batch assembly: kind 0 int32 (+add), 1 double, 2 float,
// 3 int4 member lists (+add on the members present), 4 double rounded to
// float.
struct GatherPiece {
    const void* src;
    void* dst;
    int64_t count;
    int add;
    int kind;
};
int gather_chunk();  // elements per block of launch_gather

void launch_bspmv_dot(int nblk, const BatchTab& T, const int* rp, const int* ci, const double* v, const double* p,
                      double* q, const double* d, double* part, hipStream_t s);
void launch_bresidual(int nblk, const BatchTab& T, const int* rp, const int* ci, const double* v, const double* x,
                      const double* b, double* r, const double* dinv, void* g, bool g32, double* part,
                      hipStream_t s);
void launch_bdot(int nblk, const BatchTab& T, const double* a, const double* c, double* part, hipStream_t s);
void launch_bfinish(int nseg, const int* seg_blk, const int* mask, const double* part, double* S, int slot_k,
                    hipStream_t s);
void launch_bcg_update(int nblk, const BatchTab& T, double* x, double* r, const double* p, const double* q,
                       const double* dinv, void* g, bool g32, double* part, const double* S, int slot_rho,
                       int slot_pq, hipStream_t s);
void launch_bcg_dir(int nblk, const BatchTab& T, const double* z, const double* p, double* pn, const double* S,
                    int slot_new, int slot_old, hipStream_t s);
void launch_bzero(int nblk, const BatchTab& T, double* x, hipStream_t s);
// Algorithm 5 over a batch (two-sum kernels write their second partials at part + nblk).
void launch_bbicg_s(int nblk, const BatchTab& T, const double* r, const double* v, double* sv, const double* S,
                    int slot_rho, int slot_rv, hipStream_t s);
void launch_bspmv_dot2(int nblk, const BatchTab& T, const int* rp, const int* ci, const double* v, const double* st,
                       double* t, const double* sv, double* part, hipStream_t s);
void launch_bbicg_update(int nblk, const BatchTab& T, double* x, double* r, const double* pt, const double* st,
                         const double* sv, const double* t, const double* rb, double* part, const double* S,
                         int slot_rho, int slot_rv, int slot_tt, int slot_ts, hipStream_t s);
void launch_bbicg_dir(int nblk, const BatchTab& T, const double* r, const double* p, const double* v, double* pn,
                      const double* S, int slot_rho, int slot_rv, int slot_tt, int slot_ts, int slot_rhonew,
                      hipStream_t s);
template <class T>
void launch_bdense(int nblk, const BDense<T>* dd, const int2* tab, hipStream_t s);
void launch_gather(int nblk, const GatherPiece* pcs, const int2* tab, hipStream_t s);

}  // namespace amg
