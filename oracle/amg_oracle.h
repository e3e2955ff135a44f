/*
 * amg_oracle.h -- plain, slow, sequential CPU oracle of the aggregation-AMG
 * preconditioned Krylov method of "SParSH-AMG: A library for hybrid CPU-GPU
 * algebraic multigrid and preconditioned iterative methods" (Ganesan & Shah).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no source with the HIP library.
 *
 * Everything is FP64 with int32 0-based CSR indices, single-threaded, with
 * loops in index order.  Host pointers only.  Status codes use the same
 * numeric values as the product library so tests can compare them.
 */
#ifndef AMG_ORACLE_H
#define AMG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_OK = 0,
    ORACLE_EINVAL = 1,
    ORACLE_ENOMEM = 2,
    ORACLE_ENOTCONV = 3,
    ORACLE_EBREAKDOWN = 4,
    ORACLE_ENOTFINITE = 5,
    ORACLE_ESTALL = 6,
    ORACLE_ESINGULAR = 7
};

typedef struct {
    int32_t passes_per_level; /* HEM passes composed into one level (2)        */
    int32_t max_coarse_rows;  /* stop coarsening at n <= this (64)             */
    int32_t max_levels;       /* hierarchy depth limit, coarsest included (32) */
    int32_t max_dense_rows;   /* largest coarsest level accepted on a stall  *
                               * or at the depth limit (4096)                  */
    double omega;             /* Jacobi damping (2/3)                          */
    int32_t pre, post;        /* smoothing sweeps (1, 1)                       */
    double stall_ratio;       /* a level of n <= max_dense_rows rows becomes   *
                               * the coarsest when coarsening it would keep    *
                               * n_c >= stall_ratio * n rows (0.9); 1 stops    *
                               * only when no row is merged                    */
    int32_t hem;              /* 0: node-based matching (Algorithm 2), 1: edge- *
                               * based (Algorithm 3) (0)                       */
    int32_t alternate;        /* 1: node-based passes alternate direction, the *
                               * setup's passes counted from 0 across levels:  *
                               * even passes from the first index, odd ones    *
                               * from the last (0)                             */
} oracle_params;

typedef struct {
    int32_t iters;        /* number of solution updates                 */
    double rel_res;       /* recursive ||r|| / ||b|| at the stop        */
    double true_rel_res;  /* ||b - A x|| / ||b|| at the stop            */
    int32_t status;
} oracle_info;

/* Section 2.1.1, Algorithm 2: one node-based heavy-edge-matching pass.
 * mate[i] = partner of i, or -1 if i stays an unaggregated singleton. */
int oracle_hem_pass(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate);

/* Section 2.1.1, matching from the last index: the pass of Algorithm 2 with
 * the vertices visited in descending order and each row scanned in descending
 * column order, so equal weights go to the highest column index.  mate as in
 * oracle_hem_pass. */
int oracle_hem_pass_desc(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate);

/* Section 2.1.1, Algorithm 3: edge-based heavy-edge matching.  Every stored
 * non-zero off-diagonal entry (i, j) is an edge of weight |a_ij|; the list is
 * sorted by weight descending, ties by the smaller endpoint ascending, then
 * the larger ascending, and scanned once, matching both endpoints of an edge
 * whose endpoints are both unmatched.  mate as in oracle_hem_pass. */
int oracle_ehem_pass(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate);

/* Algorithm 2, counter C: aggregate ids in visiting order; returns n_c. */
int32_t oracle_number(int32_t n, const int32_t* mate, int32_t* agg);

/* Section 2.1.1: Galerkin product P^T B P with the 0/1 prolongation of agg.
 * oracle_rap_nnz returns the coarse nnz; oracle_rap fills caller buffers
 * (crp[nc+1], cci[nnz_c], cv[nnz_c]). */
int64_t oracle_rap_nnz(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* agg, int32_t nc);
int oracle_rap(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* agg, int32_t nc,
               int32_t* crp, int32_t* cci, double* cv);

/* y = A x */
void oracle_spmv(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const double* x, double* y);

/* Dense row-major partial-pivot LU (largest |pivot|, lowest row on ties). */
int oracle_lu_factor(int32_t n, double* a, int32_t* piv);
void oracle_lu_solve(int32_t n, const double* lu, const int32_t* piv, const double* b, double* x);

/* Hierarchy (Section 3 setup phase). */
typedef struct oracle_hier oracle_hier;
void oracle_params_default(oracle_params* p);
oracle_hier* oracle_setup(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const oracle_params* p,
                          int32_t* status);
int32_t oracle_nlevels(const oracle_hier* h);
int oracle_level_size(const oracle_hier* h, int32_t k, int32_t* n, int64_t* nnz);
int oracle_export_level(const oracle_hier* h, int32_t k, int32_t* rp, int32_t* ci, double* v, int32_t* agg);
void oracle_destroy(oracle_hier* h);

/* Algorithm 1: one V-cycle from a zero initial guess, z = M^{-1} f. */
int oracle_vcycle(const oracle_hier* h, const double* f, double* z);

/* Algorithm 4 (method 0, PCG), Algorithm 5 (method 1, BiCGStab), or
 * Algorithm 1 iterated as a stationary solver (method 2: x += V(b - A x),
 * stopping on the recomputed residual; precond and true_res_period unused).
 * precond = 1 applies one V-cycle per preconditioner call, 0 uses M = I.
 * x holds the initial guess on entry and the iterate on return. */
int oracle_krylov(const oracle_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                  int32_t true_res_period, int32_t precond, oracle_info* info);

#ifdef __cplusplus
}
#endif
#endif
