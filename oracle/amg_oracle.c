/*
 * amg_oracle.c -- sequential CPU oracle of the aggregation-AMG Krylov method.
 *
 * TEST INFRASTRUCTURE ONLY (see amg_oracle.h).  Written for reading, not for
 * speed: every loop runs in index order, every sum is a plain left-to-right
 * accumulation, and each function names the passage of the paper it follows.
 *
 * Readings taken where the paper is silent or garbled:
 *  - among equal heavy-edge weights the lowest column index wins (the highest
 *    in a pass from the last index); explicit zeros are not edges;
 *  - a level that stalls (no row merged) or reaches the depth limit becomes
 *    the dense coarsest level if it has at most max_dense_rows (4096) rows;
 *  - a level applies `passes_per_level` matching passes, each on the Galerkin
 *    operator of the previous pass, and composes their aggregate maps;
 *  - a coarse entry (I,J) is the sum of the fine entries b_ij with i in I,
 *    agg(j) = J, taken in order of ascending i and then ascending j; the first
 *    contribution initialises the sum.  Entries whose sum is 0 are kept;
 *  - the coarsest level is solved by dense partial-pivot LU;
 *  - damped Jacobi smoothing starts from a zero guess on every level;
 *  - the residual update of PCG subtracts alpha*A*p;
 *  - BiCGStab starts with p_0 = r_0 and shadow residual r_0, and updates the
 *    search direction with A applied to the preconditioned direction;
 *  - convergence is ||r||/||b|| <= rtol on the recursive residual, confirmed
 *    by recomputing b - A x (also every `true_res_period` iterations).
 */
#include "amg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV 64

/* ------------------------------------------------------------------------ */
/* Section 2.1.1, Algorithm 2: node-based heavy edge matching.               */
/* ------------------------------------------------------------------------ */
/* Preference between two free neighbours of a vertex: the heavier coupling  */
/* |a_ij| wins; between equal weights the lower column wins when vertices    */
/* are visited upward and the higher column when they are visited downward   */
/* (the neighbour met first in the visiting direction).                      */
static int prefer(double w, int32_t j, double best_w, int32_t best_j, int down) {
    if (best_j < 0) return 1;
    if (w != best_w) return w > best_w;
    return down ? j > best_j : j < best_j;
}

/* The most preferred neighbour of vertex i that is still free: a stored,   */
/* non-zero off-diagonal entry a_ij with j not yet taken.  -1 if none.       */
static int32_t heaviest_free(const int32_t* rp, const int32_t* ci, const double* v, const char* taken, int32_t i,
                             int down) {
    int32_t best_j = -1;
    double best_w = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = ci[e];
        if (j == i || v[e] == 0.0 || taken[j]) continue;
        const double w = fabs(v[e]);
        if (prefer(w, j, best_w, best_j, down)) {
            best_w = w;
            best_j = j;
        }
    }
    return best_j;
}

/* One greedy pass: each vertex, in visiting order, that nobody has taken    */
/* yet takes its most preferred free neighbour (both become a pair) or,      */
/* without one, stays alone.  mate[u] = partner, or -1 for a singleton.      */
static int greedy_pass(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate, int down) {
    char* taken = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!taken) return ORACLE_ENOMEM;
    for (int32_t u = 0; u < n; ++u) mate[u] = -1;
    for (int32_t t = 0; t < n; ++t) {
        const int32_t u = down ? n - 1 - t : t;
        if (taken[u]) continue;
        taken[u] = 1;
        const int32_t w = heaviest_free(rp, ci, v, taken, u, down);
        if (w >= 0) {
            mate[u] = w;
            mate[w] = u;
            taken[w] = 1;
        }
    }
    free(taken);
    return ORACLE_OK;
}

/* Vertices visited from the first index (the order Algorithm 2 prints). */
int oracle_hem_pass(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate) {
    return greedy_pass(n, rp, ci, v, mate, 0);
}

/* Section 2.1.1, matching from the last index: the same rule with the      */
/* vertices visited from n-1 down to 0, equal weights going to the higher   */
/* column.                                                                   */
int oracle_hem_pass_desc(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate) {
    return greedy_pass(n, rp, ci, v, mate, 1);
}

typedef struct {
    double w;
    int32_t lo, hi;
} oedge;

static int edge_order(const void* a, const void* b) {
    const oedge* x = (const oedge*)a;
    const oedge* y = (const oedge*)b;
    if (x->w != y->w) return x->w > y->w ? -1 : 1; /* heaviest first */
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    return 0;
}

int oracle_ehem_pass(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t* mate) {
    int64_t m = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] != i && v[e] != 0.0) ++m;
    oedge* T = (oedge*)malloc(sizeof(oedge) * (size_t)(m > 0 ? m : 1));
    char* assigned = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!T || !assigned) {
        free(T), free(assigned);
        return ORACLE_ENOMEM;
    }
    m = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t j = ci[e];
            if (j == i || v[e] == 0.0) continue;
            T[m].w = fabs(v[e]);
            T[m].lo = i < j ? i : j;
            T[m].hi = i < j ? j : i;
            ++m;
        }
    qsort(T, (size_t)m, sizeof(oedge), edge_order);
    for (int32_t i = 0; i < n; ++i) mate[i] = -1;
    for (int64_t k = 0; k < m; ++k) {
        const int32_t i = T[k].lo, j = T[k].hi;
        if (!assigned[i] && !assigned[j]) {
            mate[i] = j;
            mate[j] = i;
            assigned[i] = assigned[j] = 1;
        }
    }
    free(T), free(assigned);
    return ORACLE_OK;
}

/* Algorithm 2, coarse counter C: the coarse id is handed out when the lower */
/* vertex of a pair (or a singleton) is visited, so ids follow the minimum   */
/* fine index of each aggregate.                                             */
int32_t oracle_number(int32_t n, const int32_t* mate, int32_t* agg) {
    int32_t c = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (mate[i] < 0) {
            agg[i] = c++;
        } else if (i < mate[i]) {
            agg[i] = c;
            agg[mate[i]] = c;
            ++c;
        }
    }
    return c;
}

/* Member lists of each aggregate, members in ascending fine index. */
static int members(int32_t n, const int32_t* agg, int32_t nc, int32_t** mptr, int32_t** mem) {
    int32_t* p = (int32_t*)calloc((size_t)nc + 1, sizeof(int32_t));
    int32_t* m = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    if (!p || !m || !fill) {
        free(p), free(m), free(fill);
        return ORACLE_ENOMEM;
    }
    for (int32_t i = 0; i < n; ++i) p[agg[i] + 1]++;
    for (int32_t c = 0; c < nc; ++c) p[c + 1] += p[c];
    for (int32_t c = 0; c < nc; ++c) fill[c] = p[c];
    for (int32_t i = 0; i < n; ++i) m[fill[agg[i]]++] = i; /* ascending i */
    free(fill);
    *mptr = p;
    *mem = m;
    return ORACLE_OK;
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Section 2.1.1: A_c = P^T B P with P_{i,agg(i)} = 1.  Entry (I,J) is the sum */
/* of b_ij over i in I and agg(j) = J.  Dense-accumulator (Gustavson) form.    */
static int64_t rap_impl(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* agg,
                        int32_t nc, int32_t* crp, int32_t* cci, double* cv) {
    int32_t *mptr = NULL, *mem = NULL;
    if (members(n, agg, nc, &mptr, &mem) != ORACLE_OK) return -1;
    int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    double* acc = (double*)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    if (!mark || !acc || !list) {
        free(mptr), free(mem), free(mark), free(acc), free(list);
        return -1;
    }
    for (int32_t c = 0; c < nc; ++c) mark[c] = -1;
    int64_t nnz = 0;
    if (crp) crp[0] = 0;
    for (int32_t I = 0; I < nc; ++I) {
        int32_t len = 0;
        for (int32_t t = mptr[I]; t < mptr[I + 1]; ++t) {
            int32_t i = mem[t];
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                int32_t J = agg[ci[e]];
                if (mark[J] != I) {
                    mark[J] = I;
                    acc[J] = v ? v[e] : 0.0; /* first contribution */
                    list[len++] = J;
                } else if (v) {
                    acc[J] += v[e];
                }
            }
        }
        qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
        if (cci) {
            for (int32_t t = 0; t < len; ++t) {
                cci[nnz + t] = list[t];
                cv[nnz + t] = acc[list[t]];
            }
        }
        nnz += len;
        if (crp) crp[I + 1] = (int32_t)nnz;
    }
    free(mptr), free(mem), free(mark), free(acc), free(list);
    return nnz;
}

int64_t oracle_rap_nnz(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* agg, int32_t nc) {
    return rap_impl(n, rp, ci, NULL, agg, nc, NULL, NULL, NULL);
}

int oracle_rap(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* agg, int32_t nc,
               int32_t* crp, int32_t* cci, double* cv) {
    return rap_impl(n, rp, ci, v, agg, nc, crp, cci, cv) < 0 ? ORACLE_ENOMEM : ORACLE_OK;
}

void oracle_spmv(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const double* x, double* y) {
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * x[ci[e]];
        y[i] = s;
    }
}

/* Coarsest-level direct solver (Section 2, coarse level solver): textbook    */
/* Doolittle LU with partial pivoting, P A = L U, stored in place.            */
int oracle_lu_factor(int32_t n, double* a, int32_t* piv) {
    for (int32_t k = 0; k < n; ++k) {
        int32_t p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int32_t i = k + 1; i < n; ++i) {
            double t = fabs(a[(size_t)i * n + k]);
            if (t > best) {
                best = t;
                p = i;
            }
        }
        piv[k] = p;
        if (best == 0.0) return ORACLE_ESINGULAR;
        if (p != k)
            for (int32_t j = 0; j < n; ++j) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        for (int32_t i = k + 1; i < n; ++i) {
            double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
            a[(size_t)i * n + k] = l;
            for (int32_t j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return ORACLE_OK;
}

void oracle_lu_solve(int32_t n, const double* lu, const int32_t* piv, const double* b, double* x) {
    for (int32_t i = 0; i < n; ++i) x[i] = b[i];
    for (int32_t k = 0; k < n; ++k) { /* apply the row swaps in order */
        double t = x[k];
        x[k] = x[piv[k]];
        x[piv[k]] = t;
    }
    for (int32_t i = 0; i < n; ++i) /* L y = P b, unit diagonal */
        for (int32_t j = 0; j < i; ++j) x[i] -= lu[(size_t)i * n + j] * x[j];
    for (int32_t i = n - 1; i >= 0; --i) { /* U x = y */
        for (int32_t j = i + 1; j < n; ++j) x[i] -= lu[(size_t)i * n + j] * x[j];
        x[i] /= lu[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Hierarchy                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t *rp, *ci;
    double* v;
    double* dinv;
    int32_t* agg; /* map to level k+1 (NULL on the coarsest level) */
} olevel;

struct oracle_hier {
    oracle_params p;
    int32_t nlev; /* levels 0..nlev-1, the last is solved directly */
    olevel lev[MAXLEV];
    double* lu;
    int32_t* piv;
};

void oracle_params_default(oracle_params* p) {
    p->passes_per_level = 2;
    p->max_coarse_rows = 64;
    p->max_levels = 32;
    p->max_dense_rows = 4096;
    p->stall_ratio = 0.9;
    p->hem = 0;
    p->alternate = 0;
    p->omega = 2.0 / 3.0;
    p->pre = 1;
    p->post = 1;
}

static void free_level(olevel* L) {
    free(L->rp), free(L->ci), free(L->v), free(L->dinv), free(L->agg);
    memset(L, 0, sizeof(*L));
}

void oracle_destroy(oracle_hier* h) {
    if (!h) return;
    for (int32_t k = 0; k < MAXLEV; ++k) free_level(&h->lev[k]);
    free(h->lu), free(h->piv);
    free(h);
}

static int check_csr(int32_t n, const int32_t* rp, const int32_t* ci, const double* v) {
    if (n <= 0 || rp[0] != 0) return ORACLE_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return ORACLE_EINVAL;
        int diag = 0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return ORACLE_EINVAL;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return ORACLE_EINVAL;
            if (!isfinite(v[e])) return ORACLE_ENOTFINITE;
            if (ci[e] == i) {
                if (v[e] == 0.0) return ORACLE_EINVAL;
                diag = 1;
            }
        }
        if (!diag) return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

static int make_dinv(olevel* L) {
    L->dinv = (double*)malloc(sizeof(double) * (size_t)L->n);
    if (!L->dinv) return ORACLE_ENOMEM;
    for (int32_t i = 0; i < L->n; ++i) {
        L->dinv[i] = 0.0;
        for (int32_t e = L->rp[i]; e < L->rp[i + 1]; ++e)
            if (L->ci[e] == i) L->dinv[i] = 1.0 / L->v[e];
        if (L->dinv[i] == 0.0 || !isfinite(L->dinv[i])) return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/* One coarsening step: passes_per_level rounds of (Alg. 2 + Galerkin product), */
/* composing the aggregate maps.  On success fills *C and fine->agg.  `first`   */
/* is the setup-wide index of the level's first pass; with `alternate` the odd  */
/* ones run from the last index.  Coarse ids follow each aggregate's smallest   */
/* fine index in either direction.                                             */
static int coarsen(olevel* F, int32_t passes, int32_t hem, int32_t alternate, int32_t first, olevel* C) {
    int32_t n = F->n;
    int32_t* rp = F->rp;
    int32_t* ci = F->ci;
    double* v = F->v;
    int owned = 0; /* whether rp/ci/v are intermediate products to free */
    int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->n);
    int32_t* mate = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->n);
    int32_t* agg = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->n);
    if (!comp || !mate || !agg) return ORACLE_ENOMEM;
    for (int32_t i = 0; i < F->n; ++i) comp[i] = i;
    for (int32_t p = 0; p < passes; ++p) {
        if (hem == 1) {
            if (oracle_ehem_pass(n, rp, ci, v, mate) != ORACLE_OK) return ORACLE_ENOMEM;
        } else if (alternate && ((first + p) & 1)) {
            if (oracle_hem_pass_desc(n, rp, ci, v, mate) != ORACLE_OK) return ORACLE_ENOMEM;
        } else {
            if (oracle_hem_pass(n, rp, ci, v, mate) != ORACLE_OK) return ORACLE_ENOMEM;
        }
        int32_t nc = oracle_number(n, mate, agg); /* ids by each aggregate's minimum fine index */
        int64_t nnzc = oracle_rap_nnz(n, rp, ci, agg, nc);
        int32_t* crp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nc + 1));
        int32_t* cci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnzc > 0 ? nnzc : 1));
        double* cv = (double*)malloc(sizeof(double) * (size_t)(nnzc > 0 ? nnzc : 1));
        if (nnzc < 0 || !crp || !cci || !cv) return ORACLE_ENOMEM;
        oracle_rap(n, rp, ci, v, agg, nc, crp, cci, cv);
        for (int32_t i = 0; i < F->n; ++i) comp[i] = agg[comp[i]]; /* compose */
        if (owned) free(rp), free(ci), free(v);
        rp = crp, ci = cci, v = cv, n = nc, owned = 1;
    }
    free(mate), free(agg);
    C->n = n;
    C->nnz = rp[n];
    C->rp = rp, C->ci = ci, C->v = v;
    F->agg = comp;
    return make_dinv(C);
}

static int copy_level(olevel* L, int32_t n, const int32_t* rp, const int32_t* ci, const double* v) {
    L->n = n;
    L->nnz = rp[n];
    L->rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    L->ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->nnz > 0 ? L->nnz : 1));
    L->v = (double*)malloc(sizeof(double) * (size_t)(L->nnz > 0 ? L->nnz : 1));
    if (!L->rp || !L->ci || !L->v) return ORACLE_ENOMEM;
    memcpy(L->rp, rp, sizeof(int32_t) * ((size_t)n + 1));
    memcpy(L->ci, ci, sizeof(int32_t) * (size_t)L->nnz);
    memcpy(L->v, v, sizeof(double) * (size_t)L->nnz);
    return make_dinv(L);
}

/* Section 3, setup phase: coarsen until the level is small enough for the    */
/* direct solver, then factor the coarsest matrix once.                       */
oracle_hier* oracle_setup(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, const oracle_params* p,
                          int32_t* status) {
    int st = check_csr(n, rp, ci, v);
    if (st != ORACLE_OK) {
        *status = st;
        return NULL;
    }
    oracle_hier* h = (oracle_hier*)calloc(1, sizeof(oracle_hier));
    if (!h) {
        *status = ORACLE_ENOMEM;
        return NULL;
    }
    if (p) h->p = *p;
    else oracle_params_default(&h->p);
    int32_t maxlev = h->p.max_levels < MAXLEV ? h->p.max_levels : MAXLEV;
    if (h->p.passes_per_level < 1 || maxlev < 1 || h->p.pre < 0 || h->p.post < 0 ||
        !(h->p.stall_ratio > 0.0 && h->p.stall_ratio <= 1.0) || h->p.hem < 0 || h->p.hem > 1 ||
        h->p.alternate < 0 || h->p.alternate > 1 || (h->p.alternate && h->p.hem)) {
        oracle_destroy(h);
        *status = ORACLE_EINVAL;
        return NULL;
    }
    st = copy_level(&h->lev[0], n, rp, ci, v);
    int32_t k = 0;
    while (st == ORACLE_OK) {
        olevel* F = &h->lev[k];
        if (F->n <= h->p.max_coarse_rows) break;
        if (k + 1 >= maxlev) { /* depth limit reached above the coarse size */
            if (F->n > h->p.max_dense_rows) st = ORACLE_ESTALL;
            break;
        }
        st = coarsen(F, h->p.passes_per_level, h->p.hem, h->p.alternate, k * h->p.passes_per_level, &h->lev[k + 1]);
        if (st != ORACLE_OK) break;
        if (h->lev[k + 1].n == F->n) { /* no progress */
            free_level(&h->lev[k + 1]);
            free(F->agg);
            F->agg = NULL;
            if (F->n > h->p.max_dense_rows) st = ORACLE_ESTALL;
            break;
        }
        /* poor progress on a level the dense solve can take: it is the coarsest */
        if ((double)h->lev[k + 1].n >= h->p.stall_ratio * (double)F->n && F->n <= h->p.max_dense_rows) {
            free_level(&h->lev[k + 1]);
            free(F->agg);
            F->agg = NULL;
            break;
        }
        ++k;
    }
    if (st != ORACLE_OK) {
        oracle_destroy(h);
        *status = st;
        return NULL;
    }
    h->nlev = k + 1;
    olevel* L = &h->lev[k];
    free(L->agg);
    L->agg = NULL;
    int32_t m = L->n;
    h->lu = (double*)calloc((size_t)m * m, sizeof(double));
    h->piv = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    if (!h->lu || !h->piv) {
        oracle_destroy(h);
        *status = ORACLE_ENOMEM;
        return NULL;
    }
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = L->rp[i]; e < L->rp[i + 1]; ++e) h->lu[(size_t)i * m + L->ci[e]] = L->v[e];
    st = oracle_lu_factor(m, h->lu, h->piv);
    if (st != ORACLE_OK) {
        oracle_destroy(h);
        *status = st;
        return NULL;
    }
    *status = ORACLE_OK;
    return h;
}

int32_t oracle_nlevels(const oracle_hier* h) { return h->nlev; }

int oracle_level_size(const oracle_hier* h, int32_t k, int32_t* n, int64_t* nnz) {
    if (k < 0 || k >= h->nlev) return ORACLE_EINVAL;
    *n = h->lev[k].n;
    *nnz = h->lev[k].nnz;
    return ORACLE_OK;
}

int oracle_export_level(const oracle_hier* h, int32_t k, int32_t* rp, int32_t* ci, double* v, int32_t* agg) {
    if (k < 0 || k >= h->nlev) return ORACLE_EINVAL;
    const olevel* L = &h->lev[k];
    if (rp) memcpy(rp, L->rp, sizeof(int32_t) * ((size_t)L->n + 1));
    if (ci) memcpy(ci, L->ci, sizeof(int32_t) * (size_t)L->nnz);
    if (v) memcpy(v, L->v, sizeof(double) * (size_t)L->nnz);
    if (agg && L->agg) memcpy(agg, L->agg, sizeof(int32_t) * (size_t)L->n);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: V-cycle(k, f, 0, A_k) with damped Jacobi smoothing.          */
/* ------------------------------------------------------------------------ */
/* x <- x + omega * D^{-1} (f - A x), the whole old x used on the right. */
static void jacobi(const olevel* L, double omega, const double* f, double* x, double* tmp) {
    oracle_spmv(L->n, L->rp, L->ci, L->v, x, tmp);
    for (int32_t i = 0; i < L->n; ++i) x[i] = x[i] + omega * (L->dinv[i] * (f[i] - tmp[i]));
}

static void vcycle(const oracle_hier* h, int32_t k, const double* f, double* x) {
    const olevel* L = &h->lev[k];
    int32_t n = L->n;
    if (k == h->nlev - 1) { /* exact solve on the coarsest level */
        oracle_lu_solve(n, h->lu, h->piv, f, x);
        return;
    }
    double omega = h->p.omega;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
    const olevel* C = &h->lev[k + 1];
    double* fc = (double*)malloc(sizeof(double) * (size_t)C->n);
    double* ec = (double*)malloc(sizeof(double) * (size_t)C->n);
    /* presmoothing from the zero initial guess */
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    for (int32_t s = 0; s < h->p.pre; ++s) jacobi(L, omega, f, x, tmp);
    /* residual r = f - A x and restriction f_c = P^T r (members ascending) */
    oracle_spmv(n, L->rp, L->ci, L->v, x, tmp);
    for (int32_t i = 0; i < n; ++i) tmp[i] = f[i] - tmp[i];
    char* seen = (char*)calloc((size_t)C->n, 1);
    for (int32_t i = 0; i < n; ++i) {
        int32_t I = L->agg[i];
        if (!seen[I]) {
            fc[I] = tmp[i];
            seen[I] = 1;
        } else {
            fc[I] += tmp[i];
        }
    }
    free(seen);
    /* coarse correction, then prolongation x += P e_c */
    vcycle(h, k + 1, fc, ec);
    for (int32_t i = 0; i < n; ++i) x[i] += ec[L->agg[i]];
    for (int32_t s = 0; s < h->p.post; ++s) jacobi(L, omega, f, x, tmp);
    free(tmp), free(fc), free(ec);
}

int oracle_vcycle(const oracle_hier* h, const double* f, double* z) {
    vcycle(h, 0, f, z);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithms 4 and 5                                                       */
/* ------------------------------------------------------------------------ */
static double dot(int32_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void precondition(const oracle_hier* h, int32_t precond, const double* r, double* z) {
    if (precond) vcycle(h, 0, r, z);
    else memcpy(z, r, sizeof(double) * (size_t)h->lev[0].n);
}

/* r = b - A x, returns ||r|| */
static double true_residual(const olevel* A, const double* b, const double* x, double* r) {
    oracle_spmv(A->n, A->rp, A->ci, A->v, x, r);
    for (int32_t i = 0; i < A->n; ++i) r[i] = b[i] - r[i];
    return sqrt(dot(A->n, r, r));
}

static int pcg(const oracle_hier* h, const double* b, double* x, double rtol, int32_t maxit, int32_t period,
               int32_t precond, oracle_info* info) {
    const olevel* A = &h->lev[0];
    int32_t n = A->n;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n), *p = malloc(sizeof(double) * n),
           *q = malloc(sizeof(double) * n);
    int st = ORACLE_ENOTCONV;
    double nb = sqrt(dot(n, b, b));
    info->iters = 0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        info->rel_res = info->true_rel_res = 0.0;
        st = ORACLE_OK;
        goto done;
    }
    double rel = true_residual(A, b, x, r) / nb;
    info->rel_res = info->true_rel_res = rel;
    if (rel <= rtol) {
        st = ORACLE_OK;
        goto done;
    }
    precondition(h, precond, r, z);
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    for (int32_t it = 1; it <= maxit; ++it) {
        oracle_spmv(n, A->rp, A->ci, A->v, p, q);
        double pq = dot(n, p, q);
        if (!isfinite(pq) || pq == 0.0 || !isfinite(rho)) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        info->iters = it;
        rel = sqrt(dot(n, r, r)) / nb;
        info->rel_res = rel;
        if (!isfinite(rel)) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        if (rel <= rtol || (period > 0 && it % period == 0)) {
            double tr = true_residual(A, b, x, r) / nb; /* residual replacement */
            info->true_rel_res = tr;
            if (tr <= rtol) {
                st = ORACLE_OK;
                break;
            }
        }
        precondition(h, precond, r, z);
        double rho_new = dot(n, r, z);
        if (!isfinite(rho_new) || rho_new == 0.0) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        double beta = rho_new / rho;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
done:
    free(r), free(z), free(p), free(q);
    return st;
}

static int bicgstab(const oracle_hier* h, const double* b, double* x, double rtol, int32_t maxit, int32_t period,
                    int32_t precond, oracle_info* info) {
    const olevel* A = &h->lev[0];
    int32_t n = A->n;
    size_t sz = sizeof(double) * (size_t)n;
    double *r = malloc(sz), *rb = malloc(sz), *p = malloc(sz), *pt = malloc(sz), *v = malloc(sz), *s = malloc(sz),
           *st_ = malloc(sz), *t = malloc(sz);
    int st = ORACLE_ENOTCONV;
    double nb = sqrt(dot(n, b, b));
    info->iters = 0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        info->rel_res = info->true_rel_res = 0.0;
        st = ORACLE_OK;
        goto done;
    }
    double rel = true_residual(A, b, x, r) / nb;
    info->rel_res = info->true_rel_res = rel;
    if (rel <= rtol) {
        st = ORACLE_OK;
        goto done;
    }
    memcpy(rb, r, sz);
    memcpy(p, r, sz);
    double rho = dot(n, r, rb);
    for (int32_t it = 1; it <= maxit; ++it) {
        precondition(h, precond, p, pt);
        oracle_spmv(n, A->rp, A->ci, A->v, pt, v);
        double rv = dot(n, rb, v);
        if (!isfinite(rv) || rv == 0.0 || !isfinite(rho) || rho == 0.0) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        double alpha = rho / rv;
        for (int32_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        precondition(h, precond, s, st_);
        oracle_spmv(n, A->rp, A->ci, A->v, st_, t);
        double tt = dot(n, t, t), ts = dot(n, t, s);
        if (!isfinite(tt) || !isfinite(ts) || tt == 0.0) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        double omega = ts / tt;
        for (int32_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * pt[i] + omega * st_[i];
            r[i] = s[i] - omega * t[i];
        }
        info->iters = it;
        rel = sqrt(dot(n, r, r)) / nb;
        info->rel_res = rel;
        if (!isfinite(rel)) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        if (rel <= rtol || (period > 0 && it % period == 0)) {
            double tr = true_residual(A, b, x, r) / nb;
            info->true_rel_res = tr;
            if (tr <= rtol) {
                st = ORACLE_OK;
                break;
            }
        }
        double rho_new = dot(n, r, rb);
        if (omega == 0.0 || !isfinite(rho_new) || rho_new == 0.0) {
            st = ORACLE_EBREAKDOWN;
            break;
        }
        double beta = (rho_new / rho) * (alpha / omega);
        for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        rho = rho_new;
    }
done:
    free(r), free(rb), free(p), free(pt), free(v), free(s), free(st_), free(t);
    return st;
}

/* AMG as a stationary solver (Algorithm 1 repeated, the "AMG as a solver"
 * use of Section 4): x <- x + V(b - A x) until ||b - A x|| <= rtol ||b||.
 * The residual is recomputed every iteration, so it is the true one. */
static int stationary(const oracle_hier* h, const double* b, double* x, double rtol, int32_t maxit,
                      oracle_info* info) {
    const olevel* A = &h->lev[0];
    int32_t n = A->n;
    size_t sz = sizeof(double) * (size_t)n;
    double *r = malloc(sz), *z = malloc(sz);
    int st = ORACLE_ENOTCONV;
    double nb = sqrt(dot(n, b, b));
    info->iters = 0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        info->rel_res = info->true_rel_res = 0.0;
        st = ORACLE_OK;
        goto done;
    }
    double rel = true_residual(A, b, x, r) / nb;
    info->rel_res = info->true_rel_res = rel;
    for (int32_t it = 1; rel > rtol; ++it) {
        if (it > maxit) goto done;
        oracle_vcycle(h, r, z);
        for (int32_t i = 0; i < n; ++i) x[i] += z[i];
        info->iters = it;
        rel = true_residual(A, b, x, r) / nb;
        info->rel_res = info->true_rel_res = rel;
        if (!isfinite(rel)) {
            st = ORACLE_EBREAKDOWN;
            goto done;
        }
    }
    st = ORACLE_OK;
done:
    free(r), free(z);
    return st;
}

int oracle_krylov(const oracle_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                  int32_t true_res_period, int32_t precond, oracle_info* info) {
    oracle_info local;
    if (!info) info = &local;
    memset(info, 0, sizeof(*info));
    for (int32_t i = 0; i < h->lev[0].n; ++i)
        if (!isfinite(b[i]) || !isfinite(x[i])) {
            info->status = ORACLE_ENOTFINITE;
            return ORACLE_ENOTFINITE;
        }
    int st;
    if (method == 0) st = pcg(h, b, x, rtol, maxit, true_res_period, precond, info);
    else if (method == 1) st = bicgstab(h, b, x, rtol, maxit, true_res_period, precond, info);
    else if (method == 2) st = stationary(h, b, x, rtol, maxit, info);
    else st = ORACLE_EINVAL;
    info->status = st;
    return st;
}
