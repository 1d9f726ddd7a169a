/*
 * amg_oracle.c -- plain, slow, FP64 CPU reference of sparsified AMG.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the device library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product never calls it and shares no
 * code with it.  Built with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math), single threaded (the parity build).  A second build with
 * -fopenmp (the timing build of the CPU baseline) runs the solve phase's row
 * loops and the blocks of the inner products on all host cores; every row is
 * still summed by one thread in column order and the inner products add
 * fixed blocks in block order, so both builds give the same bits.
 *
 * Paper: Bienz, Falgout, Gropp, Olson, Schroder, "Reducing Parallel
 * Communication in Algebraic Multigrid through Sparsification" (2016).
 *
 *   setup      Section 2, algorithm amg_setup (strength -> interpolation ->
 *              Galerkin product), run without the optional sparsify step, as
 *              Section 3, algorithm sparse_hybrid_setup, prescribes; C/F
 *              split by the Ruge-Stueben first pass or by PMIS, the parallel
 *              aggressive coarsening Section 1 cites.
 *   sparsify   Section 2.1, Algorithm 3 (first loop: minimal pattern M and
 *              keep set N) with the diagonal-lumping loop of Algorithm 3b
 *              (Section 3.1); Sparse Galerkin (M from the Galerkin A_{l-1})
 *              or Hybrid Galerkin (M from the sparsified \hat A_{l-1}).
 *   solve      Section 2, algorithm amg_solve (V-cycle); Section 6,
 *              algorithm adaptive_solve (windowed reintroduction).
 *
 * Where the paper is silent or garbled (strength formula, RS split, direct
 * interpolation, canonical summation order, gamma ladder, window rules) the
 * comment above each function states the reading it implements.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOTHING 1
#define OR_EINVAL -1
#define OR_EMATRIX -2
#define OR_ENOMEM -3
#define OR_ENOTCONV -5
#define OR_EBREAK -6

typedef struct {
    int nr, nc;
    int *rp, *ci;
    double *v;
} Mat;

typedef struct {
    Mat A;          /* Galerkin operator A_l (retained, never modified)     */
    Mat Ah;         /* sparsified operator \hat A_l (== A for gamma 0)      */
    Mat P;          /* interpolation P_l : R^{n_{l+1}} -> R^{n_l}           */
    Mat R;          /* R_l = P_l^T                                         */
    Mat S;          /* strength pattern S_l (values unused)                */
    int *cf;        /* 1 = C point, 0 = F point (levels < L)               */
    int *cidx;      /* coarse index of a C point, -1 for F                 */
    unsigned char *inM;   /* minimal-pattern flag per nonzero of A_l (l>=1) */
    unsigned char *keep;  /* keep flag of the last sparsify, per nnz of A_l  */
    double *rowmax;       /* m_i = max_{k!=i} |a_ik| of A_l                  */
    double gamma;
} Level;

typedef struct {
    int nlev;
    Level *lv;
    int hybrid;     /* 0: Sparse Galerkin, 1: Hybrid Galerkin (Section 3)   */
    int relax;      /* 0: weighted Jacobi, 1: hybrid symmetric Gauss-Seidel */
    int lumping;    /* 0: diagonal (Algorithm 3b), 1: strong neighbours      */
    double theta;   /* strength threshold of the setup                      */
    int gs_block;   /* rows per block of the hybrid Gauss-Seidel sweep      */
    double omega;
    int nu_pre, nu_post;
    /* coarsest-level dense factor */
    int nL;
    double *fac;    /* Cholesky factor (lower) or LU factors */
    int *piv;       /* NULL for Cholesky */
    /* work vectors per level */
    double **b, **x, **r;
} Hier;

typedef struct {
    int iters, restarts, reintroductions, converged;
    double relres, rho_avg;
} SolveInfo;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static void mat_free(Mat *m) {
    free(m->rp); free(m->ci); free(m->v);
    memset(m, 0, sizeof(*m));
}

static int mat_alloc(Mat *m, int nr, int nc, long nnz) {
    m->nr = nr; m->nc = nc;
    m->rp = (int *)calloc((size_t)nr + 1, sizeof(int));
    m->ci = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    m->v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    return (m->rp && m->ci && m->v) ? OR_OK : OR_ENOMEM;
}

static int mat_copy(Mat *dst, const Mat *src) {
    long nnz = src->rp[src->nr];
    if (mat_alloc(dst, src->nr, src->nc, nnz)) return OR_ENOMEM;
    memcpy(dst->rp, src->rp, sizeof(int) * ((size_t)src->nr + 1));
    memcpy(dst->ci, src->ci, sizeof(int) * (size_t)nnz);
    memcpy(dst->v, src->v, sizeof(double) * (size_t)nnz);
    return OR_OK;
}

/* position of column j in row i of m (columns sorted), -1 if absent */
static long find_pos(const Mat *m, int i, int j) {
    int lo = m->rp[i], hi = m->rp[i + 1] - 1;
    while (lo <= hi) {
        int mid = lo + (hi - lo) / 2;
        if (m->ci[mid] == j) return mid;
        if (m->ci[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* transpose by counting; rows of the result list source rows ascending */
static int mat_transpose(const Mat *a, Mat *t) {
    long nnz = a->rp[a->nr];
    if (mat_alloc(t, a->nc, a->nr, nnz)) return OR_ENOMEM;
    for (long p = 0; p < nnz; ++p) t->rp[a->ci[p] + 1]++;
    for (int i = 0; i < a->nc; ++i) t->rp[i + 1] += t->rp[i];
    int *fill = (int *)malloc(sizeof(int) * ((size_t)a->nc + 1));
    if (!fill) return OR_ENOMEM;
    memcpy(fill, t->rp, sizeof(int) * ((size_t)a->nc + 1));
    for (int i = 0; i < a->nr; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int q = fill[a->ci[p]]++;
            t->ci[q] = i;
            t->v[q] = a->v ? a->v[p] : 1.0;   /* a pattern without values: ones */
        }
    free(fill);
    return OR_OK;
}

/* Inner product in fixed blocks of 8,192 entries: each block summed in index
   order, the block sums added in block order, so that the result does not
   depend on how many threads form the block sums. */
#define OR_DOT_BLOCK 8192
static double dot(int n, const double *a, const double *b) {
    int nb = (n + OR_DOT_BLOCK - 1) / OR_DOT_BLOCK;
    double part_small[64];
    double *part = nb <= 64 ? part_small : (double *)malloc(sizeof(double) * (size_t)nb);
    if (!part) return NAN;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int k = 0; k < nb; ++k) {
        int lo = k * OR_DOT_BLOCK, hi = lo + OR_DOT_BLOCK < n ? lo + OR_DOT_BLOCK : n;
        double s = 0.0;
        for (int i = lo; i < hi; ++i) s += a[i] * b[i];
        part[k] = s;
    }
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    if (part != part_small) free(part);
    return s;
}

/* y = M x, each row summed in ascending column order */
static void spmv(const Mat *m, const double *x, double *y) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int i = 0; i < m->nr; ++i) {
        double s = 0.0;
        for (int p = m->rp[i]; p < m->rp[i + 1]; ++p) s += m->v[p] * x[m->ci[p]];
        y[i] = s;
    }
}

/* r = b - M x */
static void residual(const Mat *m, const double *b, const double *x, double *r) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int i = 0; i < m->nr; ++i) {
        double s = 0.0;
        for (int p = m->rp[i]; p < m->rp[i + 1]; ++p) s += m->v[p] * x[m->ci[p]];
        r[i] = b[i] - s;
    }
}

static double diag_of(const Mat *m, int i) {
    long p = find_pos(m, i, i);
    return p >= 0 ? m->v[p] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Input validation: the method is stated for SPD A (Section 1); the        */
/* parity contract additionally needs sorted unique columns and a bitwise   */
/* symmetric matrix with a positive stored diagonal.                        */
/* ------------------------------------------------------------------------ */
static int validate(int n, const int *rp, const int *ci, const double *v) {
    if (n <= 0 || rp[0] != 0) return OR_EMATRIX;
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return OR_EMATRIX;
        int has_diag = 0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) return OR_EMATRIX;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return OR_EMATRIX;
            if (!isfinite(v[p])) return OR_EMATRIX;
            if (ci[p] == i) { has_diag = 1; if (!(v[p] > 0.0)) return OR_EMATRIX; }
        }
        if (!has_diag) return OR_EMATRIX;
    }
    Mat a = {n, n, (int *)rp, (int *)ci, (double *)v};
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            long q = find_pos(&a, ci[p], i);
            if (q < 0 || memcmp(&v[q], &v[p], sizeof(double)) != 0) return OR_EMATRIX;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Strength of connection (Section 2, amg_setup, call to strength).  The    */
/* paper gives no formula; classical Ruge-Stueben on negative couplings:    */
/* S_ij = 1 iff j != i, mneg_i > 0 and -a_ij >= fl(theta * mneg_i), with     */
/* mneg_i = max_{k != i} (-a_ik).                                           */
/* ------------------------------------------------------------------------ */
static int strength(const Mat *a, double theta, Mat *s) {
    long nnz = a->rp[a->nr];
    if (mat_alloc(s, a->nr, a->nc, nnz)) return OR_ENOMEM;
    long q = 0;
    for (int i = 0; i < a->nr; ++i) {
        double mneg = 0.0;
        int any = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            if (a->ci[p] == i) continue;
            double t = -a->v[p];
            if (!any || t > mneg) { mneg = t; any = 1; }
        }
        s->rp[i] = (int)q;
        if (any && mneg > 0.0) {
            double thr = theta * mneg;
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
                if (a->ci[p] == i) continue;
                if (-a->v[p] >= thr) { s->ci[q] = a->ci[p]; s->v[q] = 1.0; ++q; }
            }
        }
    }
    s->rp[a->nr] = (int)q;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* C/F splitting (Section 2: interpolation first forms C and F).  Classical */
/* Ruge-Stueben first pass with a fixed tie-break; a binary max-heap on     */
/* (lambda, -index) with lazy deletion selects the next point.              */
/* ------------------------------------------------------------------------ */
typedef struct { int lam, idx; } HeapItem;
typedef struct { HeapItem *a; long n, cap; } Heap;

static int heap_better(HeapItem x, HeapItem y) {  /* x above y */
    return x.lam > y.lam || (x.lam == y.lam && x.idx < y.idx);
}
static int heap_push(Heap *h, int lam, int idx) {
    if (h->n == h->cap) {
        long nc = h->cap ? 2 * h->cap : 1024;
        HeapItem *na = (HeapItem *)realloc(h->a, sizeof(HeapItem) * (size_t)nc);
        if (!na) return OR_ENOMEM;
        h->a = na; h->cap = nc;
    }
    long i = h->n++;
    h->a[i].lam = lam; h->a[i].idx = idx;
    while (i > 0) {
        long p = (i - 1) / 2;
        if (!heap_better(h->a[i], h->a[p])) break;
        HeapItem t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t;
        i = p;
    }
    return OR_OK;
}
static HeapItem heap_pop(Heap *h) {
    HeapItem top = h->a[0];
    h->a[0] = h->a[--h->n];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1, r = l + 1, b = i;
        if (l < h->n && heap_better(h->a[l], h->a[b])) b = l;
        if (r < h->n && heap_better(h->a[r], h->a[b])) b = r;
        if (b == i) break;
        HeapItem t = h->a[i]; h->a[i] = h->a[b]; h->a[b] = t;
        i = b;
    }
    return top;
}

enum { PT_U = 0, PT_C = 1, PT_F = 2 };

static int rs_split(const Mat *s, int *cf) {
    int n = s->nr;
    Mat st;
    if (mat_transpose(s, &st)) return OR_ENOMEM;
    int *state = (int *)malloc(sizeof(int) * (size_t)n);
    int *lam = (int *)malloc(sizeof(int) * (size_t)n);
    int *newf = (int *)malloc(sizeof(int) * (size_t)n);
    Heap h = {0, 0, 0};
    if (!state || !lam || !newf) return OR_ENOMEM;
    for (int i = 0; i < n; ++i) {
        lam[i] = st.rp[i + 1] - st.rp[i];       /* #{j : S_ji = 1} */
        int srow = s->rp[i + 1] - s->rp[i];
        state[i] = (srow == 0 && lam[i] == 0) ? PT_F : PT_U;  /* isolated */
        if (state[i] == PT_U && heap_push(&h, lam[i], i)) return OR_ENOMEM;
    }
    while (h.n > 0) {
        HeapItem it = heap_pop(&h);
        int i = it.idx;
        if (state[i] != PT_U || it.lam != lam[i]) continue;   /* stale entry */
        int nnew = 0;
        int make_f = 0;
        if (lam[i] == 0) {
            for (int p = s->rp[i]; p < s->rp[i + 1]; ++p)
                if (state[s->ci[p]] == PT_C) { make_f = 1; break; }
        }
        if (make_f) {
            state[i] = PT_F;
            newf[nnew++] = i;
        } else {
            state[i] = PT_C;
            for (int p = st.rp[i]; p < st.rp[i + 1]; ++p) {   /* j with S_ji = 1 */
                int j = st.ci[p];
                if (state[j] == PT_U) { state[j] = PT_F; newf[nnew++] = j; }
            }
        }
        for (int t = 0; t < nnew; ++t) {
            int j = newf[t];
            for (int p = s->rp[j]; p < s->rp[j + 1]; ++p) {
                int k = s->ci[p];
                if (state[k] == PT_U) { lam[k]++; if (heap_push(&h, lam[k], k)) return OR_ENOMEM; }
            }
        }
        if (state[i] == PT_C) {
            for (int p = s->rp[i]; p < s->rp[i + 1]; ++p) {
                int k = s->ci[p];
                if (state[k] == PT_U) { lam[k]--; if (heap_push(&h, lam[k], k)) return OR_ENOMEM; }
            }
        }
    }
    for (int i = 0; i < n; ++i) cf[i] = (state[i] == PT_C) ? 1 : 0;
    free(state); free(lam); free(newf); free(h.a); mat_free(&st);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k >= 1 of the    */
/* stream seeded with `seed` is the published finaliser applied to          */
/* seed + k * 0x9E3779B97F4A7C15.  Counter based: any output on its own.    */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* PMIS coarsening (the parallel aggressive coarsening of De Sterck, Yang   */
/* and Heys that Section 1 cites).  Each point gets the weight              */
/* w_i = lambda_i + u_i, lambda_i = #{j : S_ji = 1} and u_i in [0, 1) the    */
/* top 53 bits of output i+1 of the SplitMix64 stream `seed`; i beats j if  */
/* w_i > w_j, or w_i == w_j and i < j.  Points no other point depends on    */
/* strongly (lambda_i = 0) are F from the start.  Then, in rounds until no  */
/* point is undecided: every undecided point that beats each undecided      */
/* point it is strongly connected to (S_ij or S_ji) becomes C, all of them  */
/* at once; after that every undecided point that depends strongly on a C   */
/* point becomes F.                                                         */
/* ------------------------------------------------------------------------ */
static int pmis_beats(const double *w, int i, int j) {
    return w[i] > w[j] || (w[i] == w[j] && i < j);
}

/* the rounds, for given weights w (lambda_i = 0 points start as F) */
static int pmis_rounds(const Mat *s, const Mat *st, const double *w, int *cf) {
    int n = s->nr;
    int *state = (int *)malloc(sizeof(int) * (size_t)n);
    int *pick = (int *)malloc(sizeof(int) * (size_t)n);
    if (!state || !pick) return OR_ENOMEM;
    int undecided = 0;
    for (int i = 0; i < n; ++i) {
        state[i] = st->rp[i + 1] == st->rp[i] ? PT_F : PT_U;
        undecided += state[i] == PT_U;
    }
    while (undecided > 0) {
        /* independent set of local maxima among the undecided points */
        for (int i = 0; i < n; ++i) {
            pick[i] = 0;
            if (state[i] != PT_U) continue;
            int best = 1;
            for (int p = s->rp[i]; p < s->rp[i + 1] && best; ++p) {
                int j = s->ci[p];
                if (state[j] == PT_U && pmis_beats(w, j, i)) best = 0;
            }
            for (int p = st->rp[i]; p < st->rp[i + 1] && best; ++p) {
                int j = st->ci[p];
                if (state[j] == PT_U && pmis_beats(w, j, i)) best = 0;
            }
            pick[i] = best;
        }
        for (int i = 0; i < n; ++i)
            if (pick[i]) { state[i] = PT_C; --undecided; }
        /* points that depend strongly on a C point become F */
        for (int j = 0; j < n; ++j) {
            if (state[j] != PT_U) continue;
            for (int p = s->rp[j]; p < s->rp[j + 1]; ++p)
                if (state[s->ci[p]] == PT_C) { state[j] = PT_F; --undecided; break; }
        }
    }
    for (int i = 0; i < n; ++i) cf[i] = (state[i] == PT_C) ? 1 : 0;
    free(state); free(pick);
    return OR_OK;
}

static int pmis_split(const Mat *s, uint64_t seed, int *cf) {
    int n = s->nr;
    Mat st;
    if (mat_transpose(s, &st)) return OR_ENOMEM;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!w) return OR_ENOMEM;
    for (int i = 0; i < n; ++i) {
        int lam = st.rp[i + 1] - st.rp[i];
        double u = (double)(splitmix64_at(seed, (uint64_t)i + 1) >> 11) * 0x1p-53;
        w[i] = (double)lam + u;
    }
    int rc = pmis_rounds(s, &st, w, cf);
    free(w); mat_free(&st);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Direct interpolation (Section 2, call to interpolation; the paper leaves */
/* the formula to its references).  C rows inject; an F row i interpolates  */
/* from its strong C neighbours P_i with w_ij = -(alpha a_ij)/d, where      */
/* alpha = (sum of negative off-diagonals)/(sum over P_i of a_ik) and       */
/* d = a_ii + (sum of positive off-diagonals); sums in ascending column.    */
/* ------------------------------------------------------------------------ */
static int direct_interp(const Mat *a, const Mat *s, const int *cf, const int *cidx,
                         int nc, Mat *P) {
    int n = a->nr;
    long cap = 0;
    for (int i = 0; i < n; ++i) cap += cf[i] ? 1 : (s->rp[i + 1] - s->rp[i]);
    if (mat_alloc(P, n, nc, cap)) return OR_ENOMEM;
    long q = 0;
    for (int i = 0; i < n; ++i) {
        P->rp[i] = (int)q;
        if (cf[i]) {
            P->ci[q] = cidx[i]; P->v[q] = 1.0; ++q;
            continue;
        }
        double sN = 0.0, sP = 0.0, d = 0.0;
        int npi = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            if (k == i) { d = a->v[p]; break; }
        }
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            if (k == i) continue;
            if (a->v[p] < 0.0) sN += a->v[p];
            else if (a->v[p] > 0.0) d += a->v[p];
        }
        /* strong C neighbours, ascending (S row is a sorted subset of A row) */
        for (int p = s->rp[i]; p < s->rp[i + 1]; ++p) {
            int j = s->ci[p];
            if (cf[j]) { sP += a->v[find_pos(a, i, j)]; ++npi; }
        }
        if (npi == 0) continue;                  /* no strong C neighbour: empty row */
        double alpha = sN / sP;
        for (int p = s->rp[i]; p < s->rp[i + 1]; ++p) {
            int j = s->ci[p];
            if (!cf[j]) continue;
            double aij = a->v[find_pos(a, i, j)];
            P->ci[q] = cidx[j];
            P->v[q] = -(alpha * aij) / d;
            ++q;
        }
    }
    P->rp[n] = (int)q;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Galerkin product A_c = P^T A P (Section 2, amg_setup).  Canonical order: */
/* T = A P row by row, T[k,J] accumulated over ascending l of A's row k;    */
/* C = P^T T, C[I,J] accumulated over ascending fine row k; the first term  */
/* of every sum is assigned.  A_c = (C + C^T)/2 entrywise, which makes the  */
/* coarse operator bitwise symmetric.  Pattern = symbolic product pattern.  */
/* ------------------------------------------------------------------------ */
static int cmp_int(const void *x, const void *y) {
    int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

/* row-by-row sparse product Z = X Y with the accumulation rule above */
static int spgemm(const Mat *X, const Mat *Y, Mat *Z) {
    int nr = X->nr, nc = Y->nc;
    int *mark = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    int *list = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    if (!mark || !acc || !list) return OR_ENOMEM;
    for (int j = 0; j < nc; ++j) mark[j] = -1;
    /* pass 1: counts */
    long total = 0;
    for (int i = 0; i < nr; ++i) {
        int cnt = 0;
        for (int p = X->rp[i]; p < X->rp[i + 1]; ++p) {
            int l = X->ci[p];
            for (int q = Y->rp[l]; q < Y->rp[l + 1]; ++q) {
                int J = Y->ci[q];
                if (mark[J] != i) { mark[J] = i; ++cnt; }
            }
        }
        total += cnt;
    }
    if (total > 2147483647L) return OR_ENOMEM;
    if (mat_alloc(Z, nr, nc, total)) return OR_ENOMEM;
    for (int j = 0; j < nc; ++j) mark[j] = -1;
    long w = 0;
    for (int i = 0; i < nr; ++i) {
        int cnt = 0;
        Z->rp[i] = (int)w;
        for (int p = X->rp[i]; p < X->rp[i + 1]; ++p) {
            int l = X->ci[p];
            double xv = X->v[p];
            for (int q = Y->rp[l]; q < Y->rp[l + 1]; ++q) {
                int J = Y->ci[q];
                double prod = xv * Y->v[q];
                if (mark[J] != i) { mark[J] = i; acc[J] = prod; list[cnt++] = J; }
                else acc[J] += prod;
            }
        }
        qsort(list, (size_t)cnt, sizeof(int), cmp_int);
        for (int t = 0; t < cnt; ++t) { Z->ci[w] = list[t]; Z->v[w] = acc[list[t]]; ++w; }
    }
    Z->rp[nr] = (int)w;
    free(mark); free(acc); free(list);
    return OR_OK;
}

static int galerkin(const Mat *A, const Mat *P, const Mat *R, Mat *Ac) {
    Mat T, C;
    int rc = spgemm(A, P, &T);              /* T = A P */
    if (rc) return rc;
    /* C = P^T T: row I of R lists the fine rows k with P_kI != 0 ascending,
       and R_Ik is the same double as P_kI. */
    rc = spgemm(R, &T, &C);
    mat_free(&T);
    if (rc) return rc;
    if (mat_copy(Ac, &C)) return OR_ENOMEM;
    for (int I = 0; I < C.nr; ++I)
        for (int p = C.rp[I]; p < C.rp[I + 1]; ++p) {
            long q = find_pos(&C, C.ci[p], I);
            if (q < 0) { mat_free(&C); return OR_EMATRIX; }
            Ac->v[p] = 0.5 * (C.v[p] + C.v[q]);
        }
    mat_free(&C);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Coarsest-level direct solve (amg_solve: solve on the coarsest level).    */
/* Dense Cholesky of \hat A_L, Gaussian elimination with partial pivoting    */
/* if a pivot is not positive.                                              */
/* ------------------------------------------------------------------------ */
static int coarse_factor(Hier *h) {
    Mat *a = &h->lv[h->nlev - 1].Ah;
    int n = a->nr;
    free(h->fac); free(h->piv); h->fac = NULL; h->piv = NULL;
    h->nL = n;
    double *d = (double *)calloc((size_t)n * n, sizeof(double));
    if (!d) return OR_ENOMEM;
    for (int i = 0; i < n; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) d[(size_t)i * n + a->ci[p]] = a->v[p];
    double *L = (double *)calloc((size_t)n * n, sizeof(double));
    if (!L) return OR_ENOMEM;
    int ok = 1;
    for (int j = 0; j < n && ok; ++j) {
        double s = d[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) { ok = 0; break; }
        double ljj = sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = d[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    if (ok) { h->fac = L; free(d); return OR_OK; }
    free(L);
    int *piv = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!piv) return OR_ENOMEM;
    for (int k = 0; k < n; ++k) {
        int pr = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(d[(size_t)i * n + k]) > fabs(d[(size_t)pr * n + k])) pr = i;
        piv[k] = pr;
        if (d[(size_t)pr * n + k] == 0.0) { free(piv); free(d); return OR_EMATRIX; }
        if (pr != k)
            for (int j = 0; j < n; ++j) {
                double t = d[(size_t)k * n + j]; d[(size_t)k * n + j] = d[(size_t)pr * n + j]; d[(size_t)pr * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            d[(size_t)i * n + k] /= d[(size_t)k * n + k];
            for (int j = k + 1; j < n; ++j) d[(size_t)i * n + j] -= d[(size_t)i * n + k] * d[(size_t)k * n + j];
        }
    }
    h->fac = d; h->piv = piv;
    return OR_OK;
}

static void coarse_solve(const Hier *h, const double *b, double *x) {
    int n = h->nL;
    const double *F = h->fac;
    for (int i = 0; i < n; ++i) x[i] = b[i];
    if (!h->piv) {                         /* L L^T x = b */
        for (int i = 0; i < n; ++i) {
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= F[(size_t)i * n + k] * x[k];
            x[i] = s / F[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int k = i + 1; k < n; ++k) s -= F[(size_t)k * n + i] * x[k];
            x[i] = s / F[(size_t)i * n + i];
        }
    } else {                               /* P A = L U */
        for (int k = 0; k < n; ++k) {
            int p = h->piv[k];
            if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
        }
        for (int i = 0; i < n; ++i) {
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= F[(size_t)i * n + k] * x[k];
            x[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int k = i + 1; k < n; ++k) s -= F[(size_t)i * n + k] * x[k];
            x[i] = s / F[(size_t)i * n + i];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Setup (Section 2 amg_setup with nongalerkin = False, as called by        */
/* Section 3 sparse_hybrid_setup).  Coarsen while n_l > max_size and fewer  */
/* than max_levels levels exist; stop if the split yields no C point or     */
/* only C points.                                                           */
/* ------------------------------------------------------------------------ */
static int build_M(Hier *h, int l, const Mat *fine_op);
static int sparsify_level(Hier *h, int l, double gamma);
static int nongalerkin_level(Hier *h, int l, double gamma);

void or_free(Hier *h);

/* ng_gamma (nullable, ng_count entries): the method of non-Galerkin coarse
   grids (Section 2.1; amg_setup with its optional sparsify): right after its
   Galerkin product, A_{l+1} is sparsified with tolerance ng_gamma[l+1] and
   replaces the product, so the next level is built from it.
   coarsen: 0 = Ruge-Stueben first pass, 1 = PMIS with the weights of level l
   drawn from the SplitMix64 stream seed + l. */
int or_setup(int n, const int *rp, const int *ci, const double *v, double theta,
             int max_coarse, int max_levels, double omega, int nu_pre, int nu_post,
             const double *ng_gamma, int ng_count, int coarsen, uint64_t seed, Hier **out) {
    *out = NULL;
    if (n <= 0 || !rp || !ci || !v || max_levels < 1 || max_coarse < 1 || coarsen < 0 || coarsen > 1)
        return OR_EINVAL;
    int rc = validate(n, rp, ci, v);
    if (rc) return rc;
    Hier *h = (Hier *)calloc(1, sizeof(Hier));
    h->lv = (Level *)calloc((size_t)max_levels, sizeof(Level));
    h->omega = omega; h->nu_pre = nu_pre; h->nu_post = nu_post;
    h->relax = 0; h->gs_block = 1;
    h->lumping = 0; h->theta = theta;
    Mat A0 = {n, n, (int *)rp, (int *)ci, (double *)v};
    if (mat_copy(&h->lv[0].A, &A0)) return OR_ENOMEM;
    int L = 0;
    while (h->lv[L].A.nr > max_coarse && L < max_levels - 1) {
        Level *cur = &h->lv[L];
        int nl = cur->A.nr;
        if ((rc = strength(&cur->A, theta, &cur->S))) return rc;
        cur->cf = (int *)malloc(sizeof(int) * (size_t)nl);
        cur->cidx = (int *)malloc(sizeof(int) * (size_t)nl);
        rc = coarsen == 1 ? pmis_split(&cur->S, seed + (uint64_t)L, cur->cf) : rs_split(&cur->S, cur->cf);
        if (rc) return rc;
        int nc = 0;
        for (int i = 0; i < nl; ++i) cur->cidx[i] = cur->cf[i] ? nc++ : -1;
        if (nc == 0 || nc == nl) {
            mat_free(&cur->S); free(cur->cf); free(cur->cidx);
            cur->cf = cur->cidx = NULL;
            break;
        }
        if ((rc = direct_interp(&cur->A, &cur->S, cur->cf, cur->cidx, nc, &cur->P))) return rc;
        if ((rc = mat_transpose(&cur->P, &cur->R))) return rc;
        if ((rc = galerkin(&cur->A, &cur->P, &cur->R, &h->lv[L + 1].A))) return rc;
        if (ng_gamma) {
            double g = L + 1 < ng_count ? ng_gamma[L + 1] : 0.0;
            if (!(g >= 0.0 && g <= 1.0)) return OR_EINVAL;
            if (g > 0.0 && (rc = nongalerkin_level(h, L + 1, g))) return rc;
        }
        ++L;
    }
    h->nlev = L + 1;
    for (int l = 0; l < h->nlev; ++l) {
        Level *lv = &h->lv[l];
        if (mat_copy(&lv->Ah, &lv->A)) return OR_ENOMEM;
        lv->gamma = 0.0;
        long nnz = lv->A.rp[lv->A.nr];
        lv->keep = (unsigned char *)malloc((size_t)(nnz > 0 ? nnz : 1));
        memset(lv->keep, 1, (size_t)(nnz > 0 ? nnz : 1));
        if (l >= 1 && (rc = build_M(h, l, &h->lv[l - 1].A))) return rc;
    }
    h->b = (double **)calloc((size_t)h->nlev, sizeof(double *));
    h->x = (double **)calloc((size_t)h->nlev, sizeof(double *));
    h->r = (double **)calloc((size_t)h->nlev, sizeof(double *));
    for (int l = 0; l < h->nlev; ++l) {
        int nl = h->lv[l].A.nr;
        h->b[l] = (double *)calloc((size_t)nl, sizeof(double));
        h->x[l] = (double *)calloc((size_t)nl, sizeof(double));
        h->r[l] = (double *)calloc((size_t)nl, sizeof(double));
    }
    if ((rc = coarse_factor(h))) return rc;
    *out = h;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Minimal sparsity pattern (Algorithm 3, first line after form-injection): */
/* M = edges(Phat^T A P + P^T A Phat) with Phat the injection onto the C     */
/* points and A the finer operator: the Galerkin A_{l-1} for Sparse Galerkin */
/* and the sparsified \hat A_{l-1} for Hybrid Galerkin (Section 3, the two  */
/* sparsify calls of sparse_hybrid_setup).  Row I of Phat^T A P is the union */
/* over l' in row c(I) of A of the columns of row l' of P; P^T A Phat is its */
/* transpose.  Structural pattern, stored as one flag per nonzero of A_l.   */
/* ------------------------------------------------------------------------ */
static int build_M(Hier *h, int l, const Mat *fine_op) {
    Level *fine = &h->lv[l - 1];
    Level *lv = &h->lv[l];
    long nnz = lv->A.rp[lv->A.nr];
    free(lv->inM);
    lv->inM = (unsigned char *)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
    if (!lv->inM) return OR_ENOMEM;
    for (int f = 0; f < fine_op->nr; ++f) {
        if (!fine->cf[f]) continue;
        int I = fine->cidx[f];
        for (int p = fine_op->rp[f]; p < fine_op->rp[f + 1]; ++p) {
            int lp = fine_op->ci[p];
            for (int q = fine->P.rp[lp]; q < fine->P.rp[lp + 1]; ++q) {
                int J = fine->P.ci[q];
                long a = find_pos(&lv->A, I, J);
                long b = find_pos(&lv->A, J, I);
                if (a < 0 || b < 0) return OR_EMATRIX;
                lv->inM[a] = 1;
                lv->inM[b] = 1;
            }
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* sparsify with diagonal lumping (Algorithm 3 keep set + Algorithm 3b).    */
/* m_i = max_{k != i} |a_ik|.  (i,j) enters N when (i,j) is in M or          */
/* |a_ij| >= gamma m_i, and N is closed under transposition, so with A and M */
/* symmetric: keep(i,j) = i == j or M_ij or |a_ij| >= fl(gamma m_i) or       */
/* |a_ij| >= fl(gamma m_j).  Kept entries are copied; dropped ones are       */
/* added to the diagonal: \hat a_ii = a_ii + sum of dropped a_ij (ascending).*/
/* The ismax branch of Algorithm 3b cannot fire for gamma <= 1 because the   */
/* row maximum always passes the gamma test.                                */
/* ------------------------------------------------------------------------ */
static void row_max(const Mat *a, double *m) {
    for (int i = 0; i < a->nr; ++i) {
        double mx = 0.0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
            if (a->ci[p] != i && fabs(a->v[p]) > mx) mx = fabs(a->v[p]);
        m[i] = mx;
    }
}

/* ------------------------------------------------------------------------ */
/* Strong-neighbour lumping (Algorithm 3, second loop: the sparsification   */
/* of the method of non-Galerkin coarse grids that Section 2.1 starts from; */
/* Algorithm 3b replaces it by diagonal lumping).  Readings: S is the       */
/* classical strength of the operator being sparsified (setup theta), with  */
/* |S_jm| = |a_jm| for its strong entries; every kept entry starts at its   */
/* value in A (order-free, where the printed loop would overwrite shares    */
/* already added); a dropped (i,j) is shared among                          */
/* W = {m : S_jm strong, (i,m) kept} in proportion |a_jm| / sum_W |a_jk|     */
/* (the sum in ascending k): each share c is added to (i,m) and (m,i) and   */
/* subtracted from (m,m), or added once to (i,i) when m = i; with W empty    */
/* the dropped entry goes to the diagonal, as in Algorithm 3b.  Dropped      */
/* entries are visited in row-major order, so every entry adds its shares in */
/* ascending order of the dropped entry they come from.  ah: the kept        */
/* pattern holding the values of a.                                         */
/* ------------------------------------------------------------------------ */
static int strong_lump(const Mat *a, const unsigned char *keep, double theta, Mat *ah) {
    int n = a->nr;
    double *thr = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!thr) return OR_ENOMEM;
    for (int j = 0; j < n; ++j) {
        double big = 0.0;
        for (int p = a->rp[j]; p < a->rp[j + 1]; ++p)
            if (a->ci[p] != j && -a->v[p] > big) big = -a->v[p];
        thr[j] = big > 0.0 ? theta * big : -1.0;   /* -1: no strong entry */
    }
#define STRONG(j, r) (a->ci[r] != (j) && thr[j] > 0.0 && -a->v[r] >= thr[j])
#define KEPT(i, m) (find_pos(a, (i), (m)) >= 0 && keep[find_pos(a, (i), (m))])
    for (int i = 0; i < n; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int j = a->ci[p];
            if (j == i || keep[p]) continue;
            double aij = a->v[p], den = 0.0;
            int cnt = 0;
            for (int r = a->rp[j]; r < a->rp[j + 1]; ++r)
                if (STRONG(j, r) && KEPT(i, a->ci[r])) { den = den + fabs(a->v[r]); ++cnt; }
            if (cnt == 0) {
                ah->v[find_pos(ah, i, i)] += aij;
                continue;
            }
            for (int r = a->rp[j]; r < a->rp[j + 1]; ++r) {
                if (!(STRONG(j, r) && KEPT(i, a->ci[r]))) continue;
                int m = a->ci[r];
                double c = (fabs(a->v[r]) / den) * aij;
                if (m == i) {
                    ah->v[find_pos(ah, i, i)] += c;
                } else {
                    ah->v[find_pos(ah, i, m)] += c;
                    ah->v[find_pos(ah, m, i)] += c;
                    ah->v[find_pos(ah, m, m)] -= c;
                }
            }
        }
#undef STRONG
#undef KEPT
    free(thr);
    return OR_OK;
}

/* lumping of later sparsify calls: 0 = diagonal (Algorithm 3b), 1 = strong
   neighbours (Algorithm 3, second loop) */
int or_set_lumping(Hier *h, int mode) {
    if (mode != 0 && mode != 1) return OR_EINVAL;
    h->lumping = mode;
    return OR_OK;
}

/* strong-neighbour lumping of a plain CSR matrix with given keep flags:
   out receives the values of the kept pattern (row by row, kept entries in
   column order) */
int or_strong_lump_csr(int n, const int *rp, const int *ci, const double *v, const unsigned char *keep,
                       double theta, double *out) {
    Mat a = {n, n, (int *)rp, (int *)ci, (double *)v};
    long kept = 0;
    for (long p = 0; p < rp[n]; ++p) kept += keep[p] != 0;
    Mat ah;
    if (mat_alloc(&ah, n, n, kept)) return OR_ENOMEM;
    long q = 0;
    for (int i = 0; i < n; ++i) {
        ah.rp[i] = (int)q;
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (keep[p]) { ah.ci[q] = ci[p]; ah.v[q] = v[p]; ++q; }
    }
    ah.rp[n] = (int)q;
    int rc = strong_lump(&a, keep, theta, &ah);
    if (rc == OR_OK) memcpy(out, ah.v, sizeof(double) * (size_t)kept);
    mat_free(&ah);
    return rc;
}

static int sparsify_level(Hier *h, int l, double gamma) {
    Level *lv = &h->lv[l];
    Mat *a = &lv->A;
    int n = a->nr;
    long nnz = a->rp[n];
    free(lv->rowmax);
    lv->rowmax = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!lv->rowmax) return OR_ENOMEM;
    row_max(a, lv->rowmax);
    long kept = 0;
    for (int i = 0; i < n; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int j = a->ci[p];
            double av = fabs(a->v[p]);
            int k = (j == i) || lv->inM[p] || av >= gamma * lv->rowmax[i] || av >= gamma * lv->rowmax[j];
            lv->keep[p] = (unsigned char)k;
            kept += k;
        }
    Mat nh;
    if (mat_alloc(&nh, n, n, kept)) return OR_ENOMEM;
    long q = 0;
    for (int i = 0; i < n; ++i) {
        nh.rp[i] = (int)q;
        double d = 0.0;
        long dpos = -1;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
            if (a->ci[p] == i) d = a->v[p];
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            if (a->ci[p] != i && !lv->keep[p]) d += a->v[p];
        }
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            if (!lv->keep[p]) continue;
            nh.ci[q] = a->ci[p];
            if (a->ci[p] == i) dpos = q;
            nh.v[q] = a->v[p];
            ++q;
        }
        if (dpos >= 0 && h->lumping == 0) nh.v[dpos] = d;
    }
    nh.rp[n] = (int)q;
    if (h->lumping == 1) {
        int rc = strong_lump(a, lv->keep, h->theta, &nh);
        if (rc) return rc;
    }
    mat_free(&lv->Ah);
    lv->Ah = nh;
    lv->gamma = gamma;
    return OR_OK;
}

/* Non-Galerkin coarse grid: sparsify the product A_l just formed (minimal
   pattern from the hierarchy's finer operator A_{l-1}, keep set of Algorithm
   3, diagonal lumping of Algorithm 3b) and let the result be A_l itself. */
static int nongalerkin_level(Hier *h, int l, double gamma) {
    Level *lv = &h->lv[l];
    long nnz = lv->A.rp[lv->A.nr];
    int rc = build_M(h, l, &h->lv[l - 1].A);
    if (rc) return rc;
    lv->keep = (unsigned char *)malloc((size_t)(nnz > 0 ? nnz : 1));
    if (!lv->keep) return OR_ENOMEM;
    if ((rc = sparsify_level(h, l, gamma))) return rc;
    mat_free(&lv->A);
    lv->A = lv->Ah;
    memset(&lv->Ah, 0, sizeof(Mat));
    free(lv->keep); free(lv->inM); free(lv->rowmax);
    lv->keep = NULL; lv->inM = NULL; lv->rowmax = NULL;
    lv->gamma = 0.0;
    return OR_OK;
}

/* gamma[l] for l = 0 .. nlev-1; gamma[0] is ignored (A_0 is never sparsified,
   Section 3: sparse_hybrid_setup starts at the first coarse operator). */
int or_sparsify(Hier *h, const double *gamma) {
    for (int l = 1; l < h->nlev; ++l)
        if (!(gamma[l] >= 0.0 && gamma[l] <= 1.0)) return OR_EINVAL;
    for (int l = 1; l < h->nlev; ++l) {
        int rc = 0;
        /* Hybrid Galerkin: M_l from \hat A_{l-1}, which the previous pass of
           this loop has just produced (finest level first) */
        if (h->hybrid && (rc = build_M(h, l, &h->lv[l - 1].Ah))) return rc;
        if ((rc = sparsify_level(h, l, gamma[l]))) return rc;
    }
    return coarse_factor(h);
}

/* Selects Sparse (0) or Hybrid (1) Galerkin for later sparsify and
   reintroduce calls and rebuilds every M_l from the current operators. */
int or_set_method(Hier *h, int hybrid) {
    if (hybrid != 0 && hybrid != 1) return OR_EINVAL;
    h->hybrid = hybrid;
    for (int l = 1; l < h->nlev; ++l) {
        int rc = build_M(h, l, hybrid ? &h->lv[l - 1].Ah : &h->lv[l - 1].A);
        if (rc) return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Reintroduction (Section 6, adaptive_solve, and the Example there):       */
/* start at the finest coarse level with gamma > 0, lower gamma on s levels */
/* (gamma/10, or 0 when gamma/10 < gamma_min) and re-sparsify those levels  */
/* from the retained Galerkin operators.                                    */
/* ------------------------------------------------------------------------ */
int or_reintroduce(Hier *h, int s, double gamma_min, int *first_changed) {
    int ls = -1;
    for (int l = 1; l < h->nlev; ++l)
        if (h->lv[l].gamma > 0.0) { ls = l; break; }
    if (first_changed) *first_changed = ls;
    if (ls < 0) return OR_NOTHING;
    for (int l = ls; l < h->nlev; ++l) {
        int rc = 0;
        double g = h->lv[l].gamma;
        if (l < ls + s) {
            g = g / 10.0;
            if (!(g >= gamma_min)) g = 0.0;
        } else if (!h->hybrid || g == 0.0) {
            continue;
        }
        /* Hybrid Galerkin: a coarser level's M depends on the operator just
           changed, so every coarser sparsified level is redone at its gamma */
        if (h->hybrid && (rc = build_M(h, l, &h->lv[l - 1].Ah))) return rc;
        if ((rc = sparsify_level(h, l, g))) return rc;
    }
    return coarse_factor(h);
}

/* ------------------------------------------------------------------------ */
/* V-cycle (Section 2, amg_solve) with weighted Jacobi relaxation           */
/*   x <- x + omega (b - \hat A x) / diag(\hat A).                            */
/* Coarse initial guesses are zero and b_{l+1} = P_l^T (b_l - \hat A_l x_l).  */
/* ------------------------------------------------------------------------ */
static void jacobi(const Mat *a, const double *b, double *x, double *tmp, double omega) {
    residual(a, b, x, tmp);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int i = 0; i < a->nr; ++i) x[i] = x[i] + omega * tmp[i] / diag_of(a, i);
}

/* ------------------------------------------------------------------------ */
/* Hybrid Gauss-Seidel (the relaxation of the paper's experiments, Section  */
/* 5, there with one block per process): the rows are split into            */
/* contiguous blocks of `block` rows; inside a block the sweep is           */
/* Gauss-Seidel (a row uses the new values of the rows of its block visited */
/* before it), across blocks it is Jacobi (old values).  Forward sweeps     */
/* visit a block's rows in ascending order, backward sweeps in descending   */
/* order.  Row i: x_i = (b_i - sum_{j != i} a_ij y_j) / a_ii, the terms     */
/* subtracted in ascending column order.                                    */
/* ------------------------------------------------------------------------ */
static void hybrid_gs(const Mat *a, const double *b, const double *xold, double *xnew, int block,
                      int forward) {
    int n = a->nr;
    for (int r0 = 0; r0 < n; r0 += block) {
        int r1 = r0 + block < n ? r0 + block : n;
        for (int t = 0; t < r1 - r0; ++t) {
            int i = forward ? r0 + t : r1 - 1 - t;
            double s = b[i], d = 0.0;
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
                int j = a->ci[p];
                if (j == i) { d = a->v[p]; continue; }
                int visited = j >= r0 && j < r1 && (forward ? j < i : j > i);
                s = s - a->v[p] * (visited ? xnew[j] : xold[j]);
            }
            xnew[i] = s / d;
        }
    }
}

/* one hybrid Gauss-Seidel sweep on a plain CSR matrix (no hierarchy) */
int or_gs_sweep(int n, const int *rp, const int *ci, const double *v, const double *b, const double *xold,
                double *xnew, int block, int forward) {
    if (n <= 0 || block < 1) return OR_EINVAL;
    Mat a = {n, n, (int *)rp, (int *)ci, (double *)v};
    hybrid_gs(&a, b, xold, xnew, block, forward);
    return OR_OK;
}

/* relax: 0 = weighted Jacobi, 1 = hybrid symmetric Gauss-Seidel with blocks
   of `block` rows (V-cycles sweep forward before the coarse correction and
   backward after it, so the cycle stays a symmetric preconditioner) */
int or_set_relaxation(Hier *h, int relax, int block) {
    if ((relax != 0 && relax != 1) || block < 1) return OR_EINVAL;
    h->relax = relax;
    h->gs_block = block;
    return OR_OK;
}

/* nu sweeps of the configured relaxation on level l; tmp: n_l scratch */
static void relax(Hier *h, const Mat *a, const double *b, double *x, double *tmp, int forward, int nu) {
    for (int s = 0; s < nu; ++s) {
        if (h->relax == 1) {
            memcpy(tmp, x, sizeof(double) * (size_t)a->nr);
            hybrid_gs(a, b, tmp, x, h->gs_block, forward);
        } else {
            jacobi(a, b, x, tmp, h->omega);
        }
    }
}

static void vcycle(Hier *h, const double *b0, double *x0) {
    int L = h->nlev - 1;
    memcpy(h->b[0], b0, sizeof(double) * (size_t)h->lv[0].A.nr);
    memcpy(h->x[0], x0, sizeof(double) * (size_t)h->lv[0].A.nr);
    for (int l = 0; l < L; ++l) {
        Level *lv = &h->lv[l];
        relax(h, &lv->Ah, h->b[l], h->x[l], h->r[l], 1, h->nu_pre);
        residual(&lv->Ah, h->b[l], h->x[l], h->r[l]);
        spmv(&lv->R, h->r[l], h->b[l + 1]);
        memset(h->x[l + 1], 0, sizeof(double) * (size_t)h->lv[l + 1].A.nr);
    }
    coarse_solve(h, h->b[L], h->x[L]);
    for (int l = L - 1; l >= 0; --l) {
        Level *lv = &h->lv[l];
        spmv(&lv->P, h->x[l + 1], h->r[l]);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int i = 0; i < lv->A.nr; ++i) h->x[l][i] += h->r[l][i];
        relax(h, &lv->Ah, h->b[l], h->x[l], h->r[l], 0, h->nu_post);
    }
    memcpy(x0, h->x[0], sizeof(double) * (size_t)h->lv[0].A.nr);
}

int or_vcycle(Hier *h, const double *b, double *x) { vcycle(h, b, x); return OR_OK; }

/* ------------------------------------------------------------------------ */
/* Outer iteration: stationary AMG or AMG-preconditioned CG (Hestenes-       */
/* Stiefel), optionally with the adaptive window of Section 6:              */
/*  * every k iterations the true residual is formed and the window factor  */
/*    rho = (|r_end| / |r_start|)^(1/k) is measured;                         */
/*  * if rho > rho_max and a coarse level still drops entries, reintroduce  */
/*    on s levels; if the window diverged (|r_end| > |r_start|) x reverts to */
/*    its value at the window start; CG restarts with the new hierarchy.    */
/* Converged iff |r| <= tol |r_0| (2-norm, r_0 = b - A x_0).  For CG the     */
/* test uses the recursively updated residual.                              */
/* ------------------------------------------------------------------------ */
#define OR_STATIONARY 0
#define OR_PCG 1

int or_solve(Hier *h, const double *b, double *x, int method, double tol, int maxit,
             int adaptive, int k, int s, double rho_max, double gamma_min,
             SolveInfo *info, double *hist) {
    int n = h->lv[0].A.nr;
    const Mat *A = &h->lv[0].A;
    SolveInfo in = {0, 0, 0, 0, 0.0, 0.0};
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *xw = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q || !xw) return OR_ENOMEM;
    if (adaptive && k < 1) return OR_EINVAL;
    int rc = OR_ENOTCONV;
    residual(A, b, x, r);
    double nr0 = sqrt(dot(n, r, r));
    double nr = nr0;
    if (hist) hist[0] = nr0;
    if (!isfinite(nr0)) { rc = OR_EBREAK; goto done; }
    if (nr0 == 0.0) { in.converged = 1; rc = OR_OK; goto done; }
    memcpy(xw, x, sizeof(double) * (size_t)n);
    double nws = nr0;        /* true residual norm at the window start */
    int inwin = 0;
    double rz = 0.0;
    if (method == OR_PCG) {
        memset(z, 0, sizeof(double) * (size_t)n);
        vcycle(h, r, z);
        memcpy(p, z, sizeof(double) * (size_t)n);
        rz = dot(n, r, z);
    }
    while (in.iters < maxit) {
        if (method == OR_PCG) {
            spmv(A, p, q);
            double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { rc = OR_EBREAK; break; }
            double alpha = rz / pq;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
            for (int i = 0; i < n; ++i) {
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * q[i];
            }
        } else {
            vcycle(h, b, x);
            residual(A, b, x, r);
        }
        in.iters++;
        inwin++;
        nr = sqrt(dot(n, r, r));
        if (hist) hist[in.iters] = nr;
        if (!isfinite(nr)) { rc = OR_EBREAK; break; }
        if (nr <= tol * nr0) { in.converged = 1; rc = OR_OK; break; }
        int restart = 0;
        if (adaptive && inwin == k) {
            double *rt = q;                  /* q is free until the next A p */
            residual(A, b, x, rt);
            double nrt = sqrt(dot(n, rt, rt));
            double rho = pow(nrt / nws, 1.0 / (double)k);
            int any = 0;
            for (int l = 1; l < h->nlev; ++l) if (h->lv[l].gamma > 0.0) any = 1;
            if (rho > rho_max && any) {
                int first;
                int rr = or_reintroduce(h, s, gamma_min, &first);
                if (rr < 0) { rc = rr; break; }
                in.reintroductions++;
                if (nrt > nws) {                /* window diverged: revert x */
                    memcpy(x, xw, sizeof(double) * (size_t)n);
                    residual(A, b, x, r);
                    nrt = sqrt(dot(n, r, r));
                } else {
                    memcpy(r, rt, sizeof(double) * (size_t)n);
                }
                restart = 1;
            }
            memcpy(xw, x, sizeof(double) * (size_t)n);
            nws = nrt;
            inwin = 0;
        }
        if (method == OR_PCG) {
            memset(z, 0, sizeof(double) * (size_t)n);
            vcycle(h, r, z);
            double rz_new = dot(n, r, z);
            if (restart) {
                in.restarts++;
                memcpy(p, z, sizeof(double) * (size_t)n);
            } else {
                double beta = rz_new / rz;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
                for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            }
            rz = rz_new;
        } else if (restart) {
            in.restarts++;
        }
    }
done:
    residual(A, b, x, r);
    in.relres = nr0 > 0.0 ? sqrt(dot(n, r, r)) / nr0 : 0.0;
    in.rho_avg = (in.iters > 0 && in.relres > 0.0) ? pow(in.relres, 1.0 / in.iters) : 0.0;
    if (info) *info = in;
    free(r); free(z); free(p); free(q); free(xw);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Accessors for the tests                                                  */
/* ------------------------------------------------------------------------ */
int or_num_levels(const Hier *h) { return h->nlev; }

/* sizes: n, nnz(A), nnz(Ahat), nnz(P), n_coarse */
void or_level_sizes(const Hier *h, int l, long *out5) {
    const Level *lv = &h->lv[l];
    out5[0] = lv->A.nr;
    out5[1] = lv->A.rp[lv->A.nr];
    out5[2] = lv->Ah.rp[lv->Ah.nr];
    out5[3] = lv->P.rp ? lv->P.rp[lv->P.nr] : 0;
    out5[4] = lv->P.rp ? lv->P.nc : 0;
}

double or_level_gamma(const Hier *h, int l) { return h->lv[l].gamma; }

/* which: 0 = A, 1 = Ahat, 2 = P, 3 = R, 4 = S */
int or_export(const Hier *h, int l, int which, int *rp, int *ci, double *v) {
    const Level *lv = &h->lv[l];
    const Mat *m = which == 0 ? &lv->A : which == 1 ? &lv->Ah : which == 2 ? &lv->P
                 : which == 3 ? &lv->R : &lv->S;
    if (!m->rp) return OR_EINVAL;
    long nnz = m->rp[m->nr];
    if (rp) memcpy(rp, m->rp, sizeof(int) * ((size_t)m->nr + 1));
    if (ci) memcpy(ci, m->ci, sizeof(int) * (size_t)nnz);
    if (v) memcpy(v, m->v, sizeof(double) * (size_t)nnz);
    return OR_OK;
}

/* PMIS rounds on the strength pattern (rp, ci) of n points with the given
   weights instead of lambda + u (lets a test choose weights that tie) */
int or_pmis_rounds(int n, const int *rp, const int *ci, const double *w, int *cf) {
    Mat s = {n, n, (int *)rp, (int *)ci, NULL}, st;
    if (mat_transpose(&s, &st)) return OR_ENOMEM;
    int rc = pmis_rounds(&s, &st, w, cf);
    mat_free(&st);
    return rc;
}

/* output k >= 1 of the SplitMix64 stream `seed` (the PMIS weights' source) */
uint64_t or_splitmix64(uint64_t seed, uint64_t k) { return splitmix64_at(seed, k); }

/* which: 0 = inM, 1 = keep (per nonzero of A_l) */
int or_export_mask(const Hier *h, int l, int which, unsigned char *out) {
    const Level *lv = &h->lv[l];
    long nnz = lv->A.rp[lv->A.nr];
    const unsigned char *m = which == 0 ? lv->inM : lv->keep;
    if (!m) return OR_EINVAL;
    memcpy(out, m, (size_t)nnz);
    return OR_OK;
}

int or_export_cf(const Hier *h, int l, int *cf) {
    const Level *lv = &h->lv[l];
    if (!lv->cf) return OR_EINVAL;
    memcpy(cf, lv->cf, sizeof(int) * (size_t)lv->A.nr);
    return OR_OK;
}

int or_export_rowmax(const Hier *h, int l, double *m) {
    const Level *lv = &h->lv[l];
    if (lv->rowmax) { memcpy(m, lv->rowmax, sizeof(double) * (size_t)lv->A.nr); return OR_OK; }
    row_max(&lv->A, m);
    return OR_OK;
}

/* Single steps of the V-cycle on level l, for per-kernel parity checks.
   op 0: out = b - Ahat_l x          (residual)
   op 1: out = one Jacobi sweep of x  (x not modified)
   op 2: out = R_l in                 (restriction, out has n_{l+1})
   op 3: out = x + P_l in             (interpolate and correct; x has n_l)
   op 4: out = Ahat_L^{-1} b          (coarsest solve, l ignored)
   op 5: out = A_l x                  (Galerkin operator product)
   op 6: out = Ahat_l x                                                     */
int or_level_op(Hier *h, int l, int op, const double *in, const double *x, double *out) {
    Level *lv = &h->lv[l];
    int n = lv->A.nr;
    switch (op) {
    case 0: residual(&lv->Ah, in, x, out); return OR_OK;
    case 1: {
        double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
        memcpy(out, x, sizeof(double) * (size_t)n);
        jacobi(&lv->Ah, in, out, tmp, h->omega);
        free(tmp);
        return OR_OK;
    }
    case 2: if (!lv->R.rp) return OR_EINVAL; spmv(&lv->R, in, out); return OR_OK;
    case 3: {
        if (!lv->P.rp) return OR_EINVAL;
        spmv(&lv->P, in, out);
        for (int i = 0; i < n; ++i) out[i] = x[i] + out[i];
        return OR_OK;
    }
    case 4: coarse_solve(h, in, out); return OR_OK;
    case 5: spmv(&lv->A, x, out); return OR_OK;
    case 6: spmv(&lv->Ah, x, out); return OR_OK;
    case 7: case 8: hybrid_gs(&lv->Ah, in, x, out, h->gs_block, op == 7); return OR_OK;
    }
    return OR_EINVAL;
}

void or_free(Hier *h) {
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) {
        Level *lv = &h->lv[l];
        mat_free(&lv->A); mat_free(&lv->Ah); mat_free(&lv->P); mat_free(&lv->R); mat_free(&lv->S);
        free(lv->cf); free(lv->cidx); free(lv->inM); free(lv->keep); free(lv->rowmax);
        if (h->b) { free(h->b[l]); free(h->x[l]); free(h->r[l]); }
    }
    free(h->b); free(h->x); free(h->r);
    free(h->lv); free(h->fac); free(h->piv);
    free(h);
}
