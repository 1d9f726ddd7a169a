/*
 * Exercise of the C oracle's entry points for the host sanitizer run
 * (AddressSanitizer + UndefinedBehaviorSanitizer): setup with both
 * coarsenings and with non-Galerkin coarse grids, sparsification under both
 * lumpings and both methods, reintroduction, every export, the level
 * operations and solves with both relaxations.  Test infrastructure: built
 * and run by tests/test_sanitizers_cpu.py; exits non-zero on a failed status.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct Hier Hier;
int or_setup(int n, const int *rp, const int *ci, const double *v, double theta, int max_coarse, int max_levels,
             double omega, int nu_pre, int nu_post, const double *ng_gamma, int ng_count, int coarsen,
             uint64_t seed, Hier **out);
void or_free(Hier *h);
int or_sparsify(Hier *h, const double *gamma);
int or_set_method(Hier *h, int hybrid);
int or_set_lumping(Hier *h, int mode);
int or_set_relaxation(Hier *h, int relax, int block);
int or_reintroduce(Hier *h, int s, double gamma_min, int *first_changed);
int or_vcycle(Hier *h, const double *b, double *x);
int or_num_levels(const Hier *h);
void or_level_sizes(const Hier *h, int l, long *out5);
int or_export(const Hier *h, int l, int which, int *rp, int *ci, double *v);
int or_export_mask(const Hier *h, int l, int which, unsigned char *out);
int or_export_cf(const Hier *h, int l, int *cf);
int or_export_rowmax(const Hier *h, int l, double *m);
int or_level_op(Hier *h, int l, int op, const double *in, const double *x, double *out);
typedef struct { int iters, restarts, reintroductions, converged; double relres, rho_avg; } SolveInfo;
int or_solve(Hier *h, const double *b, double *x, int method, double tol, int maxit, int adaptive, int k, int s,
             double rho_max, double gamma_min, SolveInfo *info, double *hist);

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); exit(1); } } while (0)

/* 2D (nz = 1) or 3D Poisson on an nx x ny x nz grid, Dirichlet boundaries eliminated */
static int poisson(int nx, int ny, int nz, int **rp, int **ci, double **v) {
    int n = nx * ny * nz, q = 0;
    *rp = malloc(sizeof(int) * (n + 1));
    *ci = malloc(sizeof(int) * 7 * n);
    *v = malloc(sizeof(double) * 7 * n);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int r = (k * ny + j) * nx + i;
                (*rp)[r] = q;
                int nb[7] = {r - nx * ny, r - nx, r - 1, r, r + 1, r + nx, r + nx * ny};
                int ok[7] = {k > 0, j > 0, i > 0, 1, i < nx - 1, j < ny - 1, k < nz - 1};
                for (int t = 0; t < 7; ++t) {
                    if (!ok[t]) continue;
                    (*ci)[q] = nb[t];
                    (*v)[q] = nb[t] == r ? (nz > 1 ? 6.0 : 4.0) : -1.0;
                    ++q;
                }
            }
    (*rp)[n] = q;
    return n;
}

static void rhs(int n, double *b) {
    uint64_t z = 12345;
    for (int i = 0; i < n; ++i) {
        z = z * 6364136223846793005ull + 1442695040888963407ull;
        b[i] = (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    }
}

static void exercise(Hier *h, int n) {
    int L = or_num_levels(h);
    CHECK(L >= 2);
    double *gam = calloc(L, sizeof(double));
    for (int l = 2; l < L; ++l) gam[l] = 1.0;
    CHECK(or_sparsify(h, gam) == 0);
    for (int l = 0; l < L; ++l) {
        long s[5];
        or_level_sizes(h, l, s);
        int nl = (int)s[0];
        int *rp = malloc(sizeof(int) * (nl + 1));
        int *ci = malloc(sizeof(int) * (s[1] > 0 ? s[1] : 1));
        double *v = malloc(sizeof(double) * (s[1] > 0 ? s[1] : 1));
        CHECK(or_export(h, l, 0, rp, ci, v) == 0);
        CHECK(or_export(h, l, 1, rp, ci, v) == 0);
        if (l + 1 < L) {
            int *rp2 = malloc(sizeof(int) * (nl + 1));
            int *rp3 = malloc(sizeof(int) * (s[4] + 1));
            int *ci2 = malloc(sizeof(int) * (s[3] > 0 ? s[3] : 1));
            double *v2 = malloc(sizeof(double) * (s[3] > 0 ? s[3] : 1));
            CHECK(or_export(h, l, 2, rp2, ci2, v2) == 0);
            CHECK(or_export(h, l, 3, rp3, ci2, v2) == 0);
            int *cf = malloc(sizeof(int) * nl);
            CHECK(or_export_cf(h, l, cf) == 0);
            double *in = calloc(nl, sizeof(double)), *xc = calloc(s[4], sizeof(double));
            double *out = calloc(nl, sizeof(double)), *outc = calloc(s[4], sizeof(double));
            rhs(nl, in);
            CHECK(or_level_op(h, l, 0, in, in, out) == 0);
            CHECK(or_level_op(h, l, 1, in, in, out) == 0);
            CHECK(or_level_op(h, l, 2, in, NULL, outc) == 0);
            CHECK(or_level_op(h, l, 3, xc, in, out) == 0);
            free(rp2); free(rp3); free(ci2); free(v2); free(cf); free(in); free(xc); free(out); free(outc);
        }
        if (l >= 1) {
            unsigned char *mk = malloc(s[1] > 0 ? s[1] : 1);
            CHECK(or_export_mask(h, l, 0, mk) == 0);
            CHECK(or_export_mask(h, l, 1, mk) == 0);
            double *m = malloc(sizeof(double) * nl);
            CHECK(or_export_rowmax(h, l, m) == 0);
            free(mk); free(m);
        }
        free(rp); free(ci); free(v);
    }
    double *b = malloc(sizeof(double) * n), *x = calloc(n, sizeof(double)), *hist = malloc(sizeof(double) * 301);
    rhs(n, b);
    SolveInfo info;
    int rc = or_solve(h, b, x, 1, 1e-10, 300, 1, 2, 1, 0.0, 0.01, &info, hist);
    CHECK(rc == 0 && info.converged && info.reintroductions >= 1);
    memset(x, 0, sizeof(double) * n);
    CHECK(or_solve(h, b, x, 0, 1e-8, 300, 0, 3, 1, 0.5, 0.01, &info, hist) == 0);
    CHECK(or_vcycle(h, b, x) == 0);
    int first = -1;
    while (or_reintroduce(h, 1, 0.01, &first) == 0) {}
    free(b); free(x); free(hist); free(gam);
}

int main(void) {
    int *rp, *ci;
    double *v;
    for (int dim = 2; dim <= 3; ++dim) {
        int n = dim == 2 ? poisson(24, 20, 1, &rp, &ci, &v) : poisson(10, 9, 8, &rp, &ci, &v);
        for (int coarsen = 0; coarsen < 2; ++coarsen) {
            Hier *h = NULL;
            CHECK(or_setup(n, rp, ci, v, 0.25, 20, 25, 2.0 / 3.0, 1, 1, NULL, 0, coarsen, 7, &h) == 0);
            exercise(h, n);
            CHECK(or_set_lumping(h, 1) == 0);
            CHECK(or_set_method(h, 1) == 0);
            exercise(h, n);
            CHECK(or_set_relaxation(h, 1, 8) == 0);
            CHECK(or_set_lumping(h, 0) == 0);
            exercise(h, n);
            or_free(h);
        }
        double ng[25];
        for (int l = 0; l < 25; ++l) ng[l] = l >= 2 ? 0.1 : 0.0;
        Hier *h = NULL;
        CHECK(or_setup(n, rp, ci, v, 0.25, 20, 25, 2.0 / 3.0, 1, 1, ng, 25, 0, 0, &h) == 0);
        exercise(h, n);
        or_free(h);
        /* invalid input: an asymmetric entry is refused */
        v[1] = -0.5;
        h = NULL;
        CHECK(or_setup(n, rp, ci, v, 0.25, 20, 25, 2.0 / 3.0, 1, 1, NULL, 0, 0, 0, &h) != 0 && h == NULL);
        free(rp); free(ci); free(v);
    }
    printf("oracle sanitizer exercise: ok\n");
    return 0;
}
