/*
 * amg.h -- C ABI of the MI355X sparsified-AMG library (libamg355.so).
 *
 * Method: Bienz, Falgout, Gropp, Olson, Schroder, "Reducing Parallel
 * Communication in Algebraic Multigrid through Sparsification".  The library
 * solves A x = b for a symmetric positive definite A (Section 1) in two
 * phases: a setup that builds the Galerkin hierarchy (Section 2, amg_setup)
 * and retains it, a sparsification post-pass over the coarse operators
 * (Section 3, Sparse Galerkin, with the diagonal lumping of Algorithm 3b,
 * Section 3.1), and a solve phase (Section 2, amg_solve V-cycle; used alone
 * or as the preconditioner of CG) with the adaptive reintroduction of
 * Section 6 (adaptive_solve).
 *
 * Conventions for every entry point:
 *  - No C++ exception crosses the ABI; every call returns an amg_status.
 *  - Matrices are CSR with int32 row pointers (n+1), int32 column indices
 *    sorted ascending within each row, and float64 values.
 *  - "Device" pointers are HIP device memory on the GPU that was current
 *    when the handle was created; all device work is issued on the handle's
 *    stream.  "Host" pointers are ordinary host memory.
 *  - A handle is not thread safe.  Distinct handles are independent.
 *  - A failed call leaves the previously built hierarchy usable: new
 *    sparsified operators are built first and swapped in afterwards.
 *  - On failure amg_last_error(h) describes the cause.
 */
#ifndef AMG355_AMG_H
#define AMG355_AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amg_ctx* amg_handle;
typedef struct amg_batch_ctx* amg_batch;

typedef enum {
    AMG_OK = 0,
    AMG_NOTHING_TO_REINTRODUCE = 1, /* informational: every coarse gamma is already 0 */
    AMG_NOT_READY = 2,              /* informational: amg_batch_poll without waiting, step still running */
    AMG_ERR_INVALID_ARG = -1,       /* NULL pointer, n <= 0, gamma NaN or outside [0,1], bad params */
    AMG_ERR_BAD_MATRIX = -2,        /* unsorted/duplicate/out-of-range column, missing or
                                       non-positive diagonal, non-finite value, not bitwise symmetric */
    AMG_ERR_OUT_OF_MEMORY = -3,     /* the allocator returned NULL */
    AMG_ERR_DEVICE = -4,            /* a HIP call failed */
    AMG_ERR_NOT_CONVERGED = -5,     /* maxit reached; x holds the last iterate, info is filled */
    AMG_ERR_BREAKDOWN = -6,         /* non-finite residual, or p^T A p <= 0 in CG */
    AMG_ERR_STATE = -7              /* call out of order (e.g. on a destroyed or failed handle) */
} amg_status;

/* Device-memory allocator.  alloc returns device memory of at least `bytes`
   usable on `stream`, or NULL.  free releases a block returned by alloc.
   Passing NULL for both uses hipMalloc / hipFree.  The Python binding passes
   PyTorch's caching allocator. */
typedef void* (*amg_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*amg_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

/* Setup parameters (Section 2, amg_setup inputs; strength and interpolation
   formulas are the classical Ruge-Stueben ones the paper cites). */
typedef struct {
    double theta;        /* strength threshold, default 0.25 */
    int32_t max_coarse;  /* coarsen while n > max_coarse (max_size), default 49 */
    int32_t max_levels;  /* at most this many levels, default 25 */
    double omega;        /* weighted-Jacobi weight, default 2/3 */
    int32_t nu_pre;      /* pre-smoothing sweeps, default 1 */
    int32_t nu_post;     /* post-smoothing sweeps, default 1 */
} amg_setup_params;

enum { AMG_STATIONARY = 0, AMG_PCG = 1 };

/* Solve parameters (Section 6, adaptive_solve inputs k, s, tol and the
   gamma floor gamma_min). */
typedef struct {
    int32_t method;      /* AMG_STATIONARY or AMG_PCG, default AMG_PCG */
    double rtol;         /* converged when ||r|| <= rtol ||r0||, default 1e-8 */
    int32_t maxit;       /* default 200 */
    int32_t adaptive;    /* 0/1: windowed reintroduction, default 0 */
    int32_t k;           /* iterations per convergence window, default 3 */
    int32_t s;           /* levels updated per reintroduction, default 1 */
    double rho_max;      /* reintroduce when the window factor exceeds this, default 0.5 */
    double gamma_min;    /* new gamma below this becomes 0, default 0.01 */
    int32_t precision;   /* 64 (default): the V-cycle in FP64.  32: the V-cycle in FP32
                            (operator values, vectors and accumulation; the coarsest
                            inverse stays FP64) as the preconditioner of FP64 CG, or as
                            the correction of FP64 iterative refinement for
                            AMG_STATIONARY; residuals, dot products and the stop test
                            stay FP64 */
    int32_t zero_guess;  /* 1: start from x0 = 0 whatever x holds on entry (the
                            method's initial guess): x is set to zero and the
                            initial residual is b itself, with no product by the
                            zero vector.  0 (default): x holds x0.  amg_solve and
                            amg_solve_noalloc only; amg_solve_block rejects 1 */
} amg_solve_params;

typedef struct {
    int32_t iters;            /* iterations taken (all windows) */
    int32_t restarts;         /* CG restarts after a hierarchy change */
    int32_t reintroductions;  /* calls of the gamma ladder that changed the hierarchy */
    int32_t converged;        /* 1 if ||r|| <= rtol ||r0|| */
    double relres;            /* true ||b - A x|| / ||b - A x0|| at exit */
    double rho_avg;           /* relres^(1/iters) */
} amg_solve_info;

void amg_setup_params_default(amg_setup_params* p);
void amg_solve_params_default(amg_solve_params* p);

/* Build the Galerkin hierarchy of A_0 (Section 2, amg_setup without the
   optional sparsify, as Section 3's sparse_hybrid_setup prescribes).
   row_ptr/col/val: host arrays of A_0, copied; the caller keeps them.
   params: NULL for defaults.  stream: hipStream_t for all device work
   (NULL = default stream).  alloc/free/user: device allocator (both NULL or
   both set).  On success *out holds a new handle with every coarse gamma 0
   (sparsified operators equal the Galerkin ones). */
amg_status amg_setup_from_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                              const double* val, const amg_setup_params* params,
                              void* stream, amg_alloc_fn alloc, amg_free_fn free_fn,
                              void* user, amg_handle* out);

/* The method of non-Galerkin coarse grids (Section 2.1; amg_setup with its
   optional sparsify): as amg_setup_from_csr, but each coarse product
   A_l = P_{l-1}^T A_{l-1} P_{l-1} is sparsified as soon as it is formed, with
   tolerance gamma[l] (l < count; 0 past the end; gamma[0] is ignored), the
   minimal pattern from the hierarchy's finer operator, the keep set of
   Algorithm 3 and diagonal lumping (Algorithm 3b), and it replaces the
   product: the next level's strength, split, interpolation and product are
   built from it.  The Galerkin operators are not kept, so nothing can be
   reintroduced into them; the Sparse/Hybrid Galerkin post-pass (amg_sparsify)
   and reintroduction still apply on top, relative to these operators.
   gamma: host array, each entry in [0, 1]. */
amg_status amg_setup_nongalerkin_from_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                                          const double* val, const amg_setup_params* params,
                                          const double* gamma, int32_t count, void* stream,
                                          amg_alloc_fn alloc, amg_free_fn free_fn, void* user,
                                          amg_handle* out);

/* Build the Galerkin hierarchy on the device (Section 2, amg_setup: strength,
   C/F split, direct interpolation, Galerkin product, every level).
   row_ptr/col/val: DEVICE arrays of A_0 (n + 1, nnz, nnz entries) that the
   work on `stream` may read; they are copied, and the caller keeps them.  The
   input contract is checked on the device (AMG_ERR_BAD_MATRIX names the
   first offending row).  coarsening:
     AMG_COARSEN_RS    the Ruge-Stueben first pass, run on the host from the
                       strength pattern the device builds (one download per
                       level); the hierarchy equals amg_setup_from_csr's bit
                       for bit;
     AMG_COARSEN_PMIS  PMIS, the parallel aggressive coarsening Section 1
                       cites, in rounds on the device: weights lambda_i + u_i
                       with u_i from output i+1 of the SplitMix64 stream
                       seed + l on level l; points no point depends on
                       strongly start as F; each round, undecided points that
                       beat every undecided strong neighbour (larger weight,
                       ties to the smaller index) become C, then undecided
                       points depending strongly on a C point become F.
   The products are formed as listed terms sorted stably by (row, column),
   so each entry sums its terms in the canonical order of the host setup.
   Temporary device memory of up to ~40 bytes per product term comes from the
   allocator.  Other arguments and the result as for amg_setup_from_csr. */
enum { AMG_COARSEN_RS = 0, AMG_COARSEN_PMIS = 1 };
amg_status amg_setup_device(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                            const double* val, const amg_setup_params* params, int32_t coarsening,
                            uint64_t seed, void* stream, amg_alloc_fn alloc, amg_free_fn free_fn,
                            void* user, amg_handle* out);

/* Timing of amg_setup_device's kernel classes with HIP events on the setup's
   stream, for the whole process: while enabled, every device setup adds,
   per class, the number of timed groups, their summed duration in
   milliseconds and their algorithmic bytes (each array entry moved once per
   launch; a sort of m (key, value) pairs counts 32 m, one read and one write
   of each pair).  Enabling resets the totals; enable = 0 stops timing.
   Classes AMG_SK_*: strength pattern, C/F split, interpolation (numbering
   and P), transpose (R = P^T without its sort), term listing of the
   products, sorts, combination of sorted terms into CSR, symmetrization. */
enum {
    AMG_SK_STRENGTH = 0, AMG_SK_SPLIT = 1, AMG_SK_INTERP = 2, AMG_SK_TRANSPOSE = 3,
    AMG_SK_EXPAND = 4, AMG_SK_SORT = 5, AMG_SK_COMBINE = 6, AMG_SK_SYMMETRIZE = 7, AMG_SK_NUM = 8
};
amg_status amg_setup_profile_enable(int32_t enable);
amg_status amg_setup_profile_read(int32_t kernel_class, int64_t* count, double* ms, double* bytes);

/* Sparse Galerkin sparsification with diagonal lumping (Algorithm 3 keep set,
   Algorithm 3b loop) of every level l >= first_level (first_level >= 1) with
   drop tolerance gamma in [0, 1]; levels below first_level get gamma 0.  The
   minimal pattern M_l and the row maxima of A_l are computed on the first
   call and cached; the result replaces the sparsified operators. */
amg_status amg_sparsify(amg_handle h, double gamma, int32_t first_level);

/* Same, with one tolerance per level: gamma[l] for l = 0 .. count-1
   (gamma[0] is ignored: A_0 is never sparsified; levels >= count get 0). */
amg_status amg_sparsify_levels(amg_handle h, const double* gamma, int32_t count);

/* Selects the sparsification method for later amg_sparsify,
   amg_sparsify_levels, amg_reintroduce and adaptive solves (Section 3,
   sparse_hybrid_setup).  AMG_SPARSE_GALERKIN (default): the minimal pattern
   M_l comes from the Galerkin A_{l-1}.  AMG_HYBRID_GALERKIN: from the
   sparsified \hat A_{l-1} (levels are sparsified finest first, and a
   reintroduction also redoes every coarser sparsified level at its gamma,
   since its M depends on the finer operator).  The hierarchy is not changed
   until the next sparsify. */
enum { AMG_SPARSE_GALERKIN = 0, AMG_HYBRID_GALERKIN = 1 };

/* Where amg_sparsify, amg_sparsify_levels and amg_reintroduce put the
   entries they drop (from the next such call on; existing sparsified
   operators are not redone).  AMG_LUMP_DIAGONAL (default): diagonal lumping,
   Algorithm 3b (Section 3.1).  AMG_LUMP_STRONG: the second loop of
   Algorithm 3 (the method of non-Galerkin coarse grids): a dropped entry
   (i,j) is shared among W = {m : S_jm strong, (i,m) kept}, S the classical
   strength of the operator being sparsified (setup theta), in proportion
   |a_jm|; each share c is added to (i,m) and (m,i) and subtracted from
   (m,m) (added once to (i,i) when m = i); with W empty the entry goes to the
   diagonal.  Kept entries start at their Galerkin values and every entry
   adds its shares in ascending order of the dropped entry they come from,
   so the result is symmetric bit for bit.  Row sums are kept; unlike
   diagonal lumping, positive definiteness is not guaranteed.  The
   non-Galerkin setup always lumps to the diagonal.  AMG_ERR_STATE while a
   batch engine exists, AMG_ERR_INVALID_ARG for any other value. */
enum { AMG_LUMP_DIAGONAL = 0, AMG_LUMP_STRONG = 1 };
amg_status amg_set_lumping(amg_handle h, int32_t lumping);

/* Testing hook: the launch shapes of the strong-lumping kernels on this
   handle for later sparsify / reintroduce calls.  Every shape gives the same
   bits; tests use it to compare them.  Rows of mean length >= wide_mean_row
   (default 0) run a workgroup per row with the row staged in LDS, shorter
   ones a wave per row; den_wave_mean_row < 0 (default -1) keeps the library's
   rule for the denominators' wave-per-row stage (levels of at least 16,384
   rows of fewer than 80 entries), a value >= 0 uses that stage wherever the
   mean row length is below it; levels of fewer than small_rows rows (default
   4,096) give the share kernel 1,024-thread workgroups.  AMG_ERR_STATE without
   a hierarchy, AMG_ERR_INVALID_ARG for NaN or small_rows < 0. */
amg_status amg_set_lump_shapes(amg_handle h, double wide_mean_row, double den_wave_mean_row,
                               int32_t small_rows);

/* Smoother of the V-cycle.  AMG_RELAX_JACOBI (default): weighted Jacobi with
   omega from the setup parameters.  AMG_RELAX_HYBRID_GS: hybrid Gauss-Seidel,
   the relaxation of the paper's experiments (Section 5, there with one block
   per process): the rows are split into contiguous blocks of block_rows
   rows; inside a block the sweep is Gauss-Seidel (rows visited in order use
   the new values of their block's rows visited before them), across blocks
   Jacobi with weight 1; row i becomes (b_i - sum_{j != i} a_ij y_j) / a_ii.
   Pre-smoothing sweeps forward, post-smoothing backward, so the cycle stays
   a symmetric preconditioner for CG.  One thread sweeps each block, so
   there is one row of parallelism per block: large blocks converge better
   (one block is textbook Gauss-Seidel) and run slower.  Hybrid Gauss-Seidel
   serves amg_solve with precision 64 and amg_vcycle; the FP32, block and
   batch entry points return AMG_ERR_INVALID_ARG while it is selected.
   AMG_ERR_STATE while a batch engine exists. */
enum { AMG_RELAX_JACOBI = 0, AMG_RELAX_HYBRID_GS = 1 };
amg_status amg_set_relaxation(amg_handle h, int32_t relaxation, int32_t block_rows);
amg_status amg_set_method(amg_handle h, int32_t method);

/* Reintroduction (Section 6, adaptive_solve and its Example): find the
   finest coarse level with gamma > 0 and, on it and the next s-1 levels,
   set gamma <- gamma/10 (0 if gamma/10 < gamma_min), re-sparsifying them
   from the retained Galerkin operators.  *first_changed_level (nullable)
   receives that level, or -1 with AMG_NOTHING_TO_REINTRODUCE. */
amg_status amg_reintroduce(amg_handle h, int32_t s, double gamma_min,
                           int32_t* first_changed_level);

/* Solve A_0 x = b.  b, x: device arrays of n doubles; x holds x0 on entry
   and the result on exit.  Stationary: x <- V(b, x) per iteration.  PCG:
   Hestenes-Stiefel CG preconditioned by one V-cycle z = V(r, 0), stop test on
   the recursively updated residual.  With params->adaptive, every k
   iterations the true residual is formed; if the window factor
   (||r_end||/||r_start||)^(1/k) exceeds rho_max and some coarse gamma > 0,
   amg_reintroduce(h, s, gamma_min) is applied, x reverts to the window start
   if the window diverged, and CG restarts.  params NULL = defaults.  info
   (nullable) is filled on every return that ran iterations.  hist (nullable,
   host, maxit+1 doubles) receives ||r_0|| and the residual norm after each
   iteration.  With params->zero_guess = 1 the solve starts from x0 = 0
   whatever x holds (x is zeroed, r_0 = b). */
amg_status amg_solve(amg_handle h, const double* b, double* x, const amg_solve_params* params,
                     amg_solve_info* info, double* hist);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): amg_solve
   with the same arguments, results and error codes, bit for bit, that
   allocates nothing.  Its work memory (the CG vectors r, z, p, q, the
   window-start x and the window's true residual, the dot-product partials
   and the scalar slots) lives in a static device array of the library, about
   97 MiB, that each GPU the library runs on holds until the process ends.
   Limits: n <= 2,097,152 rows and precision 64, else AMG_ERR_INVALID_ARG;
   AMG_ERR_STATE while kernel profiling is on, or when an adaptive solve
   under strong lumping could reintroduce on a level sparsified with diagonal
   lumping (whose strong-lumping buffers do not exist yet).  The hierarchy,
   its sparsified operators and the caller's b and x are used as they are.
   Every call on one GPU shares that GPU's array: calls that overlap on one
   GPU (other streams, other threads) race; calls on one stream, or
   synchronised with each other, do not. */
amg_status amg_solve_noalloc(amg_handle h, const double* b, double* x, const amg_solve_params* params,
                             amg_solve_info* info, double* hist);

/* One V-cycle (Section 2, amg_solve) in place: x <- V(b, x); device arrays. */
amg_status amg_vcycle(amg_handle h, const double* b, double* x);

/* The same cycle in FP32 (values, vectors, accumulation; FP64 coarsest
   inverse): x <- V32(b, x), device float arrays.  The first call builds the
   FP32 copies of the hierarchy's values; later sparsify/reintroduce calls
   keep them current. */
amg_status amg_vcycle32(amg_handle h, const float* b, float* x);

/* Several right-hand sides at once: A X = B for nrhs columns (1 <= nrhs <=
   16) with iterative refinement, X_c <- X_c + V(B_c - A X_c, 0) per column
   (the Section 2 V-cycle as the correction, the residual always in FP64),
   every cycle step applied to all columns in one pass over each operator.
   b, x: device FP64 arrays of n x nrhs entries, row-major (entry (i, c) at
   i*nrhs + c), 16-byte aligned; x holds the initial guesses and receives the
   solutions.  params: method must be AMG_STATIONARY and adaptive 0;
   precision 64, or 32 for a correction cycle in FP32 values, vectors and
   accumulation (FP64 coarsest inverse); NULL = defaults with those two
   fields.  Iterates until every column has ||r_c|| <= rtol ||r0_c|| (columns
   with r0_c = 0 count as converged at once) or maxit.  info (nullable):
   iters of the whole block, relres the largest column ratio.  col_iters
   (nullable, host, nrhs): the first iteration at which column c met the
   tolerance, -1 if it never did.  col_relres (nullable, host, nrhs): the
   final ||r_c|| / ||r0_c||.  Errors: AMG_ERR_INVALID_ARG for other
   parameters or misaligned arrays, AMG_ERR_NOT_CONVERGED after maxit,
   AMG_ERR_BREAKDOWN on a non-finite residual.  nrhs other than 4, 8, 16 is
   padded internally to the next of them (extra device copies of b and x). */
amg_status amg_solve_block(amg_handle h, int32_t nrhs, const double* b, double* x,
                           const amg_solve_params* params, amg_solve_info* info,
                           int32_t* col_iters, double* col_relres);

/* One V-cycle on nrhs = 4, 8 or 16 columns in place: X <- V(B, X), device
   arrays laid out as for amg_solve_block (16-byte aligned); FP64 and FP32
   (values, vectors, accumulation; FP64 coarsest inverse) versions. */
amg_status amg_vcycle_block(amg_handle h, int32_t nrhs, const double* b, double* x);
amg_status amg_vcycle_block32(amg_handle h, int32_t nrhs, const float* b, float* x);

/* Single steps of the V-cycle on level l, device arrays (for component
   checks and for callers composing their own cycles):
     AMG_OP_RESIDUAL     out = b - Ahat_l x                 (in = b)
     AMG_OP_JACOBI       out = x + omega D^-1 (b - Ahat_l x) (in = b)
     AMG_OP_RESTRICT     out = P_l^T in        (out has n_{l+1} entries)
     AMG_OP_INTERPOLATE  out = x + P_l in      (in has n_{l+1} entries)
     AMG_OP_COARSE_SOLVE out = Ahat_L^-1 in    (l ignored)
     AMG_OP_SPMV_A       out = A_l x           (Galerkin operator)
     AMG_OP_SPMV_AHAT    out = Ahat_l x
     AMG_OP_GS_FORWARD   out = one forward hybrid Gauss-Seidel sweep on
                         Ahat_l from x (in = b; out != x)
     AMG_OP_GS_BACKWARD  the backward sweep                               */
enum {
    AMG_OP_RESIDUAL = 0, AMG_OP_JACOBI = 1, AMG_OP_RESTRICT = 2, AMG_OP_INTERPOLATE = 3,
    AMG_OP_COARSE_SOLVE = 4, AMG_OP_SPMV_A = 5, AMG_OP_SPMV_AHAT = 6, AMG_OP_GS_FORWARD = 7,
    AMG_OP_GS_BACKWARD = 8
};
amg_status amg_level_op(amg_handle h, int32_t level, int32_t op, const double* in,
                        const double* x, double* out);

amg_status amg_num_levels(amg_handle h, int32_t* nlev);

/* Sizes of level l; any output pointer may be NULL.  bytes = algorithmic HBM
   bytes of one V-cycle's work on this level (relaxation, residual and
   transfers with the current sparsified operator). */
amg_status amg_get_level(amg_handle h, int32_t l, int64_t* n, int64_t* nnz_galerkin,
                         int64_t* nnz_sparse, int64_t* nnz_p, int64_t* n_coarse,
                         double* gamma, int64_t* bytes);

/* Copy an operator of level l into caller-allocated host arrays sized from
   amg_get_level: row_ptr (rows+1), col and val (nnz).  which: AMG_MAT_A
   (Galerkin A_l), AMG_MAT_AHAT (sparsified), AMG_MAT_P (P_l, n_l x n_{l+1}),
   AMG_MAT_R (R_l = P_l^T). */
enum { AMG_MAT_A = 0, AMG_MAT_AHAT = 1, AMG_MAT_P = 2, AMG_MAT_R = 3 };
amg_status amg_export_level(amg_handle h, int32_t l, int32_t which, int32_t* row_ptr,
                            int32_t* col, double* val);

/* Per-nonzero flags of A_l (host array of nnz_galerkin bytes): AMG_MASK_M
   the minimal pattern M_l, AMG_MASK_KEEP the keep decision of the last
   sparsification of level l.  Levels >= 1, after a sparsify call. */
enum { AMG_MASK_M = 0, AMG_MASK_KEEP = 1 };
amg_status amg_export_mask(amg_handle h, int32_t l, int32_t which, uint8_t* out);

/* Per-row vectors of level l (host array of n_l doubles): AMG_VEC_ROWMAX
   m_i = max_{k!=i} |a_ik| of A_l (after a sparsify call), AMG_VEC_DINV
   1/diag(Ahat_l). */
enum { AMG_VEC_ROWMAX = 0, AMG_VEC_DINV = 1 };
amg_status amg_export_vector(amg_handle h, int32_t l, int32_t which, double* out);

/* C/F split of level l < L (host array of n_l ints, 1 = C). */
amg_status amg_export_split(amg_handle h, int32_t l, int32_t* cf);

/* 16-bit column indices (enabled by default).  For every level's fixed
   operators A_l, P_l and R_l that the LDS-staged row kernels run on, a second
   copy of the column indices is kept as 16-bit offsets from a base per row
   block of those kernels, when every block's columns span at most 65535 (it
   does for banded operators, e.g. the 7-point stencil up to 181^3): the
   kernels then move 10 instead of 12 bytes per entry.  Results are bitwise the same either way.  enable = 0 drops the
   copies (frees their memory), 1 builds them; AMG_ERR_STATE while a batch
   engine exists.  The SELL-64 copies (see amg_row_format) are compressed
   too: a square operator whose every slice of 64 rows has at most 64
   distinct offsets column - row (stencil-like operators) keeps one byte per
   entry, the position of its offset in a table of the slice's offsets;
   otherwise the columns are kept as 16-bit offsets from a base per slice
   where every slice spans at most 65535 columns; they are rebuilt in 32
   bits when the form is switched off.  amg_index_width reports the bytes
   per column index the FP64 row kernels read for matrix `which` (AMG_MAT_*)
   of level l: 1, 2 or 4 (of the SELL-64 copy where one exists; the FP32
   cycle reads the CSR form's). */
amg_status amg_set_compact_indices(amg_handle h, int32_t enable);
amg_status amg_index_width(amg_handle h, int32_t l, int32_t which, int32_t* bytes);

/* Which FP64 row kernel serves matrix `which` (AMG_MAT_*) of level l:
   AMG_FORMAT_ROW, a subgroup of lanes per CSR row (small levels, long rows);
   AMG_FORMAT_STREAM, CSR row blocks staged through LDS (large levels with
   short rows); AMG_FORMAT_SELL, a SELL-64 copy built at setup (large levels
   with short rows whose slices pad the entries by at most a tenth: one lane
   per row, a wavefront per slice of 64 rows, coalesced loads of every
   entry).  Results do not depend on it beyond rounding of the row sums. */
enum { AMG_FORMAT_ROW = 0, AMG_FORMAT_STREAM = 1, AMG_FORMAT_SELL = 2 };
amg_status amg_row_format(amg_handle h, int32_t l, int32_t which, int32_t* format);

/* Kernel timing with HIP events on the handle's stream.  While enabled,
   every launch of a kernel of class kernel_class (-1: every class) on level
   `level` (-1: every level) is bracketed by a pair of events;
   amg_profile_read returns the number of bracketed launches and their summed
   duration in milliseconds since the last amg_profile_enable call.  Classes:
   AMG_K_*.  Enabling resets the counters; enable = 0 stops timing. */
enum {
    AMG_K_JACOBI = 0, AMG_K_JACOBI_ZERO = 1, AMG_K_RESIDUAL = 2, AMG_K_RESTRICT = 3,
    AMG_K_INTERP = 4, AMG_K_COARSE = 5, AMG_K_SPMV_DOT = 6, AMG_K_VECTOR = 7,
    AMG_K_SPARSIFY = 8,
    /* inside AMG_K_SPARSIFY, strong-neighbour lumping only: the share
       denominators, and the shares added into the kept entries */
    AMG_K_LUMP_DEN = 9, AMG_K_LUMP_SHARES = 10,
    AMG_K_NUM = 11
};
amg_status amg_profile_enable(amg_handle h, int32_t enable, int32_t kernel_class, int32_t level);
amg_status amg_profile_read(amg_handle h, int32_t kernel_class, int32_t level, int64_t* count,
                            double* total_ms);

/* ---- continuous batching -------------------------------------------------
   A batch engine serves a stream of right-hand sides on one hierarchy: up to
   `slots` (4, 8 or 16) of them are solved together by PCG (Section 5, with
   the Section 2 V-cycle as the preconditioner, one CG recurrence per slot and
   every kernel launch shared by all slots), and a slot that finishes can take
   a new right-hand side at the next step while the others keep iterating.  A
   slot's arithmetic does not depend on the other slots or on which slot it
   occupies: its result is bitwise the one amg_solve_block (method PCG, same
   slot count and precision, x0 = 0) gives for that right-hand side.  All
   device work goes to the handle's stream.  While a batch exists, the
   handle's solve, cycle and sparsify entry points return AMG_ERR_STATE. */

/* Device bytes amg_batch_create would allocate for this handle (block work
   space, CG vectors, FP32 copies of the hierarchy if not made yet). */
amg_status amg_batch_bytes(amg_handle h, int32_t slots, int32_t precision, int64_t* bytes);

/* Creates the batch engine of h.  precision 32: the V-cycle in FP32 (values,
   vectors, accumulation) preconditioning FP64 CG; 64: all FP64.  A slot
   finishes when ||r|| <= rtol ||b|| (x0 = 0) or after maxit iterations.
   flags: AMG_BATCH_GRAPHS replays each iteration as a captured HIP graph
   (same kernels, same results; ignored on the null stream and while
   profiling is enabled).  AMG_ERR_STATE if h already has a batch. */
enum { AMG_BATCH_GRAPHS = 1 };
amg_status amg_batch_create(amg_handle h, int32_t slots, int32_t precision, double rtol, int32_t maxit,
                            int32_t flags, amg_batch* out);

/* Copies rhs (device, n doubles) into a free slot; its solve starts at the
   next step.  *slot receives the slot index.  AMG_ERR_STATE if no slot is
   free (a finished slot is free again after amg_batch_collect). */
amg_status amg_batch_submit(amg_batch b, const double* rhs, int32_t* slot);

/* Enqueues `iters` (>= 1) iterations of every active slot, the submitted
   slots starting in the first, and returns without waiting; *launched
   (nullable) = 0 if no slot had work.  The stop test runs on the device after
   every iteration, so a slot stops at its own convergence iteration whatever
   `iters` is (later iterations of the step leave it unchanged); new slots
   can start only at a step boundary.  AMG_ERR_STATE if the previous step has
   not been completed by amg_batch_poll. */
amg_status amg_batch_step(amg_batch b, int32_t iters, int32_t* launched);

/* Completes the last step: wait != 0 blocks until it has run; wait == 0
   returns AMG_NOT_READY if it is still running.  finished (nullable, host,
   slots entries) receives 1 for each slot that finished in this step
   (converged, broke down or reached maxit).  AMG_OK if no step was pending. */
amg_status amg_batch_poll(amg_batch b, int32_t wait, int32_t* finished);

/* Copies the solution of a finished slot into x (device, n doubles; enqueued
   on the handle's stream) and frees the slot.  iters, relres (the CG
   residual ratio ||r||/||b|| when it stopped) and status (AMG_OK,
   AMG_ERR_NOT_CONVERGED or AMG_ERR_BREAKDOWN) are nullable.  AMG_ERR_STATE
   if the slot has not finished. */
amg_status amg_batch_collect(amg_batch b, int32_t slot, double* x, int32_t* iters, double* relres,
                             int32_t* status);

/* Per-slot state (host, slots entries): 0 free, 1 submitted, 2 iterating,
   3 finished and not yet collected. */
amg_status amg_batch_slots(amg_batch b, int32_t* state);

/* Waits for pending work, frees the engine and its work space. */
void amg_batch_destroy(amg_batch b);

/* Device bytes currently allocated by the handle (hierarchy, sparsified
   operators, FP32 copies, work space). */
amg_status amg_device_bytes(amg_handle h, int64_t* bytes);

void amg_destroy(amg_handle h);
const char* amg_status_string(amg_status s);
const char* amg_last_error(amg_handle h);

#ifdef __cplusplus
}
#endif
#endif /* AMG355_AMG_H */
