// Kernels of the multi-right-hand-side (block) V-cycle (gfx950, wave64).
//
// A block vector holds K columns row-interleaved: entry (i, c) at i * K + c,
// K in {4, 8, 16}.  The K values a CSR row gathers from row j of the block are
// contiguous (64 bytes for 16 FP32 columns), so one 16-byte load per lane
// fetches 4 FP32 or 2 FP64 columns, and every nonzero a_ij is read once for
// all K columns instead of once per column.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace amg355 {

// Epilogues of the block row kernel; S = A G row by row (all K columns).
enum BlockOp : int {
    kBSpmv = 0,         // Y = S                                  (restriction)
    kBSpmvScale = 1,    // Y = S, Y2 = omega dinv S               (restriction + next zero-guess sweep)
    kBSpmvAdd = 2,      // Y = U + S                              (interpolate and correct)
    kBResid = 3,        // Y = U - S                              (residual)
    kBJacobi = 4,       // Y = G + omega dinv (U - S)             (weighted Jacobi)
    kBJacobiAccum = 5,  // X += G + omega dinv (U - S), X FP64    (last sweep adds the correction)
    kNumBlockOps = 6
};

// Block width (columns held per row) used for nrhs right-hand sides: 4, 8 or 16.
//
// Every launcher below that takes `live` computes only the leading columns
// when it is not null: *live (a device double) is the number of leading
// columns that matter, and lanes whose columns all lie past it do nothing
// (those columns keep whatever they held; their dot products are 0).  It is
// read on the device, so captured launches follow later changes of it.
int block_width(int nrhs);
// Most partial sums any block reduction writes (for the partials buffer).
int block_partials_needed();

// One block row operation over a CSR matrix with values of type T (the
// gathered block G has a.cols... rows, U/Y/Y2 have a.rows rows; all K wide).
// dinv is per row.  acc (kBJacobiAccum only) is the FP64 block that receives
// the sweep's result added to it.
void launch_block_op(BlockOp op, int k, const CsrT<double>& a, const double* g, const double* u,
                     const double* dinv, double omega, double* y, double* y2, double* acc,
                     hipStream_t st,
                     const double* live = nullptr);
void launch_block_op(BlockOp op, int k, const CsrT<float>& a, const float* g, const float* u,
                     const float* dinv, float omega, float* y, float* y2, double* acc,
                     hipStream_t st,
                     const double* live = nullptr);

// Deterministic per-column reductions: per-workgroup partials (>=
// block_partials_needed() doubles) summed in a fixed order into result[0..K).
struct ColumnDots {
    double* partials;
    double* result;
};

// Outer residual of the FP64 system for all K columns: r = b - A x in FP64,
// stored as rt = (T) r and zt = omega dinvt rt (the zero-guess first sweep of
// the next correction cycle), and as r64 when not null; norms2 receives
// sum_i r_ic^2 per column.
void launch_block_outer_residual(int k, const CsrView& a, const double* x, const double* b,
                                 const double* dinvt, double omega, double* rt, double* zt, double* r64,
                                 ColumnDots norms2, hipStream_t st,
                                 const double* live = nullptr);
void launch_block_outer_residual(int k, const CsrView& a, const double* x, const double* b,
                                 const float* dinvt, float omega, float* rt, float* zt, double* r64,
                                 ColumnDots norms2, hipStream_t st,
                                 const double* live = nullptr);

// ---- conjugate gradients on every column at once (FP64 iterates) -----------
// Column c's scalars live in scal[i + c].  Columns with scal[i_act + c] == 0
// are frozen (converged): their x, r and p are not changed.

// q = A p (FP64) with dot[c] = p_c . q_c
void launch_block_spmv_dot(int k, const CsrView& a, const double* p, double* q, ColumnDots dot, hipStream_t st,
                           const double* live = nullptr);
// alpha_c = scal[i_num+c] / scal[i_den+c]; x += alpha p; r -= alpha q;
// norms[c] = |r_c|^2; rt = (T) r and zt = omega dinvt rt.  A column whose
// denominator is not positive and finite is left unchanged and sets
// flags[c] = 1.
void launch_block_cg_update_xr(int n, int k, double* x, double* r, const double* p, const double* q,
                               const double* scal, int i_num, int i_den, int i_act, double* flags,
                               const double* dinvt, double omega, double* rt, double* zt, ColumnDots norms,
                               hipStream_t st,
                               const double* live = nullptr);
void launch_block_cg_update_xr(int n, int k, double* x, double* r, const double* p, const double* q,
                               const double* scal, int i_num, int i_den, int i_act, double* flags,
                               const float* dinvt, float omega, float* rt, float* zt, ColumnDots norms,
                               hipStream_t st,
                               const double* live = nullptr);
// p = z + beta_c p with beta_c = scal[i_num+c] / scal[i_den+c] on active
// columns; p = z in every column if restart_all, else in the columns with
// scal[i_restart+c] != 0 (i_restart < 0: none); z in FP64 or FP32 (widened)
void launch_block_cg_update_p(int n, int k, double* p, const double* z, const double* scal, int i_num,
                              int i_den, int i_act, int i_restart, bool restart_all, hipStream_t st,
                              const double* live = nullptr);
void launch_block_cg_update_p(int n, int k, double* p, const float* z, const double* scal, int i_num,
                              int i_den, int i_act, int i_restart, bool restart_all, hipStream_t st,
                              const double* live = nullptr);
// Fresh start of the columns with scal[i_load+c] != 0: x_c = 0, r_c = b_c,
// rt_c = (T) b_c, zt_c = omega dinvt rt_c, norms[c] = |b_c|^2 (other columns
// untouched; their norms are 0)
void launch_block_load_columns(int n, int k, const double* scal, int i_load, const double* b, double* x,
                               double* r, const double* dinvt, double omega, double* rt, double* zt,
                               ColumnDots norms, hipStream_t st);
void launch_block_load_columns(int n, int k, const double* scal, int i_load, const double* b, double* x,
                               double* r, const float* dinvt, float omega, float* rt, float* zt,
                               ColumnDots norms, hipStream_t st);
// Slot bookkeeping after an iteration, on the device: for active columns
// count the iteration and stop a column whose ||r|| <= rtol ||b|| (state 1),
// that reached maxit (2) or broke down (3).  Columns loaded in the iteration
// (i_load >= 0) first take |b|^2 from scal[i_new+c] and a reset counter; a
// zero right-hand side stops at once (state 1, 0 iterations).  Updates the
// active flags; scal[i_rel+c] = ||r|| / ||b||.
void launch_block_converge(int k, double* scal, int i_act, int i_norm, int i_nr0, int i_flag, int i_iter, int i_stat,
                           int i_rel, int i_load, int i_new, double rtol, int maxit, hipStream_t st);
// column c of a K-wide block from / to a plain vector of n entries
void launch_block_column_in(int n, int k, int c, const double* v, double* blk, hipStream_t st);
void launch_block_column_out(int n, int k, int c, const double* blk, double* v, hipStream_t st);
// The preconditioner's last level-0 sweep z = G + omega dinv (U - A G), kept in
// the cycle's precision, with dot[c] = r64_c . (double) z_c (the CG inner
// product r.z; the widening is exact)
void launch_block_sweep_dot(int k, const CsrT<double>& a, const double* g, const double* u, const double* dinv,
                            double omega, double* zt, const double* r64, ColumnDots dot, hipStream_t st,
                            const double* live = nullptr);
void launch_block_sweep_dot(int k, const CsrT<float>& a, const float* g, const float* u, const float* dinv,
                            float omega, float* zt, const double* r64, ColumnDots dot, hipStream_t st,
                            const double* live = nullptr);
// zt = x with dot[c] = r64_c . (double) x_c
void launch_block_copy_dot(int n, int k, const double* x, double* zt, const double* r64, ColumnDots dot,
                           hipStream_t st, const double* live = nullptr);
void launch_block_copy_dot(int n, int k, const float* x, float* zt, const double* r64, ColumnDots dot,
                           hipStream_t st, const double* live = nullptr);

// Y = Ainv B for the FP64 dense inverse of the coarsest operator (n x n) and
// K-wide blocks; accumulation in FP64.
void launch_block_dense_matvec(int n, int k, const double* ainv, const double* b, double* y,
                               hipStream_t st,
                               const double* live = nullptr);
void launch_block_dense_matvec(int n, int k, const double* ainv, const float* b, float* y,
                               hipStream_t st,
                               const double* live = nullptr);

// X += (double) E over n * k entries
void launch_block_accumulate(int64_t count, double* x, const float* e, hipStream_t st);
void launch_block_accumulate(int64_t count, double* x, const double* e, hipStream_t st);

// Copies between a caller's n x nrhs block (row stride nrhs) and a K-wide
// block (columns nrhs..K-1 zero on packing, dropped on unpacking).
void launch_block_pack(int n, int nrhs, int k, const double* src, double* dst, hipStream_t st);
void launch_block_unpack(int n, int nrhs, int k, const double* src, double* dst, hipStream_t st);

}  // namespace amg355
