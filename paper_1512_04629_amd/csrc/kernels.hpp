// Device kernels of the sparsified-AMG hot path (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amg355 {

// Read-only view of a device CSR matrix with values of type T.
template <class T>
struct CsrT {
    const int32_t* rp;
    const int32_t* ci;
    const T* v;
    int rows;
    double mean_row;   // nnz / rows, host side launch configuration only
    // optional 16-bit form of ci read by the LDS-staged kernels: the column
    // of an entry of row block b (rows [b idx_rb, (b + 1) idx_rb)) is
    // cbase[b] + ci16[p]; used only by launches with idx_rb rows per block
    const uint16_t* ci16 = nullptr;
    const int32_t* cbase = nullptr;
    int idx_rb = 0;
    // LDS-staged kernels without a dot product visit the row blocks in
    // descending order (each row's result does not depend on the order)
    int rev = 0;
    // optional SELL-64 copy of the matrix (FP64 values only), used by the row
    // operations when present: rows in slices of 64 (one wavefront, one lane
    // per row); entry k of row 64 s + lane at sl_off[s] + 64 k + lane, slice
    // s holding (sl_off[s + 1] - sl_off[s]) / 64 entries per row; rows
    // shorter than their slice padded with zero values
    const int32_t* sl_off = nullptr;
    const int32_t* sl_col = nullptr;
    const T* sl_val = nullptr;
    int sl_maxw = 0;     // widest slice, host side launch configuration only
    // 16-bit form of sl_col (then sl_col is null): the column of an entry of
    // slice s is sl_base[s] + sl_col16[p]
    const uint16_t* sl_col16 = nullptr;
    const int32_t* sl_base = nullptr;
    // 8-bit form (then sl_col and sl_col16 are null): every slice s lists at
    // most 64 distinct offsets column - row in sl_tab[64 s .. 64 s + 63], and
    // the column of entry p of row r is r + sl_tab[64 s + sl_idx8[p]]
    const uint8_t* sl_idx8 = nullptr;
    const int32_t* sl_tab = nullptr;
};
using CsrView = CsrT<double>;
using CsrView32 = CsrT<float>;

// Epilogues of the CSR row kernel.  s_i = sum_j a_ij g_j (for kZeroJacobiResid
// the gathered value is omega * dinv_j * u_j).
enum RowOp : int {
    kSpmv = 0,            // y_i = s_i
    kSpmvAdd = 1,         // y_i = u_i + s_i                 (interpolate and correct)
    kResid = 2,           // y_i = u_i - s_i                 (residual)
    kResidNorm = 3,       // kResid, dot += y_i^2
    kJacobi = 4,          // y_i = g_i + omega dinv_i (u_i - s_i)
    kJacobiDot = 5,       // kJacobi, dot += u_i y_i
    kZeroJacobiResid = 6, // y2_i = omega dinv_i u_i, y_i = u_i - s_i   (x0 = 0 sweep fused with residual)
    kSpmvDot = 7,         // y_i = s_i, dot += g_i s_i
    kSpmvScale = 8,       // y_i = s_i, y2_i = omega dinv_i s_i   (restriction that also forms
                          //                                        the next level's zero-guess sweep)
    kNumRowOps = 9
};

// Deterministic two-level reduction target: per-block partials (summed in
// block order by a one-block finishing kernel) and the slot that receives
// the final sum.
struct DotTarget {
    double* partials;     // >= number of blocks of the launch
    double* result;       // receives the sum
};

// Lanes per row for a matrix with the given mean row length.
int pick_width(double mean_row_len);

// Number of blocks a row launch with this width uses (for partial buffers),
// and the most any row launch uses.
int row_launch_blocks(int rows, int width);
int max_row_launch_blocks();

// Returns, for the ops that form a dot product (kResidNorm, kJacobiDot,
// kSpmvDot), the number of per-workgroup partials written to dot.partials,
// which launch_dot_finish then adds in order into *dot.result; 0 otherwise.
int launch_row_op(RowOp op, int width, const CsrView& a, const double* g, const double* u,
                  const double* dinv, double omega, double* y, double* y2, DotTarget dot,
                  hipStream_t st);
void launch_dot_finish(const DotTarget& dot, int nparts, hipStream_t st);
// Arms two events for the next launch_row_op on this thread: its row kernel
// records its own start and end in them (not the dot's finishing launch).
// clear_launch_events disarms them and tells whether they were still armed.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool clear_launch_events();
// single precision: values, vectors and accumulation in FP32 (no dot ops)
void launch_row_op(RowOp op, int width, const CsrView32& a, const float* g, const float* u,
                   const float* dinv, float omega, float* y, float* y2, hipStream_t st);

// ---- vector kernels -----------------------------------------------------
// x += alpha p; r -= alpha q; dot -> |r|^2, with alpha = scal[i_num]/scal[i_den];
// if zs is not null also zs = omega dinv r (the next V-cycle's zero-guess
// sweep).  If scal[i_den] is not positive and finite, nothing is updated and
// *flag = 1.0.
// With r32 not null also r32 = (float) r and zs32 = omega dinv32 r32 (the
// FP32 preconditioner's right-hand side and zero-guess sweep).
void launch_cg_update_xr(int n, double* x, double* r, const double* p, const double* q,
                         const double* scal, int i_num, int i_den, double* flag, DotTarget dot,
                         const double* dinv, double omega, double* zs, float* r32,
                         const float* dinv32, float* zs32, hipStream_t st);
// p = z + beta p with beta = scal[i_num]/scal[i_den]; if restart, p = z.
void launch_cg_update_p(int n, double* p, const double* z, const double* scal, int i_num,
                        int i_den, hipStream_t st);
// y = omega dinv x (zero-guess smoothing of one sweep without residual)
void launch_scaled_copy(int n, double* y, const double* dinv, const double* x, double omega,
                        hipStream_t st);
void launch_copy(int n, double* y, const double* x, hipStream_t st);
// host[0..n) = scal[0..n) and host[n] = *extra (0 if extra is null) into
// host-coherent memory, then *flag = seq (one workgroup; the values are
// visible to the host before the flag)
void launch_publish_scalars(int n, const double* scal, double* host, uint32_t* flag, uint32_t seq,
                            const int* extra, hipStream_t st);
void launch_fill_f64(int64_t n, double* p, double v, hipStream_t st);
// dot -> sum_i a_i b_i
void launch_dot(int n, const double* a, const double* b, DotTarget dot, hipStream_t st);
// y = u - A g and y2 = u2 - A g2 with ||y2||^2 into dot, in one pass over the
// SELL-64 copy of A (the bits of the two separate residual launches);
// returns the number of partials to finish, 0 (nothing launched) when A has
// no SELL-64 copy
int launch_sell_dual_resid(const CsrView& a, const double* g, const double* u, double* y, const double* g2,
                           const double* u2, double* y2, DotTarget dot, hipStream_t st);
// x = 0, r = b, dot = ||b||^2: the start of a solve from the zero vector
void launch_zero_guess_start(int n, const double* b, double* x, double* r, DotTarget dot, hipStream_t st);
// number of blocks of a vector-kernel launch over n entries (for partial buffers)
int vector_launch_blocks(int n);
void launch_fill_u8(int64_t n, uint8_t* p, uint8_t v, hipStream_t st);
void launch_fill_u32(int64_t n, unsigned* p, unsigned v, hipStream_t st);
// y = Ainv b for a dense row-major n x n inverse
void launch_dense_matvec(int n, const double* ainv, const double* b, double* y, hipStream_t st);
// inverse of a dense n x n operator given in CSR (n <= dense_invert_max()),
// Gauss-Jordan with partial pivoting; *singular set to 1 on a zero pivot
int dense_invert_max();
void launch_dense_invert(const CsrView& a, double* inv, int* singular, hipStream_t st);
// dinv_i = 1 / a_ii
// (and its FP32 rounding when dinv32 is not null)
void launch_inverse_diagonal(const CsrView& a, double* dinv, float* dinv32, hipStream_t st);
// same as launch_dense_matvec with FP32 vectors (inverse and accumulation FP64)
void launch_dense_matvec(int n, const double* ainv, const float* b, float* y, hipStream_t st);
// precision conversions and FP32 vector helpers
void launch_narrow(int64_t n, float* y, const double* x, hipStream_t st);
void launch_widen_dot(int n, double* y, const float* x, const double* u, DotTarget dot, hipStream_t st);
void launch_add_widened(int n, double* x, const float* e, hipStream_t st);
void launch_scaled_copy(int n, float* y, const float* dinv, const float* x, float omega, hipStream_t st);
void launch_copy(int n, float* y, const float* x, hipStream_t st);
void launch_fill_f32(int64_t n, float* p, float v, hipStream_t st);

// ---- coarse tail: the V-cycle below a level in one workgroup ---------------
// Levels t..L of a V(1,1) cycle with zero initial guesses: down (residual of
// the prescaled sweep, restriction writing the next level's prescaled sweep),
// coarsest dense solve, up (interpolation + post-smoothing).  Level k of the
// tail is lv[k]; lv[count-1] is the coarsest.  On entry lv[0].b holds the
// right-hand side and lv[0].x the first sweep omega D^-1 b; on exit the
// level-t result is in lv[0].xt.
constexpr int kTailMaxLevels = 12;
template <class T>
struct TailCsr {
    const int32_t* rp;
    const int32_t* ci;
    const T* v;
    int rows;
    int cap;             // entries ci and v hold (for a sparsified operator its capacity)
};
template <class T>
struct TailLevel {
    TailCsr<T> A;        // sparsified operator of the level
    TailCsr<T> R, P;     // restriction to / interpolation from the next level
    const T* dinv;
    T *b, *x, *xt, *r;
};
template <class T>
struct TailArgs {
    TailLevel<T> lv[kTailMaxLevels];
    int count;
    const double* coarse_inv;   // FP64 in both precisions
    T omega;
};
// When the tail has at most 6 levels and everything it touches fits the
// workgroup's LDS, the launch first copies the operators, the coarsest
// inverse and the level-t right-hand side and sweep there (every entry an
// operator's capacity holds, so the copy needs no count from the device) and
// runs the cycle on the copies, writing only the level-t result back;
// otherwise the cycle runs on the arrays in memory.
void launch_coarse_tail(const TailArgs<double>& t, hipStream_t st);
void launch_coarse_tail(const TailArgs<float>& t, hipStream_t st);

// ---- sparsification kernels ----------------------------------------------
// Marks M_l: for coarse row I with fine point f = c_points[I], every column J
// of P rows l' in row f of A_{l-1} gives (I,J) and (J,I) in A_l.
void launch_mark_minimal_pattern(int nc, const int32_t* c_points, const int32_t* afine_rp,
                                 const int32_t* afine_ci, const int32_t* p_rp,
                                 const int32_t* p_ci, const int32_t* ac_rp, const int32_t* ac_ci,
                                 uint8_t* in_m, int* missing, hipStream_t st);
// 16-bit column indices for row blocks of rb rows: cbase[b] = smallest
// column in block b, ci16[p] = ci[p] - cbase[b]; *wide (zeroed by the
// caller) counts the blocks whose columns span more than 65535 (then the form
// is unusable)
void launch_compress_index(int rows, int rb, const int32_t* rp, const int32_t* ci, uint16_t* ci16,
                           int32_t* cbase, int* wide, hipStream_t st);
// rows per block of the LDS-staged kernels on this matrix, 0 if row
// operations on it run on the subgroup kernels (which read 32-bit indices)
int stream_block_rows(const CsrView& a);

// SELL-64 copy of a CSR matrix (see CsrT).  launch_sell_widths writes 64
// times the longest row of every slice into width64[0..nslices); after an
// exclusive scan of those into off[0..nslices], launch_sell_fill writes the
// entries: a row's entries in column order, then (value 0, column of the
// row's last entry, or 0 for an empty row) up to its slice's width.
int sell_slices(int rows);
// 8-bit columns of a SELL-64 copy: tab[64 s ..] lists the distinct offsets
// column - row of slice s (rows past the end excluded), idx8[p] the position
// of entry p's offset there; *wide (zeroed by the caller) counts the slices
// with more than 64 distinct offsets (then the form is unusable)
void launch_sell_dictionary(int rows, const int32_t* off, const int32_t* col, uint8_t* idx8, int32_t* tab,
                            int* wide, hipStream_t st);
// 16-bit columns of a SELL-64 copy: base[s] = smallest column of slice s,
// col16[p] = col[p] - base[s]; *wide (zeroed by the caller) counts the slices
// whose columns span more than 65535 (then the form is unusable)
void launch_sell_compress(int rows, const int32_t* off, const int32_t* col, uint16_t* col16, int32_t* base,
                          int* wide, hipStream_t st);
void launch_sell_widths(int rows, const int32_t* rp, int32_t* width64, hipStream_t st);
void launch_sell_fill(int rows, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* off,
                      int32_t* col, double* val, hipStream_t st);
// the row operations take the SELL copy of an operator that use_stream_kernel
// would stream (large, rows of at most 24 entries on average)
bool sell_candidate(const CsrView& a);

// m_i = max_{k != i} |a_ik|
void launch_row_max(int width, const CsrView& a, double* m, hipStream_t st);
// keep flags and per-row kept counts for tolerance gamma; bsum (may be
// null) receives the kept count of each of the launch's keep_count_blocks
// blocks of rows
void launch_keep_count(int width, const CsrView& a, const uint8_t* in_m, const double* m,
                       double gamma, uint8_t* keep, int32_t* cnt, int32_t* bsum, hipStream_t st);
int keep_count_blocks(int width, int rows);
// in-place exclusive scans of up to kMaxScanJobs int32 arrays, one launch
constexpr int kMaxScanJobs = 16;
struct ScanJobs {
    int32_t* data[kMaxScanJobs];
    int n[kMaxScanJobs];
    int count = 0;
};
void launch_scan_jobs(const ScanJobs& jobs, hipStream_t st);
// several small levels' keep flags (and later their compaction) in one launch,
// 64 lanes a row (keep_count_blocks(64, rows) blocks a level): bsum receives
// the level's block counts, and compaction reads their scan from it
constexpr int kMaxMergedLevels = 8;
struct SparsifyLevel {
    CsrView a;
    const uint8_t* in_m;
    const double* m;
    double gamma;
    uint8_t* keep;
    int32_t* cnt;
    int32_t* bsum;
    int32_t* new_rp;
    int32_t* new_ci;
    double* new_v;
    double* dinv;
    float* new_v32;
    float* dinv32;
    int block0;   // set by the launchers
};
struct SparsifyLevels {
    SparsifyLevel lv[kMaxMergedLevels];
    int count = 0;
};
void launch_keep_count_merged(SparsifyLevels& L, hipStream_t st);
void launch_compact_lump_merged(SparsifyLevels& L, hipStream_t st);
// exclusive scan of cnt[0..n) into out[0..n], out[n] = total; scratch >= scan_scratch_ints(n)
int64_t scan_scratch_ints(int n);
void launch_exclusive_scan(int n, const int32_t* cnt, int32_t* out, int32_t* scratch,
                           hipStream_t st);
// compaction of the kept entries with the dropped ones added to the diagonal
// (new_v32/dinv32 not null: also the FP32 copies); cnt: the rows' kept
// counts, boff: the exclusive scan of the keep_count launch's block sums
// (same width); writes the row pointers new_rp[0..rows]
void launch_compact_lump(int width, const CsrView& a, const uint8_t* keep, const int32_t* cnt,
                         const int32_t* boff, int32_t* new_rp, int32_t* new_ci, double* new_v, double* dinv,
                         float* new_v32, float* dinv32, hipStream_t st);

}  // namespace amg355
