// Strong-neighbour lumping of a sparsified operator (Algorithm 3, second
// loop): a dropped entry (i,j) is shared among the strong neighbours m of j
// that row i keeps, in proportion |a_jm|; each share c is added to (i,m)
// and (m,i) and subtracted from (m,m) (added once to (i,i) when m = i); with
// no such neighbour the entry goes to the diagonal.  Every entry adds its
// shares in ascending order of the dropped entry they come from, so the
// result is symmetric bit for bit and independent of the launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amg355 {

// Launch shapes of the lumping kernels; every choice gives the same bits.
// Rows of mean length >= wide_mean_row run a workgroup per row with the row
// staged in LDS (default 0: every level; it was the faster on every level of
// the 3D Poisson hierarchies measured, 34 to 108 entries a row), shorter
// ones a wave per row.  Denominators: a wave per row with its own LDS stage
// on levels of at least 16,384 rows of fewer than 80 entries on average, or,
// if den_wave_mean_row >= 0, wherever mean_row < den_wave_mean_row.  The
// share kernel's workgroups have 1,024 threads on levels of fewer than
// small_rows rows (measured on 3D Poisson: 821 and 129 rows 263 -> 156 and
// 141 -> 90 us; 5,191 rows 372 -> 542 us), 256 otherwise.
struct LumpShapes {
    double wide_mean_row = 0.0;
    double den_wave_mean_row = -1.0;
    int small_rows = 4096;
};

// kept entries of a (keep flags per entry) copied unchanged into the
// pattern new_rp / new_ci / new_v (new_rp: scan of the kept counts)
void launch_compact_copy(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                         const int32_t* new_rp, int32_t* new_ci, double* new_v, hipStream_t st);
// thr[j] = theta * max_{m != j}(-a_jm), or -1 if that maximum is not positive
// (the strength of the setup: (j,m) strong iff m != j and -a_jm >= thr[j] > 0)
void launch_lump_threshold(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                           double* thr, hipStream_t st);
// den[p] for every dropped off-diagonal entry p = (i,j): the sum, in
// ascending m, of |a_jm| over m strong for j and kept in row i (0: none)
void launch_lump_den(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                     const double* thr, double* den, double mean_row, const LumpShapes& ls, hipStream_t st);
// adds every row's shares to the copied kept entries hrp / hci / hv; a must
// be bitwise symmetric with a symmetric keep set (a_jm is read as a_mj).
// Launch shapes as LumpShapes selects.
void launch_strong_lump(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                        const double* thr, const double* den, const int32_t* hrp, const int32_t* hci, double* hv,
                        double mean_row, const LumpShapes& ls, hipStream_t st);

}  // namespace amg355
