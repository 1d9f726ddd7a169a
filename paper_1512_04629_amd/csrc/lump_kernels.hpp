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
                     const double* thr, double* den, double mean_row, hipStream_t st);
// adds every row's shares to the copied kept entries hrp / hci / hv; a must
// be bitwise symmetric with a symmetric keep set (a_jm is read as a_mj).
// Both launches run a workgroup per row with the row staged in LDS, or one
// wave per row when mean_row (nnz / n) is below the threshold that the
// environment variable AMG_LUMP_WIDE_ROW sets (default 0: never); the
// denominators of levels with at least 16,384 rows of fewer than 80 entries
// on average (the environment variable AMG_LUMP_DEN_WAVE_ROW replaces both
// conditions by mean_row below its value) run a wave per row with its own
// LDS stage; the share kernel's workgroups have 1,024 threads on levels of
// fewer than 4,096 rows (the environment variable AMG_LUMP_SMALL_ROWS
// overrides the bound), 256 otherwise.  The same bits every way.
void launch_strong_lump(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                        const double* thr, const double* den, const int32_t* hrp, const int32_t* hci, double* hv,
                        double mean_row, hipStream_t st);

}  // namespace amg355
