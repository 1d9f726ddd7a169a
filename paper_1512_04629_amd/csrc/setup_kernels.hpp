// Device kernels of the hierarchy setup (Section 2, amg_setup: strength ->
// C/F split -> interpolation -> Galerkin product) for gfx950.
//
// Every step reproduces the host setup's arithmetic bit for bit: per-row
// sums run in ascending column order in one thread, and the Galerkin
// products are formed as expand -> stable sort by (row, column) -> ordered
// sums, so each entry's terms are added in the canonical order (ascending
// inner index, first term assigned).  The C/F split is either the
// Ruge-Stueben first pass (computed elsewhere) or PMIS, the parallel
// aggressive coarsening Section 1 cites, in rounds on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace amg355 {

// point states of the C/F split
constexpr int32_t kPtUndecided = 0, kPtC = 1, kPtF = 2;

// error bits of the input check and of the symmetrization
enum SetupError : int {
    kErrRowPtr = 1,          // row_ptr not 0-based, decreasing or not ending at nnz
    kErrColRange = 2,        // column index out of range
    kErrColOrder = 4,        // columns not strictly ascending in a row
    kErrNonFinite = 8,       // NaN or infinite value
    kErrNoDiag = 16,         // no stored diagonal
    kErrDiagSign = 32,       // diagonal not positive
    kErrAsymmetric = 64,     // (j,i) missing or a_ji != a_ij bitwise
    kErrPattern = 128,       // coarse product pattern not structurally symmetric
};

// err[0] |= error bits, err[1] = min offending row (init INT32_MAX)
void launch_validate_csr(int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                         int* err, hipStream_t st);

// strength (negative couplings, -a_ij >= fl(theta max_{k!=i}(-a_ik))): strong
// counts per row, then the pattern and lambda_j = #{i : S_ij} (lam zeroed by
// the caller)
void launch_strength_count(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                           int32_t* cnt, hipStream_t st);
void launch_strength_fill(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                          const int32_t* srp, int32_t* sci, int32_t* lam, hipStream_t st);

// PMIS: weights w_i = lambda_i + u_i with u_i the top 53 bits of output i+1
// of the SplitMix64 stream `seed`; lambda_i = 0 points start as F
void launch_pmis_init(int n, const int32_t* lam, uint64_t seed, double* w, int32_t* state, int32_t* mark,
                      hipStream_t st);
// one round: local maxima among undecided points become C, then undecided
// points depending strongly on a C point become F; *undecided receives the
// number left
void launch_pmis_round(int n, const int32_t* srp, const int32_t* sci, const double* w, int32_t* state,
                       int32_t* mark, int round, int32_t* undecided, hipStream_t st);

// cnt[i] = 1 for C points; after the scan cidx, c_points[cidx[i]] = i
void launch_c_flags(int n, const int32_t* state, int32_t* cnt, hipStream_t st);
void launch_c_points(int n, const int32_t* state, const int32_t* cidx, int32_t* c_points, hipStream_t st);

// direct interpolation: row sizes, then entries
void launch_interp_count(int n, const int32_t* srp, const int32_t* sci, const int32_t* state, int32_t* cnt,
                         hipStream_t st);
void launch_interp_fill(int n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* srp,
                        const int32_t* sci, const int32_t* state, const int32_t* cidx, const int32_t* prp,
                        int32_t* pci, double* pv, hipStream_t st);

// keys (column << row_bits | row) of every entry of a CSR matrix, with values
void launch_transpose_keys(int rows, const int32_t* rp, const int32_t* ci, const double* v, int row_bits,
                           uint64_t* keys, double* vals, hipStream_t st);

// products of a Galerkin step, per row of the left factor:
//   AP: row k of A times P (count = sum over A's row of P's row sizes)
//   PT: fine row k contributes P[k,I] * T[k,J] to (I,J)
void launch_ap_count(int n, const int32_t* arp, const int32_t* aci, const int32_t* prp, int64_t* cnt,
                     hipStream_t st);
void launch_ap_expand(int n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* prp,
                      const int32_t* pci, const double* pv, const int64_t* off, int col_bits, uint64_t* keys,
                      double* vals, hipStream_t st);
void launch_pt_count(int n, const int32_t* prp, const int32_t* trp, int64_t* cnt, hipStream_t st);
void launch_pt_expand(int n, const int32_t* prp, const int32_t* pci, const double* pv, const int32_t* trp,
                      const int32_t* tci, const double* tv, const int64_t* off, int col_bits, uint64_t* keys,
                      double* vals, hipStream_t st);

// sorted (key, value) list -> head flags of equal-key runs
void launch_run_heads(int64_t m, const uint64_t* keys, int64_t* flags, hipStream_t st);
// every run summed in list order (first term assigned): column and value of
// output entry head_index[q] for each head q; the run's key is copied to
// out_keys
void launch_run_sums(int64_t m, const uint64_t* keys, const double* vals, const int64_t* head_index,
                     int col_bits, int32_t* out_ci, double* out_v, uint64_t* out_keys, hipStream_t st);
// row pointer (rows + 1 entries) of m entries whose sorted keys hold the row
// above col_bits
void launch_rowptr_from_keys(int64_t m, const uint64_t* keys, int col_bits, int rows, int32_t* rp,
                             hipStream_t st);
// column and value of each sorted (key, value) pair
void launch_unpack_keys(int64_t m, const uint64_t* keys, const double* vals, int col_bits, int32_t* ci,
                        double* v, hipStream_t st);

// out_ij = (c_ij + c_ji) / 2; err |= kErrPattern where (j,i) is missing
void launch_symmetrize(int n, const int32_t* rp, const int32_t* ci, const double* v, double* out, int* err,
                       hipStream_t st);

// stable ascending sort of (key, value) pairs on bits [0, bits) (keys and
// vals are double buffers; returns which buffer holds the result) and
// exclusive scan of int64 counts (out[m] = total: in has m + 1 entries, the
// last 0); temp == nullptr queries the scratch size
hipError_t sort_pairs(void* temp, size_t& temp_bytes, uint64_t* keys[2], double* vals[2], int64_t m, int bits,
                      int& result, hipStream_t st);
hipError_t scan_counts(void* temp, size_t& temp_bytes, const int64_t* in, int64_t* out, int64_t m,
                       hipStream_t st);

}  // namespace amg355
