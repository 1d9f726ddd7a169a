// Host-side Galerkin setup of the AMG hierarchy (Section 2, amg_setup, run
// without the optional sparsify step as Section 3's sparse_hybrid_setup does).
// The hierarchy is built once on the host in deterministic order and then
// uploaded; everything after setup runs in device kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace amg355 {

struct HostCsr {
    int rows = 0, cols = 0;
    std::vector<int32_t> ptr;   // rows + 1
    std::vector<int32_t> idx;   // sorted ascending per row
    std::vector<double> val;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct HostLevel {
    HostCsr A;                       // Galerkin operator A_l
    HostCsr P;                       // interpolation P_l (empty on the coarsest level)
    HostCsr R;                       // R_l = P_l^T
    std::vector<int32_t> split;      // 1 = C point, 0 = F point (empty on the coarsest level)
    std::vector<int32_t> c_points;   // fine index of each coarse point, ascending
};

struct SetupConfig {
    double theta = 0.25;
    int max_coarse = 49;
    int max_levels = 25;
    // Method of non-Galerkin coarse grids (Section 2.1; the optional sparsify
    // of amg_setup): when not empty, the product forming level l is
    // sparsified right away with tolerance nongalerkin_gamma[l] (0 past the
    // end) and replaces it, so the next level is built from it.
    std::vector<double> nongalerkin_gamma;
};

// Checks the input contract: square, int32 CSR with sorted unique in-range
// columns, finite values, a positive stored diagonal, bitwise symmetry.
bool check_input_matrix(const HostCsr& a, std::string& why);

// Builds the Galerkin hierarchy of a (levels[0].A == a).  Returns false and
// sets why on failure.
bool build_galerkin_hierarchy(const HostCsr& a, const SetupConfig& cfg,
                              std::vector<HostLevel>& levels, std::string& why);

// R = P^T by counting sort (rows of R list the rows of P in ascending order).
HostCsr transpose_csr(const HostCsr& p);

// Ruge-Stueben first-pass C/F split (1 = C) of a strength pattern.
std::vector<int32_t> ruge_stueben_split(const HostCsr& s);

}  // namespace amg355
