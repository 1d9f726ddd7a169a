// Device kernels of the hierarchy setup (Section 2, amg_setup).  Each kernel
// states the host-setup step it reproduces; the arithmetic of every value is
// the same sequence of IEEE operations in the same order, so the device
// hierarchy is bitwise the host one (for the same C/F split).
#include "setup_kernels.hpp"

#include <algorithm>
#include <climits>

// the order of every floating-point operation is the order written here
#pragma clang fp contract(off)

namespace amg355 {

namespace {

constexpr int kSB = 256;

int grid_of(int64_t n) {
    const int64_t b = (n + kSB - 1) / kSB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

#define GRID_STRIDE(i, n)                                                               \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)(n); \
         i += (int64_t)gridDim.x * blockDim.x)

__device__ inline int64_t find_col(const int32_t* ci, int64_t b, int64_t e, int col) {
    int64_t lo = b, hi = e;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ci[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return (lo < e && ci[lo] == col) ? lo : -1;
}

// ---------------------------------------------------------------------------
// input contract: 0-based non-decreasing row_ptr ending at nnz, in-range
// strictly ascending columns, finite values, positive stored diagonal,
// bitwise symmetry (a_ji stored with the same bits as a_ij)
// ---------------------------------------------------------------------------
__global__ void validate_kernel(int n, int64_t nnz, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ ci, const double* __restrict__ v,
                                int* __restrict__ err) {
    GRID_STRIDE(ii, n) {
        const int i = (int)ii;
        int bits = 0;
        const int64_t b = rp[i], e = rp[i + 1];
        if ((i == 0 && b != 0) || (i == n - 1 && e != nnz) || b < 0 || e < b || e > nnz) {
            bits = kErrRowPtr;
        } else {
            bool diag = false;
            for (int64_t p = b; p < e; ++p) {
                const int j = ci[p];
                if (j < 0 || j >= n) {
                    bits |= kErrColRange;
                    continue;
                }
                if (p > b && j <= ci[p - 1]) bits |= kErrColOrder;
                const double a = v[p];
                if (!isfinite(a)) bits |= kErrNonFinite;
                if (j == i) {
                    diag = true;
                    if (!(a > 0.0)) bits |= kErrDiagSign;
                }
                const int64_t jb = rp[j], je = rp[j + 1];
                if (jb < 0 || je < jb || je > nnz) continue;   // row j reports its own pointers
                const int64_t q = find_col(ci, jb, je, i);
                if (q < 0 || __double_as_longlong(v[q]) != __double_as_longlong(a)) bits |= kErrAsymmetric;
            }
            if (!diag) bits |= kErrNoDiag;
        }
        if (bits) {
            atomicOr(&err[0], bits);
            atomicMin(&err[1], i);
        }
    }
}

// ---------------------------------------------------------------------------
// strength: big = max(0, max_{k!=i} -a_ik); strong iff big > 0 and
// -a_ij >= fl(theta * big), j != i
// ---------------------------------------------------------------------------
__device__ inline bool strength_threshold(int i, int64_t b, int64_t e, const int32_t* ci, const double* v,
                                          double theta, double& thr) {
    double big = 0.0;
    for (int64_t p = b; p < e; ++p)
        if (ci[p] != i) {
            const double t = -v[p];
            big = (big < t) ? t : big;
        }
    thr = theta * big;
    return big > 0.0;
}

__global__ void strength_count_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                      const double* __restrict__ v, double theta, int32_t* __restrict__ cnt) {
    GRID_STRIDE(ii, n) {
        const int i = (int)ii;
        const int64_t b = rp[i], e = rp[i + 1];
        double thr;
        int c = 0;
        if (strength_threshold(i, b, e, ci, v, theta, thr))
            for (int64_t p = b; p < e; ++p) c += (ci[p] != i && -v[p] >= thr);
        cnt[i] = c;
    }
}

__global__ void strength_fill_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const double* __restrict__ v, double theta, const int32_t* __restrict__ srp,
                                     int32_t* __restrict__ sci, int32_t* __restrict__ lam) {
    GRID_STRIDE(ii, n) {
        const int i = (int)ii;
        const int64_t b = rp[i], e = rp[i + 1];
        double thr;
        if (!strength_threshold(i, b, e, ci, v, theta, thr)) continue;
        int64_t w = srp[i];
        for (int64_t p = b; p < e; ++p) {
            const int j = ci[p];
            if (j != i && -v[p] >= thr) {
                sci[w++] = j;
                atomicAdd(&lam[j], 1);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// PMIS
// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k >= 1 of the
// stream seeded with `seed` is the finaliser applied to seed + k * golden
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void pmis_init_kernel(int n, const int32_t* __restrict__ lam, uint64_t seed, double* __restrict__ w,
                                 int32_t* __restrict__ state, int32_t* __restrict__ mark) {
    GRID_STRIDE(i, n) {
        const double u = (double)(splitmix64_at(seed, (uint64_t)i + 1) >> 11) * 0x1p-53;
        w[i] = (double)lam[i] + u;
        state[i] = lam[i] == 0 ? kPtF : kPtUndecided;
        mark[i] = 0;
    }
}

// i beats j: larger weight, equal weights: smaller index
__device__ inline bool beats(const double* w, int i, int j) { return w[i] > w[j] || (w[i] == w[j] && i < j); }

// every strong edge j -> k between undecided points marks its loser
__global__ void pmis_mark_kernel(int n, const int32_t* __restrict__ srp, const int32_t* __restrict__ sci,
                                 const double* __restrict__ w, const int32_t* __restrict__ state,
                                 int32_t* __restrict__ mark, int round, int32_t* __restrict__ undecided) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *undecided = 0;
    GRID_STRIDE(jj, n) {
        const int j = (int)jj;
        if (state[j] != kPtUndecided) continue;
        for (int64_t p = srp[j]; p < srp[j + 1]; ++p) {
            const int k = sci[p];
            if (state[k] != kPtUndecided) continue;
            if (beats(w, j, k)) mark[k] = round;
            else mark[j] = round;
        }
    }
}

__global__ void pmis_select_kernel(int n, int32_t* __restrict__ state, const int32_t* __restrict__ mark,
                                   int round) {
    GRID_STRIDE(i, n) {
        if (state[i] == kPtUndecided && mark[i] != round) state[i] = kPtC;
    }
}

// undecided points that depend strongly on a C point become F; the rest are
// counted.  Only U -> F changes happen here, so the C tests are race free.
__global__ void pmis_fmark_kernel(int n, const int32_t* __restrict__ srp, const int32_t* __restrict__ sci,
                                  int32_t* state, int32_t* __restrict__ undecided) {
    GRID_STRIDE(jj, n) {
        const int j = (int)jj;
        if (state[j] != kPtUndecided) continue;
        bool to_f = false;
        for (int64_t p = srp[j]; p < srp[j + 1] && !to_f; ++p) to_f = state[sci[p]] == kPtC;
        if (to_f) state[j] = kPtF;
        else atomicAdd(undecided, 1);
    }
}

__global__ void c_flags_kernel(int n, const int32_t* __restrict__ state, int32_t* __restrict__ cnt) {
    GRID_STRIDE(i, n) cnt[i] = state[i] == kPtC;
}

__global__ void c_points_kernel(int n, const int32_t* __restrict__ state, const int32_t* __restrict__ cidx,
                                int32_t* __restrict__ c_points) {
    GRID_STRIDE(i, n) {
        if (state[i] == kPtC) c_points[cidx[i]] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// direct interpolation: C rows inject; an F row interpolates from its strong
// C neighbours with w_ij = -(alpha a_ij) / d, alpha = (sum of negative
// off-diagonals) / (sum of a_ij over strong C neighbours), d = a_ii + (sum
// of positive off-diagonals), every sum in ascending column order
// ---------------------------------------------------------------------------
__global__ void interp_count_kernel(int n, const int32_t* __restrict__ srp, const int32_t* __restrict__ sci,
                                    const int32_t* __restrict__ state, int32_t* __restrict__ cnt) {
    GRID_STRIDE(ii, n) {
        const int i = (int)ii;
        if (state[i] == kPtC) {
            cnt[i] = 1;
            continue;
        }
        int c = 0;
        for (int64_t p = srp[i]; p < srp[i + 1]; ++p) c += state[sci[p]] == kPtC;
        cnt[i] = c;
    }
}

__global__ void interp_fill_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                   const double* __restrict__ v, const int32_t* __restrict__ srp,
                                   const int32_t* __restrict__ sci, const int32_t* __restrict__ state,
                                   const int32_t* __restrict__ cidx, const int32_t* __restrict__ prp,
                                   int32_t* __restrict__ pci, double* __restrict__ pv) {
    GRID_STRIDE(ii, n) {
        const int i = (int)ii;
        int64_t w = prp[i];
        if (state[i] == kPtC) {
            pci[w] = cidx[i];
            pv[w] = 1.0;
            continue;
        }
        if (prp[i + 1] == w) continue;
        const int64_t b = rp[i], e = rp[i + 1];
        double dsum = 0.0;
        for (int64_t p = b; p < e; ++p)
            if (ci[p] == i) dsum = v[p];
        double neg = 0.0, strong_c = 0.0;
        for (int64_t p = b; p < e; ++p) {
            if (ci[p] == i) continue;
            const double x = v[p];
            if (x < 0.0) neg = neg + x;
            else if (x > 0.0) dsum = dsum + x;
        }
        int64_t q = b;
        for (int64_t s = srp[i]; s < srp[i + 1]; ++s) {
            const int j = sci[s];
            while (ci[q] < j) ++q;
            if (state[j] == kPtC) strong_c = strong_c + v[q];
        }
        const double alpha = neg / strong_c;
        q = b;
        for (int64_t s = srp[i]; s < srp[i + 1]; ++s) {
            const int j = sci[s];
            while (ci[q] < j) ++q;
            if (state[j] != kPtC) continue;
            const double t = alpha * v[q];
            pci[w] = cidx[j];
            pv[w] = -t / dsum;
            ++w;
        }
    }
}

// ---------------------------------------------------------------------------
// transposes and products through sorted keys (row << col_bits | col)
// ---------------------------------------------------------------------------
__global__ void transpose_keys_kernel(int rows, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                      const double* __restrict__ v, int row_bits, uint64_t* __restrict__ keys,
                                      double* __restrict__ vals) {
    GRID_STRIDE(ii, rows) {
        const int i = (int)ii;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            keys[p] = ((uint64_t)(uint32_t)ci[p] << row_bits) | (uint64_t)(uint32_t)i;
            vals[p] = v[p];
        }
    }
}

// cnt has n + 1 entries; the last is 0 so that the exclusive scan ends on
// the total
__global__ void ap_count_kernel(int n, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                const int32_t* __restrict__ prp, int64_t* __restrict__ cnt) {
    GRID_STRIDE(kk, (int64_t)n + 1) {
        const int k = (int)kk;
        int64_t c = 0;
        if (k < n)
            for (int64_t p = arp[k]; p < arp[k + 1]; ++p) c += prp[aci[p] + 1] - prp[aci[p]];
        cnt[k] = c;
    }
}

// T = A P: row k lists, for each l of A's row in ascending order, the terms
// a_kl p_lJ over P's row l
__global__ void ap_expand_kernel(int n, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                 const double* __restrict__ av, const int32_t* __restrict__ prp,
                                 const int32_t* __restrict__ pci, const double* __restrict__ pv,
                                 const int64_t* __restrict__ off, int col_bits, uint64_t* __restrict__ keys,
                                 double* __restrict__ vals) {
    GRID_STRIDE(kk, n) {
        const int k = (int)kk;
        int64_t o = off[k];
        const uint64_t row = (uint64_t)(uint32_t)k << col_bits;
        for (int64_t p = arp[k]; p < arp[k + 1]; ++p) {
            const int l = aci[p];
            const double a = av[p];
            for (int64_t q = prp[l]; q < prp[l + 1]; ++q) {
                keys[o] = row | (uint64_t)(uint32_t)pci[q];
                vals[o] = a * pv[q];
                ++o;
            }
        }
    }
}

__global__ void pt_count_kernel(int n, const int32_t* __restrict__ prp, const int32_t* __restrict__ trp,
                                int64_t* __restrict__ cnt) {
    GRID_STRIDE(kk, (int64_t)n + 1) {
        const int k = (int)kk;
        cnt[k] = k < n ? (int64_t)(prp[k + 1] - prp[k]) * (int64_t)(trp[k + 1] - trp[k]) : 0;
    }
}

// C = P^T T: fine row k gives the terms p_kI t_kJ; listing the fine rows in
// ascending order makes the terms of each (I, J) ascend in k
__global__ void pt_expand_kernel(int n, const int32_t* __restrict__ prp, const int32_t* __restrict__ pci,
                                 const double* __restrict__ pv, const int32_t* __restrict__ trp,
                                 const int32_t* __restrict__ tci, const double* __restrict__ tv,
                                 const int64_t* __restrict__ off, int col_bits, uint64_t* __restrict__ keys,
                                 double* __restrict__ vals) {
    GRID_STRIDE(kk, n) {
        const int k = (int)kk;
        int64_t o = off[k];
        for (int64_t p = prp[k]; p < prp[k + 1]; ++p) {
            const uint64_t row = (uint64_t)(uint32_t)pci[p] << col_bits;
            const double x = pv[p];
            for (int64_t q = trp[k]; q < trp[k + 1]; ++q) {
                keys[o] = row | (uint64_t)(uint32_t)tci[q];
                vals[o] = x * tv[q];
                ++o;
            }
        }
    }
}

// flags has m + 1 entries (the last 0)
__global__ void run_heads_kernel(int64_t m, const uint64_t* __restrict__ keys, int64_t* __restrict__ flags) {
    GRID_STRIDE(q, m + 1) flags[q] = q < m && (q == 0 || keys[q] != keys[q - 1]);
}

__global__ void run_sums_kernel(int64_t m, const uint64_t* __restrict__ keys, const double* __restrict__ vals,
                                const int64_t* __restrict__ head_index, int col_bits, int32_t* __restrict__ out_ci,
                                double* __restrict__ out_v, uint64_t* __restrict__ out_keys) {
    const uint64_t mask = (1ull << col_bits) - 1;
    GRID_STRIDE(q, m) {
        const uint64_t key = keys[q];
        if (q > 0 && keys[q - 1] == key) continue;
        double sum = vals[q];
        for (int64_t r = q + 1; r < m && keys[r] == key; ++r) sum = sum + vals[r];
        const int64_t s = head_index[q];
        out_ci[s] = (int32_t)(key & mask);
        out_v[s] = sum;
        out_keys[s] = key;
    }
}

__global__ void rowptr_from_keys_kernel(int64_t m, const uint64_t* __restrict__ keys, int col_bits, int rows,
                                        int32_t* __restrict__ rp) {
    if (m == 0) {
        GRID_STRIDE(c, (int64_t)rows + 1) rp[c] = 0;
        return;
    }
    GRID_STRIDE(q, m) {
        const int64_t r = (int64_t)(keys[q] >> col_bits);
        const int64_t prev = q == 0 ? -1 : (int64_t)(keys[q - 1] >> col_bits);
        for (int64_t c = prev + 1; c <= r; ++c) rp[c] = (int32_t)q;
        if (q == m - 1)
            for (int64_t c = r + 1; c <= rows; ++c) rp[c] = (int32_t)m;
    }
}

__global__ void unpack_keys_kernel(int64_t m, const uint64_t* __restrict__ keys, const double* __restrict__ vals,
                                   int col_bits, int32_t* __restrict__ ci, double* __restrict__ v) {
    const uint64_t mask = (1ull << col_bits) - 1;
    GRID_STRIDE(q, m) {
        ci[q] = (int32_t)(keys[q] & mask);
        v[q] = vals[q];
    }
}

__global__ void symmetrize_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const double* __restrict__ v, double* __restrict__ out, int* __restrict__ err) {
    GRID_STRIDE(ii, n) {
        const int i = (int)ii;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            const int64_t q = find_col(ci, rp[j], rp[j + 1], i);
            if (q < 0) {
                atomicOr(err, (int)kErrPattern);
                out[p] = v[p];
                continue;
            }
            out[p] = 0.5 * (v[p] + v[q]);
        }
    }
}

}  // namespace

void launch_validate_csr(int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v, int* err,
                         hipStream_t st) {
    hipLaunchKernelGGL(validate_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, nnz, rp, ci, v, err);
}

void launch_strength_count(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                           int32_t* cnt, hipStream_t st) {
    hipLaunchKernelGGL(strength_count_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, rp, ci, v, theta, cnt);
}

void launch_strength_fill(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                          const int32_t* srp, int32_t* sci, int32_t* lam, hipStream_t st) {
    hipLaunchKernelGGL(strength_fill_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, rp, ci, v, theta, srp, sci,
                       lam);
}

void launch_pmis_init(int n, const int32_t* lam, uint64_t seed, double* w, int32_t* state, int32_t* mark,
                      hipStream_t st) {
    hipLaunchKernelGGL(pmis_init_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, lam, seed, w, state, mark);
}

void launch_pmis_round(int n, const int32_t* srp, const int32_t* sci, const double* w, int32_t* state,
                       int32_t* mark, int round, int32_t* undecided, hipStream_t st) {
    hipLaunchKernelGGL(pmis_mark_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, srp, sci, w, state, mark, round,
                       undecided);
    hipLaunchKernelGGL(pmis_select_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, state, mark, round);
    hipLaunchKernelGGL(pmis_fmark_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, srp, sci, state, undecided);
}

void launch_c_flags(int n, const int32_t* state, int32_t* cnt, hipStream_t st) {
    hipLaunchKernelGGL(c_flags_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, state, cnt);
}

void launch_c_points(int n, const int32_t* state, const int32_t* cidx, int32_t* c_points, hipStream_t st) {
    hipLaunchKernelGGL(c_points_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, state, cidx, c_points);
}

void launch_interp_count(int n, const int32_t* srp, const int32_t* sci, const int32_t* state, int32_t* cnt,
                         hipStream_t st) {
    hipLaunchKernelGGL(interp_count_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, srp, sci, state, cnt);
}

void launch_interp_fill(int n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* srp,
                        const int32_t* sci, const int32_t* state, const int32_t* cidx, const int32_t* prp,
                        int32_t* pci, double* pv, hipStream_t st) {
    hipLaunchKernelGGL(interp_fill_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, rp, ci, v, srp, sci, state, cidx,
                       prp, pci, pv);
}

void launch_transpose_keys(int rows, const int32_t* rp, const int32_t* ci, const double* v, int row_bits,
                           uint64_t* keys, double* vals, hipStream_t st) {
    hipLaunchKernelGGL(transpose_keys_kernel, dim3(grid_of(rows)), dim3(kSB), 0, st, rows, rp, ci, v, row_bits,
                       keys, vals);
}

void launch_ap_count(int n, const int32_t* arp, const int32_t* aci, const int32_t* prp, int64_t* cnt,
                     hipStream_t st) {
    hipLaunchKernelGGL(ap_count_kernel, dim3(grid_of((int64_t)n + 1)), dim3(kSB), 0, st, n, arp, aci, prp, cnt);
}

void launch_ap_expand(int n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* prp,
                      const int32_t* pci, const double* pv, const int64_t* off, int col_bits, uint64_t* keys,
                      double* vals, hipStream_t st) {
    hipLaunchKernelGGL(ap_expand_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, arp, aci, av, prp, pci, pv, off,
                       col_bits, keys, vals);
}

void launch_pt_count(int n, const int32_t* prp, const int32_t* trp, int64_t* cnt, hipStream_t st) {
    hipLaunchKernelGGL(pt_count_kernel, dim3(grid_of((int64_t)n + 1)), dim3(kSB), 0, st, n, prp, trp, cnt);
}

void launch_pt_expand(int n, const int32_t* prp, const int32_t* pci, const double* pv, const int32_t* trp,
                      const int32_t* tci, const double* tv, const int64_t* off, int col_bits, uint64_t* keys,
                      double* vals, hipStream_t st) {
    hipLaunchKernelGGL(pt_expand_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, prp, pci, pv, trp, tci, tv, off,
                       col_bits, keys, vals);
}

void launch_run_heads(int64_t m, const uint64_t* keys, int64_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(run_heads_kernel, dim3(grid_of(m + 1)), dim3(kSB), 0, st, m, keys, flags);
}

void launch_run_sums(int64_t m, const uint64_t* keys, const double* vals, const int64_t* head_index,
                     int col_bits, int32_t* out_ci, double* out_v, uint64_t* out_keys, hipStream_t st) {
    hipLaunchKernelGGL(run_sums_kernel, dim3(grid_of(m)), dim3(kSB), 0, st, m, keys, vals, head_index, col_bits,
                       out_ci, out_v, out_keys);
}

void launch_rowptr_from_keys(int64_t m, const uint64_t* keys, int col_bits, int rows, int32_t* rp,
                             hipStream_t st) {
    hipLaunchKernelGGL(rowptr_from_keys_kernel, dim3(grid_of(std::max<int64_t>(m, (int64_t)rows + 1))),
                       dim3(kSB), 0, st, m, keys, col_bits, rows, rp);
}

void launch_unpack_keys(int64_t m, const uint64_t* keys, const double* vals, int col_bits, int32_t* ci,
                        double* v, hipStream_t st) {
    hipLaunchKernelGGL(unpack_keys_kernel, dim3(grid_of(m)), dim3(kSB), 0, st, m, keys, vals, col_bits, ci, v);
}

void launch_symmetrize(int n, const int32_t* rp, const int32_t* ci, const double* v, double* out, int* err,
                       hipStream_t st) {
    hipLaunchKernelGGL(symmetrize_kernel, dim3(grid_of(n)), dim3(kSB), 0, st, n, rp, ci, v, out, err);
}

namespace {

// ---------------------------------------------------------------------------
// Exclusive scan of int64 counts and a stable LSD radix sort of (key, value)
// pairs: the sort that groups the Galerkin product's terms by (row, column)
// and the transpose's entries by (column, row).
// ---------------------------------------------------------------------------

// scan: 4,096 entries per block (256 threads, 16 consecutive entries each)
constexpr int kScanPer = 16;
constexpr int kScanTile64 = kSB * kScanPer;

// block-wide exclusive scan of one int64 per thread (wave shuffles, then the
// four wave totals through LDS); *total receives the block's sum
__device__ __forceinline__ int64_t block_exclusive_scan64(int64_t v, int64_t* wsum, int64_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kSB / 64; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    *total = all;
    __syncthreads();
    return before + incl - v;
}

__global__ __launch_bounds__(kSB) void scan64_reduce_kernel(int64_t n, const int64_t* __restrict__ in,
                                                            int64_t* __restrict__ bsum) {
    __shared__ int64_t wsum[kSB / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile64;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + (int64_t)k * kSB + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_exclusive_scan64(s, wsum, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// the block sums, scanned in place by one workgroup of 1,024 threads, each
// owning a contiguous range
__global__ __launch_bounds__(1024) void scan64_blocks_kernel(int64_t nb, int64_t* bsum) {
    __shared__ int64_t part[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = threadIdx.x * per, hi = std::min<int64_t>(nb, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += bsum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t t = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t v = bsum[i];
        bsum[i] = run;
        run += v;
    }
}

// each thread scans its 16 consecutive entries after the block-wide scan of
// the thread sums; entries staged through LDS so that both the loads and the
// stores are coalesced
__global__ __launch_bounds__(kSB) void scan64_apply_kernel(int64_t n, const int64_t* __restrict__ in,
                                                           const int64_t* __restrict__ boff,
                                                           int64_t* __restrict__ out) {
    __shared__ int64_t tile[kScanTile64 + kScanTile64 / 32];
    __shared__ int64_t wsum[kSB / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile64;
    // padded index: one spare slot every 32 entries keeps a thread's 16
    // consecutive entries off each other's LDS banks
    auto at = [](int i) { return i + (i >> 5); };
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = k * kSB + threadIdx.x;
        tile[at(i)] = base + i < n ? in[base + i] : 0;
    }
    __syncthreads();
    int64_t v[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = tile[at(threadIdx.x * kScanPer + k)];
        s += v[k];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan64(s, wsum, &tot) + boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        tile[at(threadIdx.x * kScanPer + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = k * kSB + threadIdx.x;
        if (base + i < n) out[base + i] = tile[at(i)];
    }
}

int64_t scan64_blocks(int64_t n) { return std::max<int64_t>(1, (n + kScanTile64 - 1) / kScanTile64); }

void launch_scan64(int64_t n, const int64_t* in, int64_t* out, int64_t* bsum, hipStream_t st) {
    const int64_t nb = scan64_blocks(n);
    hipLaunchKernelGGL(scan64_reduce_kernel, dim3((unsigned)nb), dim3(kSB), 0, st, n, in, bsum);
    hipLaunchKernelGGL(scan64_blocks_kernel, dim3(1), dim3(1024), 0, st, nb, bsum);
    hipLaunchKernelGGL(scan64_apply_kernel, dim3((unsigned)nb), dim3(kSB), 0, st, n, in, bsum, out);
}

// radix sort: 8-bit digits, 4,096 pairs per block (16 rounds of 256, pair
// r * 256 + t of the block held by thread t), so that a block's pairs in
// round order are its pairs in input order
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixRounds = 16;
constexpr int kRadixTile = kSB * kRadixRounds;
static_assert(kRadixBins == kSB, "one digit per thread in the offset steps");

// lanes of this wave holding the same digit (lanes with valid = false take
// part in no group); eight ballots, one per digit bit
__device__ __forceinline__ uint64_t same_digit_lanes(int d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t ones = __ballot((d >> b) & 1);
        peers &= ((d >> b) & 1) ? ones : ~ones;
    }
    return peers;
}

__device__ __forceinline__ uint64_t lanes_below() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}

// per-block digit counts, digit-major: cnt[d * nb + block]
__global__ __launch_bounds__(kSB) void radix_count_kernel(int64_t m, int shift, const uint64_t* __restrict__ keys,
                                                          int64_t* __restrict__ cnt, int64_t nb) {
    __shared__ int hist[kRadixBins];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    uint64_t k[kRadixRounds];
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t e = base + (int64_t)r * kSB + threadIdx.x;
        k[r] = e < m ? keys[e] : 0;
    }
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const bool valid = base + (int64_t)r * kSB + threadIdx.x < m;
        const int d = (int)((k[r] >> shift) & (kRadixBins - 1));
        const uint64_t peers = same_digit_lanes(d, valid);
        // the lowest lane of each group adds the group's size
        if (valid && (peers & lanes_below()) == 0) atomicAdd(&hist[d], __popcll(peers));
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * nb + blockIdx.x] = hist[threadIdx.x];
}

// block-wide exclusive scan of one int per thread (kSB threads)
__device__ __forceinline__ int block_exclusive_scan_i32(int v, int* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0;
#pragma unroll
    for (int k = 0; k < kSB / 64; ++k)
        if (k < w) before += wsum[k];
    __syncthreads();
    return before + incl - v;
}

// stable scatter.  Pair (r, t) of the block (held by thread t in round r)
// takes slot tstart[d] + (pairs of digit d in earlier rounds) + (in earlier
// waves of this round) + (in lower lanes of its wave) of the block's tile,
// tstart the block's exclusive scan of its digit counts, so that the slots
// hold the tile's pairs sorted stably by digit.  The pairs are staged in LDS
// in slot order, keys and then values, and written out slot by slot: slot q
// of digit d goes to first[d] + q - tstart[d], so consecutive threads write
// consecutive positions of one digit's run.
__global__ __launch_bounds__(kSB) void radix_scatter_kernel(int64_t m, int shift,
                                                            const uint64_t* __restrict__ kin,
                                                            const double* __restrict__ vin,
                                                            uint64_t* __restrict__ kout,
                                                            double* __restrict__ vout,
                                                            const int64_t* __restrict__ cnt,
                                                            const int64_t* __restrict__ first, int64_t nb) {
    constexpr int kWaves = kSB / 64;
    __shared__ int next[kRadixBins];              // next free slot per digit
    __shared__ int wcnt[kWaves][kRadixBins];      // this round's count per wave and digit
    __shared__ int wpos[kWaves][kRadixBins];      // this round's first slot per wave and digit
    __shared__ int64_t gbase[kRadixBins];         // output position of slot 0 of each digit
    __shared__ int wsum[kWaves];
    __shared__ uint64_t stage[kRadixTile];
    const int t = threadIdx.x, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    uint64_t k[kRadixRounds];
    double v[kRadixRounds];
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t e = base + (int64_t)r * kSB + t;
        k[r] = e < m ? kin[e] : 0;
        v[r] = e < m ? vin[e] : 0.0;
    }
    const int64_t ci = (int64_t)t * nb + blockIdx.x;
    const int tstart = block_exclusive_scan_i32((int)cnt[ci], wsum);
    next[t] = tstart;
    gbase[t] = first[ci] - tstart;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) wcnt[q][t] = 0;
    __syncthreads();
    int slot[kRadixRounds];
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const bool valid = base + (int64_t)r * kSB + t < m;
        const int d = (int)((k[r] >> shift) & (kRadixBins - 1));
        const uint64_t peers = same_digit_lanes(d, valid);
        const int rank = __popcll(peers & lanes_below());
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        {
            // thread t owns digit t: first slots of its waves, then clear
            int p = next[t];
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                wpos[q][t] = p;
                p += wcnt[q][t];
                wcnt[q][t] = 0;
            }
            next[t] = p;
        }
        __syncthreads();
        slot[r] = valid ? wpos[w][d] + rank : -1;
    }
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r)
        if (slot[r] >= 0) stage[slot[r]] = k[r];
    __syncthreads();
    const int here = (int)min<int64_t>(kRadixTile, m - base);
    int dq[kRadixRounds];
#pragma unroll
    for (int q = 0; q < kRadixRounds; ++q) {
        const int idx = q * kSB + t;
        dq[q] = 0;
        if (idx < here) {
            const uint64_t key = stage[idx];
            dq[q] = (int)((key >> shift) & (kRadixBins - 1));
            kout[gbase[dq[q]] + idx] = key;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r)
        if (slot[r] >= 0) stage[slot[r]] = __double_as_longlong(v[r]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRadixRounds; ++q) {
        const int idx = q * kSB + t;
        if (idx < here) vout[gbase[dq[q]] + idx] = __longlong_as_double((long long)stage[idx]);
    }
}

size_t align_up(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

hipError_t sort_pairs(void* temp, size_t& temp_bytes, uint64_t* keys[2], double* vals[2], int64_t m, int bits,
                      int& result, hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, (m + kRadixTile - 1) / kRadixTile);
    const int64_t ncnt = nb * kRadixBins;
    const size_t cnt_bytes = align_up(sizeof(int64_t) * (size_t)ncnt);
    const size_t need = 2 * cnt_bytes + align_up(sizeof(int64_t) * (size_t)scan64_blocks(ncnt));
    const int passes = (std::max(bits, 0) + kRadixBits - 1) / kRadixBits;
    result = passes & 1;
    if (temp == nullptr) {
        temp_bytes = need;
        return hipSuccess;
    }
    if (temp_bytes < need) return hipErrorInvalidValue;
    if (m <= 0) return hipSuccess;
    if (nb > INT_MAX) return hipErrorInvalidValue;
    int64_t* cnt = static_cast<int64_t*>(temp);
    int64_t* first = reinterpret_cast<int64_t*>(static_cast<char*>(temp) + cnt_bytes);
    int64_t* bsum = reinterpret_cast<int64_t*>(static_cast<char*>(temp) + 2 * cnt_bytes);
    for (int p = 0; p < passes; ++p) {
        const int src = p & 1, dst = src ^ 1, shift = p * kRadixBits;
        hipLaunchKernelGGL(radix_count_kernel, dim3((unsigned)nb), dim3(kSB), 0, st, m, shift, keys[src], cnt, nb);
        launch_scan64(ncnt, cnt, first, bsum, st);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kSB), 0, st, m, shift, keys[src],
                           vals[src], keys[dst], vals[dst], cnt, first, nb);
    }
    return hipGetLastError();
}

hipError_t scan_counts(void* temp, size_t& temp_bytes, const int64_t* in, int64_t* out, int64_t m,
                       hipStream_t st) {
    const int64_t n = m + 1;
    const size_t need = align_up(sizeof(int64_t) * (size_t)scan64_blocks(n));
    if (temp == nullptr) {
        temp_bytes = need;
        return hipSuccess;
    }
    if (temp_bytes < need || scan64_blocks(n) > INT_MAX) return hipErrorInvalidValue;
    launch_scan64(n, in, out, static_cast<int64_t*>(temp), st);
    return hipGetLastError();
}

}  // namespace amg355
