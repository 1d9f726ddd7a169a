// Strong-neighbour lumping kernels: every sum and share in the order the
// definition fixes (ascending columns; shares of a target in ascending order
// of their source entry), contraction off.  The threshold and the copy run
// one thread per row, the denominators and the shares one wave per row.
#include "lump_kernels.hpp"

#include <algorithm>
#include <cmath>

#pragma clang fp contract(off)

namespace amg355 {

namespace {

constexpr int kLB = 256;
constexpr int kWaves = kLB / 64;

int grid_of(int n) { return std::max(1, std::min((n + kLB - 1) / kLB, 16384)); }
int wave_grid_of(int n) { return std::max(1, std::min((n + kWaves - 1) / kWaves, 65536)); }

#define ROW_LOOP(i, n) for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

__device__ inline int find_in_row(const int32_t* ci, int b, int e, int col) {
    int lo = b, hi = e;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ci[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return (lo < e && ci[lo] == col) ? lo : -1;
}

__device__ inline bool strong_at(const int32_t* ci, const double* v, const double* thr, int j, int r) {
    return ci[r] != j && thr[j] > 0.0 && -v[r] >= thr[j];
}

__global__ void compact_copy_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    const double* __restrict__ v, const uint8_t* __restrict__ keep,
                                    const int32_t* __restrict__ new_rp, int32_t* __restrict__ new_ci,
                                    double* __restrict__ new_v) {
    ROW_LOOP(i, n) {
        int w = new_rp[i];
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (keep[p]) {
                new_ci[w] = ci[p];
                new_v[w] = v[p];
                ++w;
            }
    }
}

__global__ void lump_threshold_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                      const double* __restrict__ v, double theta, double* __restrict__ thr) {
    ROW_LOOP(j, n) {
        double big = 0.0;
        for (int p = rp[j]; p < rp[j + 1]; ++p)
            if (ci[p] != j && -v[p] > big) big = -v[p];
        thr[j] = big > 0.0 ? theta * big : -1.0;
    }
}

// one wave per row i (kWaves per workgroup), lanes over the row's entries
#define WAVE_ROW_LOOP(i, n)                                                                         \
    for (int i = blockIdx.x * kWaves + (int)(threadIdx.x >> 6); i < (n); i += gridDim.x * kWaves)

__global__ void __launch_bounds__(kLB) lump_den_kernel(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const uint8_t* __restrict__ keep,
                                                       const double* __restrict__ thr, double* __restrict__ den) {
    const int lane = threadIdx.x & 63;
    WAVE_ROW_LOOP(i, n) {
        const int ib = rp[i], ie = rp[i + 1];
        for (int p = ib + lane; p < ie; p += 64) {
            const int j = ci[p];
            if (j == i || keep[p]) continue;
            // strong neighbours m of j in ascending order, matched against
            // the ascending columns of row i by a merge walk
            double d = 0.0;
            int w = ib;
            for (int r = rp[j]; r < rp[j + 1]; ++r) {
                if (!strong_at(ci, v, thr, j, r)) continue;
                const int m = ci[r];
                while (w < ie && ci[w] < m) ++w;
                if (w < ie && ci[w] == m && keep[w]) d = d + fabs(v[r]);
            }
            den[p] = d;
        }
    }
}

// Position of column col in the ascending columns ci[w..e), walking w
// forward (a merge against an ascending sequence of col); -1 if absent.
__device__ inline int walk_to(const int32_t* ci, int& w, int e, int col) {
    while (w < e && ci[w] < col) ++w;
    return (w < e && ci[w] == col) ? w : -1;
}

// acc plus the shares the dropped entries (s,j) of row s give to node x, in
// ascending j: (|a_jx| / den) a_sj where (j,x) is strong.  The operator is
// bitwise symmetric, so a_jx is read as a_xj from row x, found by a merge
// walk of row s against row x: no row j is touched.  (s,x) is kept, so x
// belongs to every such W and den > 0.
__device__ inline double pull_row(const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                                  const double* thr, const double* den, int s, int x, double acc) {
    int w = rp[x];
    const int we = rp[x + 1];
    for (int q = rp[s]; q < rp[s + 1]; ++q) {
        const int j = ci[q];
        if (j == s || keep[q]) continue;
        const int r = walk_to(ci, w, we, j);
        if (r < 0) continue;
        const double t = thr[j], ajx = v[r];
        if (t > 0.0 && -ajx >= t) acc = acc + (fabs(ajx) / den[q]) * v[q];
    }
    return acc;
}

// Row k of the lumped operator, one wave.  Kept sets are symmetric, so the
// shares an entry (k,m) receives come from exactly two rows: dropped (k,j)
// sharing with m, and dropped (m,j) sharing with k, added in ascending order
// of the source entry (the lower row first).  (m,k) receives the same shares
// in the same order from the same start value, so one lane per (k,m) with
// m > k adds them serially and writes both entries.  The diagonal receives
// shares from every row it keeps (itself included); the lanes form one chunk
// of 64 entries of a source row at a time and the wave adds the chunk's
// shares in lane order.  Requires a bitwise symmetric operator (every
// Galerkin and non-Galerkin coarse operator is).
__global__ void __launch_bounds__(kLB) strong_lump_kernel(int n, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const double* __restrict__ v,
                                                          const uint8_t* __restrict__ keep,
                                                          const double* __restrict__ thr,
                                                          const double* __restrict__ den,
                                                          const int32_t* __restrict__ hrp,
                                                          const int32_t* __restrict__ hci,
                                                          double* __restrict__ hv) {
    const int lane = threadIdx.x & 63;
    WAVE_ROW_LOOP(k, n) {
        const int hb = hrp[k], he = hrp[k + 1];
        for (int t = hb + lane; t < he; t += 64) {
            const int m = hci[t];
            if (m <= k) continue;
            double acc = pull_row(rp, ci, v, keep, thr, den, k, m, hv[t]);
            acc = pull_row(rp, ci, v, keep, thr, den, m, k, acc);
            hv[t] = acc;
            const int tm = find_in_row(hci, hrp[m], hrp[m + 1], k);
            if (tm >= 0) hv[tm] = acc;   // always found: the kept pattern is symmetric
        }
        const int dk = find_in_row(hci, hb, he, k);
        if (dk < 0) continue;   // every operator stores its diagonal; never taken (uniform over the wave)
        const int kb = rp[k], ke = rp[k + 1];
        double acc = hv[dk];
        for (int p = hb; p < he; ++p) {
            const int s = hci[p];
            const int sb = rp[s], se = rp[s + 1];
            for (int q0 = sb; q0 < se; q0 += 64) {
                const int q = q0 + lane;
                bool has = false;
                double c = 0.0;
                if (q < se && !keep[q]) {
                    const int j = ci[q];
                    const double d = den[q];
                    if (j != s && s == k) {
                        if (d == 0.0) {
                            c = v[q];   // no strong neighbour kept: the whole entry
                            has = true;
                        } else {
                            // the share to k itself, with a_jk = a_kj
                            const double t = thr[j], a = v[q];
                            if (t > 0.0 && -a >= t) {
                                c = (fabs(a) / d) * a;
                                has = true;
                            }
                        }
                    } else if (j != s && d != 0.0) {
                        // the share of (s,j) to k, with a_jk read as a_kj from row k
                        const int r = find_in_row(ci, kb, ke, j);
                        if (r >= 0) {
                            const double t = thr[j], a = v[r];
                            if (t > 0.0 && -a >= t) {
                                c = -((fabs(a) / d) * v[q]);   // a - c == a + (-c) exactly
                                has = true;
                            }
                        }
                    }
                }
                for (uint64_t mask = __ballot(has); mask != 0; mask &= mask - 1)
                    acc = acc + __shfl(c, __builtin_ctzll(mask));
            }
        }
        if (lane == 0) hv[dk] = acc;
    }
}

}  // namespace

void launch_compact_copy(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                         const int32_t* new_rp, int32_t* new_ci, double* new_v, hipStream_t st) {
    hipLaunchKernelGGL(compact_copy_kernel, dim3(grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, new_rp, new_ci,
                       new_v);
}

void launch_lump_threshold(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                           double* thr, hipStream_t st) {
    hipLaunchKernelGGL(lump_threshold_kernel, dim3(grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, theta, thr);
}

void launch_lump_den(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                     const double* thr, double* den, hipStream_t st) {
    hipLaunchKernelGGL(lump_den_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr, den);
}

void launch_strong_lump(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                        const double* thr, const double* den, const int32_t* hrp, const int32_t* hci, double* hv,
                        hipStream_t st) {
    hipLaunchKernelGGL(strong_lump_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr, den, hrp,
                       hci, hv);
}

}  // namespace amg355
