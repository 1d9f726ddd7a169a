// Strong-neighbour lumping kernels: one thread per row, every sum and share
// in the order the definition fixes (ascending columns; shares of a target
// in ascending order of their source entry), contraction off.
#include "lump_kernels.hpp"

#include <algorithm>
#include <cmath>

#pragma clang fp contract(off)

namespace amg355 {

namespace {

constexpr int kLB = 256;

int grid_of(int n) { return std::max(1, std::min((n + kLB - 1) / kLB, 16384)); }

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

__device__ inline bool kept_at(const int32_t* rp, const int32_t* ci, const uint8_t* keep, int i, int m) {
    const int q = find_in_row(ci, rp[i], rp[i + 1], m);
    return q >= 0 && keep[q];
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

__global__ void lump_den_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const double* __restrict__ v, const uint8_t* __restrict__ keep,
                                const double* __restrict__ thr, double* __restrict__ den) {
    ROW_LOOP(i, n) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (j == i || keep[p]) continue;
            double d = 0.0;
            for (int r = rp[j]; r < rp[j + 1]; ++r)
                if (strong_at(ci, v, thr, j, r) && kept_at(rp, ci, keep, i, ci[r])) d = d + fabs(v[r]);
            den[p] = d;
        }
    }
}

// row k pulls the shares of the dropped entries (i,j) of the rows i it keeps
// (i = k included), visited in ascending (i, j): the same order in which the
// definition adds them
__global__ void strong_lump_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                   const double* __restrict__ v, const uint8_t* __restrict__ keep,
                                   const double* __restrict__ thr, const double* __restrict__ den,
                                   const int32_t* __restrict__ hrp, const int32_t* __restrict__ hci,
                                   double* __restrict__ hv) {
    ROW_LOOP(k, n) {
        const int hb = hrp[k], he = hrp[k + 1];
        const int dk = find_in_row(hci, hb, he, k);
        if (dk < 0) continue;   // every operator stores its diagonal; never taken
        for (int p = rp[k]; p < rp[k + 1]; ++p) {
            if (!keep[p]) continue;
            const int i = ci[p];
            for (int q = rp[i]; q < rp[i + 1]; ++q) {
                const int j = ci[q];
                if (j == i || keep[q]) continue;
                const double aij = v[q], d = den[q];
                if (i == k) {
                    if (d == 0.0) {
                        hv[dk] = hv[dk] + aij;
                        continue;
                    }
                    for (int r = rp[j]; r < rp[j + 1]; ++r) {
                        if (!(strong_at(ci, v, thr, j, r) && kept_at(rp, ci, keep, k, ci[r]))) continue;
                        const double c = (fabs(v[r]) / d) * aij;
                        const int t = ci[r] == k ? dk : find_in_row(hci, hb, he, ci[r]);
                        if (t >= 0) hv[t] = hv[t] + c;
                    }
                } else {
                    if (d == 0.0) continue;
                    const int r = find_in_row(ci, rp[j], rp[j + 1], k);
                    if (r < 0 || !strong_at(ci, v, thr, j, r)) continue;
                    const double c = (fabs(v[r]) / d) * aij;
                    const int t = find_in_row(hci, hb, he, i);
                    if (t >= 0) hv[t] = hv[t] + c;
                    hv[dk] = hv[dk] - c;
                }
            }
        }
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
    hipLaunchKernelGGL(lump_den_kernel, dim3(grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr, den);
}

void launch_strong_lump(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                        const double* thr, const double* den, const int32_t* hrp, const int32_t* hci, double* hv,
                        hipStream_t st) {
    hipLaunchKernelGGL(strong_lump_kernel, dim3(grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr, den, hrp,
                       hci, hv);
}

}  // namespace amg355
