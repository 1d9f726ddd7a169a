// Hybrid Gauss-Seidel sweep: the rows of a block in order, each row's sum in
// ascending column order (the order and operations of the definition, so the
// result is the CPU's bit for bit).  One thread per block, reading global
// memory, or, for blocks of up to 256 rows, a workgroup per chunk of blocks
// with the terms staged in LDS.
#include "relax_kernels.hpp"

#include <algorithm>

#pragma clang fp contract(off)

namespace amg355 {

namespace {

template <bool FORWARD>
__device__ inline void gs_block_rows(int r0, int r1, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const double* __restrict__ v, const double* __restrict__ b,
                                     const double* __restrict__ xold, double* xnew);

template <bool FORWARD>
__global__ __launch_bounds__(256) void hybrid_gs_kernel(int n, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const double* __restrict__ v,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ xold, double* xnew,
                                                        int block) {
    const int64_t nblk = ((int64_t)n + block - 1) / block;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nblk;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r0 = (int)(t * block);
        const int r1 = (int)std::min<int64_t>((int64_t)r0 + block, n);
        gs_block_rows<FORWARD>(r0, r1, rp, ci, v, b, xold, xnew);
    }
}

// Staged form for blocks of at most kGsMaxRows rows.  A workgroup owns a chunk
// of R consecutive rows (whole blocks).  First all its threads turn the
// chunk's entries into terms in LDS with coalesced loads: the product
// a_ij xold_j for a term with an old value (rounded exactly as the sweep
// rounds it), a_ij and the chunk-local row of j for a term with a new value,
// the diagonal marked.  Then one lane per block runs the block's rows in
// order from LDS, subtracting the terms in ascending column order: the same
// operations in the same order as hybrid_gs_kernel.  A chunk whose entries do
// not fit takes the per-block loop of hybrid_gs_kernel.
// Largest block the staged form takes (at most kGsMaxRows).  On the 128^3
// Poisson hierarchy it is faster over whole solves for every block size up
// to 256 rows, although on the finest level alone blocks of 64 rows and more
// sweep faster in the per-block kernel.
#ifndef AMG_GS_STAGED_MAX
#define AMG_GS_STAGED_MAX 256
#endif
constexpr int kGsThreads = 256;
constexpr int kGsCap = 3072;      // staged terms per chunk
constexpr int kGsMaxRows = 256;   // rows per chunk
constexpr int16_t kGsDiag = -2, kGsOld = -1;

template <bool FORWARD>
__device__ inline void gs_block_rows(int r0, int r1, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const double* __restrict__ v, const double* __restrict__ b,
                                     const double* __restrict__ xold, double* xnew) {
    int last = -1;
    double last_x = 0.0;
    for (int k = 0; k < r1 - r0; ++k) {
        const int i = FORWARD ? r0 + k : r1 - 1 - k;
        double s = b[i], d = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (j == i) {
                d = v[p];
                continue;
            }
            const bool visited = j >= r0 && j < r1 && (FORWARD ? j < i : j > i);
            const double y = visited ? (j == last ? last_x : xnew[j]) : xold[j];
            s = s - v[p] * y;
        }
        const double xi = s / d;
        xnew[i] = xi;
        last = i;
        last_x = xi;
    }
}

template <bool FORWARD>
__global__ __launch_bounds__(kGsThreads) void hybrid_gs_staged_kernel(int n, const int32_t* __restrict__ rp,
                                                                      const int32_t* __restrict__ ci,
                                                                      const double* __restrict__ v,
                                                                      const double* __restrict__ b,
                                                                      const double* __restrict__ xold,
                                                                      double* xnew, int block, int R) {
    __shared__ double term[kGsCap];
    __shared__ int16_t tag[kGsCap];
    __shared__ uint8_t rowid[kGsCap];   // chunk-local row of each staged entry
    __shared__ int32_t lrp[kGsMaxRows + 1];
    __shared__ double lb[kGsMaxRows], ly[kGsMaxRows];
    const int nchunk = (n + R - 1) / R;
    for (int c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const int r0 = c * R, r1 = min(r0 + R, n), nr = r1 - r0;
        const int p0 = rp[r0], p1 = rp[r1];
        const int nb = (nr + block - 1) / block;
        if (p1 - p0 > kGsCap) {   // uniform over the workgroup
            for (int k = threadIdx.x; k < nb; k += blockDim.x)
                gs_block_rows<FORWARD>(r0 + k * block, min(r0 + (k + 1) * block, r1), rp, ci, v, b, xold, xnew);
            continue;
        }
        for (int t = threadIdx.x; t <= nr; t += blockDim.x) lrp[t] = rp[r0 + t] - p0;
        for (int t = threadIdx.x; t < nr; t += blockDim.x) lb[t] = b[r0 + t];
        __syncthreads();
        for (int t = threadIdx.x; t < nr; t += blockDim.x)
            for (int q = lrp[t]; q < lrp[t + 1]; ++q) rowid[q] = (uint8_t)t;
        __syncthreads();
        for (int q = threadIdx.x; q < p1 - p0; q += blockDim.x) {
            const int lo = rowid[q];
            const int i = r0 + lo;
            const int j = ci[p0 + q];
            const double a = v[p0 + q];
            if (j == i) {
                tag[q] = kGsDiag;
                term[q] = a;
                continue;
            }
            const int bs = r0 + (lo / block) * block;
            const int be = min(bs + block, r1);
            if (j >= bs && j < be && (FORWARD ? j < i : j > i)) {
                tag[q] = (int16_t)(j - r0);
                term[q] = a;
            } else {
                tag[q] = kGsOld;
                term[q] = a * xold[j];
            }
        }
        __syncthreads();
        // the chains are serial: let their wave issue ahead of the other
        // workgroups' staging waves on the same SIMD
        const bool chain_wave = (int)(threadIdx.x & ~63) < nb;
        if (chain_wave) __builtin_amdgcn_s_setprio(3);
        for (int k = threadIdx.x; k < nb; k += blockDim.x) {
            const int b0 = k * block, b1 = min(b0 + block, nr);
            int prev = -1;          // the row visited last: its value stays in a register
            double prev_x = 0.0;
            for (int s = 0; s < b1 - b0; ++s) {
                const int il = FORWARD ? b0 + s : b1 - 1 - s;
                double acc = lb[il], d = 0.0;
                for (int q0 = lrp[il], qe = lrp[il + 1]; q0 < qe; q0 += 8) {
                    // a group of up to 8 terms: the staged values first, then
                    // the new values they need, then the subtractions in order
                    double tv[8], yv[8];
                    int tg[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const bool ok = q0 + u < qe;
                        tg[u] = ok ? tag[q0 + u] : kGsOld;
                        tv[u] = ok ? term[q0 + u] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int f = tg[u];
                        yv[u] = f >= 0 ? (f == prev ? prev_x : ly[f]) : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        if (q0 + u >= qe) break;
                        const int f = tg[u];
                        if (f == kGsDiag) {
                            d = tv[u];
                            continue;
                        }
                        acc = acc - (f >= 0 ? tv[u] * yv[u] : tv[u]);
                    }
                }
                const double xi = acc / d;
                ly[il] = xi;
                xnew[r0 + il] = xi;
                prev = il;
                prev_x = xi;
            }
        }
        if (chain_wave) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
}

}  // namespace

void launch_hybrid_gs(bool forward, int n, const int32_t* rp, const int32_t* ci, const double* v,
                      const double* b, const double* xold, double* xnew, int block, double mean_row,
                      hipStream_t st) {
    if (n <= 0) return;
    if (block <= kGsMaxRows && block <= AMG_GS_STAGED_MAX) {
        // chunks of whole blocks whose entries usually fit the staging buffer
        const int per = std::max(1, std::min(kGsMaxRows / block,
                                             (int)(kGsCap / (1.15 * std::max(mean_row, 1.0) * block))));
        const int R = per * block;
        const int nchunk = (n + R - 1) / R;
        const int grid = std::max(1, std::min(nchunk, 65535));
        if (forward)
            hipLaunchKernelGGL(hybrid_gs_staged_kernel<true>, dim3(grid), dim3(kGsThreads), 0, st, n, rp, ci, v, b,
                               xold, xnew, block, R);
        else
            hipLaunchKernelGGL(hybrid_gs_staged_kernel<false>, dim3(grid), dim3(kGsThreads), 0, st, n, rp, ci, v, b,
                               xold, xnew, block, R);
        return;
    }
    const int64_t nblk = ((int64_t)n + block - 1) / block;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nblk + 255) / 256, 65535));
    if (forward)
        hipLaunchKernelGGL(hybrid_gs_kernel<true>, dim3(grid), dim3(256), 0, st, n, rp, ci, v, b, xold, xnew, block);
    else
        hipLaunchKernelGGL(hybrid_gs_kernel<false>, dim3(grid), dim3(256), 0, st, n, rp, ci, v, b, xold, xnew,
                           block);
}

}  // namespace amg355
