// Hybrid Gauss-Seidel sweep: one thread per block of rows, the rows of a
// block in order, each row's sum in ascending column order (the order and
// operations of the definition, so the result is the CPU's bit for bit).
#include "relax_kernels.hpp"

#include <algorithm>

#pragma clang fp contract(off)

namespace amg355 {

namespace {

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
        // the row visited last: its new value stays in a register
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
}

}  // namespace

void launch_hybrid_gs(bool forward, int n, const int32_t* rp, const int32_t* ci, const double* v,
                      const double* b, const double* xold, double* xnew, int block, hipStream_t st) {
    const int64_t nblk = ((int64_t)n + block - 1) / block;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nblk + 255) / 256, 65535));
    if (forward)
        hipLaunchKernelGGL(hybrid_gs_kernel<true>, dim3(grid), dim3(256), 0, st, n, rp, ci, v, b, xold, xnew, block);
    else
        hipLaunchKernelGGL(hybrid_gs_kernel<false>, dim3(grid), dim3(256), 0, st, n, rp, ci, v, b, xold, xnew,
                           block);
}

}  // namespace amg355
