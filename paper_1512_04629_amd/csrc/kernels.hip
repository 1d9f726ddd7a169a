// Device kernels of the sparsified-AMG hot path for gfx950 (CDNA4, wave64).
//
// Nothing here is a dense contraction, so no MFMA: every kernel is bound by
// HBM bandwidth (or launch latency on the small coarse levels).  The CSR row
// kernel assigns W lanes (a subgroup of the 64-lane wavefront) to a row, with
// W the power of two nearest the mean row length, so that the lanes of a
// wavefront read consecutive nonzeros; the row sum is reduced with lane
// shuffles and the epilogue (residual, Jacobi update, dot products) is fused
// into the same pass so that every vector is read once.
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>
#include <cmath>

namespace amg355 {
namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;            // MI355X: 8 accelerator complex dies, each with its own L2
#ifndef AMG_ROW_GRID_CAP
#define AMG_ROW_GRID_CAP 4096
#endif
constexpr int kRowGridCap = AMG_ROW_GRID_CAP;   // row kernels loop over tiles beyond this many blocks

// Tuning knobs (compile-time): lanes-per-row thresholds are scaled by
// AMG_WIDTH_SCALE (1 = the power of two nearest the mean row length),
// AMG_RIF is the number of row tiles in flight per subgroup, AMG_MIN_WIDTH the
// narrowest subgroup, AMG_USE_STREAM selects the LDS-staged kernel (-1: by
// matrix shape, 0: never, 1: always), AMG_XCD_REMAP toggles
// the XCD-contiguous block order.
#ifndef AMG_WIDTH_SCALE
#define AMG_WIDTH_SCALE 0.5
#endif
#ifndef AMG_RIF
#define AMG_RIF 1
#endif
#ifndef AMG_MIN_WIDTH
#define AMG_MIN_WIDTH 1
#endif
#ifndef AMG_USE_STREAM
#define AMG_USE_STREAM -1
#endif
#ifndef AMG_XCD_REMAP
#define AMG_XCD_REMAP 1
#endif
#ifndef AMG_STREAM_CAP
#define AMG_STREAM_CAP 2048
#endif
// Longest mean row the LDS-staged kernel takes.  Measured on the 128^3
// hierarchy against the subgroup kernel: level 2 (rows of 30-34 entries)
// sweep 18.3 -> 16.5 us, zero-guess residual 21.8 -> 20.5 us; level 3 (rows
// of 41-57 entries) 6.3 -> 5.0 us and 7.7 -> 5.8 us.
#ifndef AMG_STREAM_MAX_ROW
#define AMG_STREAM_MAX_ROW 64.0
#endif
#ifndef AMG_STREAM_FILL
#define AMG_STREAM_FILL 0.85
#endif
#ifndef AMG_NT
#define AMG_NT 0
#endif
#ifndef AMG_VEC4
#define AMG_VEC4 -1
#endif
// LDS-staged kernels: 2048 workgroups = 8 resident workgroups on each of the
// 256 compute units, one full wave of the machine; measured best against
// 1024, 3072 and 4096 (which leave a partial second wave).
#ifndef AMG_STREAM_GRID_CAP
#define AMG_STREAM_GRID_CAP 2048
#endif

// Matrix entries are streamed once per launch; with AMG_NT they are loaded
// non-temporally so that they do not evict the gathered vector from L2.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned short v4u16 __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T stream_ld(const T* p) {
#if AMG_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Workgroups are handed to the XCDs round-robin.  Remap so that XCD x works on
// a contiguous range of logical blocks: neighbouring rows gather neighbouring
// entries of x, which then stay in one L2.  The grid is a multiple of 8.
__device__ __forceinline__ int xcd_logical_block() {
#if AMG_XCD_REMAP
    const int per = gridDim.x / kXcds;
    return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
#else
    return blockIdx.x;
#endif
}

int round_up8(int b) { return (b + kXcds - 1) / kXcds * kXcds; }

// Events armed by set_launch_events: the next row-kernel launch records its
// own start and end in them (hipExtLaunchKernel), so that a timing of it
// covers the kernel as a profiler's kernel trace does.
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

template <class K, class... Args>
void launch_row_kernel(K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
    if (t_ev_start) {
        hipEvent_t a = t_ev_start, b = t_ev_stop;
        t_ev_start = t_ev_stop = nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, a, b, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    }
}

// column of entry p of a row block whose 16-bit base is cb
template <bool IDX16, class T>
__device__ __forceinline__ int load_col(const CsrT<T>& a, int p, int cb) {
    if constexpr (IDX16) return cb + (int)stream_ld(a.ci16 + p);
    else return stream_ld(a.ci + p);
}

template <int W, class T>
__device__ __forceinline__ T sub_sum(T v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

template <int W>
__device__ __forceinline__ double sub_max(double v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
    return v;
}

template <int W>
__device__ __forceinline__ int sub_sum_int(int v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// Block-wide sum of v; the total is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        t = lds[0];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) t += lds[w];
    }
    __syncthreads();
    return t;
}

// Deterministic grid reduction, first pass: every block stores its partial
// sum; dot_finish_kernel adds the partials in a fixed order.  (A single-pass
// last-block scheme would need an agent-scope release fence per block, which
// on gfx950 writes back the XCD's L2 and stalls the block.)
__device__ __forceinline__ void store_block_partial(double v, double* partials, int lb) {
    __shared__ double lds[kBlock / 64];
    const double t = block_sum(v, lds);
    if (threadIdx.x == 0) partials[lb] = t;
}

constexpr int kFinishBlock = 1024;

__global__ __launch_bounds__(kFinishBlock) void dot_finish_kernel(int nparts, const double* __restrict__ partials,
                                                                  double* __restrict__ result) {
    __shared__ double wsum[kFinishBlock / 64];
    // thread t takes partials t, t + 1024, ... into four accumulators in turn
    // (independent loads in flight), adds them pairwise, then a fixed shuffle
    // tree per wave and the wave sums in wave order
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kFinishBlock < nparts; i += 4 * kFinishBlock) {
        a0 += partials[i];
        a1 += partials[i + kFinishBlock];
        a2 += partials[i + 2 * kFinishBlock];
        a3 += partials[i + 3 * kFinishBlock];
    }
    if (i < nparts) a0 += partials[i];
    if (i + kFinishBlock < nparts) a1 += partials[i + kFinishBlock];
    if (i + 2 * kFinishBlock < nparts) a2 += partials[i + 2 * kFinishBlock];
    double s = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = wsum[0];
#pragma unroll
        for (int w = 1; w < kFinishBlock / 64; ++w) tot += wsum[w];
        *result = tot;
    }
}

void finish_dot(const DotTarget& dot, int nparts, hipStream_t st) {
    hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(kFinishBlock), 0, st, nparts, dot.partials, dot.result);
}

template <int OP>
constexpr bool op_has_dot() {
    return OP == kResidNorm || OP == kJacobiDot || OP == kSpmvDot;
}

// Rows in flight per subgroup: the loads of R row tiles are issued before
// any of them is consumed, so that each lane has R independent
// (row pointer -> column/value -> gathered entry) chains outstanding.
template <int W>
constexpr int rows_in_flight() {
    return W <= 16 ? AMG_RIF : 1;
}

template <class T, int W, int OP>
__global__ __launch_bounds__(kBlock) void row_kernel(CsrT<T> a, const T* __restrict__ g,
                                                     const T* u, const T* __restrict__ dinv,
                                                     T omega, T* y, T* y2,
                                                     DotTarget dot, int ntiles) {
    constexpr int kRowsPerBlock = kBlock / W;
    constexpr int R = rows_in_flight<W>();
    const int lb = xcd_logical_block();
    const int sub = threadIdx.x / W;
    const int lane = threadIdx.x & (W - 1);
    double contrib = 0.0;
    for (int t0 = lb * R; t0 < ntiles; t0 += gridDim.x * R) {
        int row[R], beg[R], end[R];
        T s[R], ui[R], gi[R], di[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            row[k] = (t0 + k) * kRowsPerBlock + sub;
            const bool act = row[k] < a.rows;
            beg[k] = act ? a.rp[row[k]] : 0;
            end[k] = act ? a.rp[row[k] + 1] : 0;
            ui[k] = gi[k] = di[k] = T(0);
            if (act && lane == 0) {
                if constexpr (OP != kSpmv && OP != kSpmvDot && OP != kSpmvScale) ui[k] = u[row[k]];
                if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kSpmvDot) gi[k] = g[row[k]];
                if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kZeroJacobiResid || OP == kSpmvScale)
                    di[k] = dinv[row[k]];
            }
        }
        // first chunk of every tile, branch-free (an empty slot re-loads the
        // row's first entry or entry 0) so that all loads are in flight together
        int jk[R];
        T vk[R], gk[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int p = beg[k] + lane;
            const int pc = p < end[k] ? p : (end[k] > beg[k] ? beg[k] : 0);
            jk[k] = a.ci[pc];
            vk[k] = a.v[pc];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int j = jk[k];
            if constexpr (OP == kZeroJacobiResid) gk[k] = omega * (dinv[j] * u[j]);
            else gk[k] = g[j];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) s[k] = (beg[k] + lane < end[k]) ? vk[k] * gk[k] : T(0);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            for (int p = beg[k] + lane + W; p < end[k]; p += W) {
                const int j = a.ci[p];
                T gj;
                if constexpr (OP == kZeroJacobiResid) gj = omega * (dinv[j] * u[j]);
                else gj = g[j];
                s[k] += a.v[p] * gj;
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T sk = sub_sum<W>(s[k]);
            if (row[k] < a.rows && lane == 0) {
                const int r = row[k];
                if constexpr (OP == kSpmv) {
                    y[r] = sk;
                } else if constexpr (OP == kSpmvAdd) {
                    y[r] = ui[k] + sk;
                } else if constexpr (OP == kResid || OP == kResidNorm) {
                    const T rr = ui[k] - sk;
                    y[r] = rr;
                    if constexpr (OP == kResidNorm) contrib += (double)rr * (double)rr;
                } else if constexpr (OP == kJacobi || OP == kJacobiDot) {
                    const T xn = gi[k] + omega * di[k] * (ui[k] - sk);
                    y[r] = xn;
                    if constexpr (OP == kJacobiDot) contrib += (double)ui[k] * (double)xn;
                } else if constexpr (OP == kZeroJacobiResid) {
                    y2[r] = omega * (di[k] * ui[k]);
                    y[r] = ui[k] - sk;
                } else if constexpr (OP == kSpmvDot) {
                    y[r] = sk;
                    contrib += (double)gi[k] * (double)sk;
                } else if constexpr (OP == kSpmvScale) {
                    y[r] = sk;
                    y2[r] = omega * (di[k] * sk);
                }
            }
        }
    }
    if constexpr (op_has_dot<OP>()) store_block_partial(contrib, dot.partials, lb);
}

template <class T, int W>
int launch_row_w(RowOp op, const CsrT<T>& a, const T* g, const T* u, const T* dinv,
                 T omega, T* y, T* y2, DotTarget dot, hipStream_t st) {
    constexpr int kRowsPerBlock = kBlock / W;
    constexpr int R = rows_in_flight<W>();
    const int ntiles = std::max(1, (a.rows + kRowsPerBlock - 1) / kRowsPerBlock);
    const int groups = (ntiles + R - 1) / R;
    const int grid = round_up8(std::min(groups, kRowGridCap));
    switch (op) {
#define AMG_ROW_CASE(OPV)                                                                      \
    case OPV:                                                                                  \
        launch_row_kernel(row_kernel<T, W, OPV>, dim3(grid), dim3(kBlock), st, a, g, u, dinv, omega, y, y2, \
                          dot, ntiles);                                                        \
        break;
        AMG_ROW_CASE(kSpmv)
        AMG_ROW_CASE(kSpmvAdd)
        AMG_ROW_CASE(kResid)
        AMG_ROW_CASE(kResidNorm)
        AMG_ROW_CASE(kJacobi)
        AMG_ROW_CASE(kJacobiDot)
        AMG_ROW_CASE(kZeroJacobiResid)
        AMG_ROW_CASE(kSpmvDot)
        AMG_ROW_CASE(kSpmvScale)
#undef AMG_ROW_CASE
        default: break;
    }
    return (op == kResidNorm || op == kJacobiDot || op == kSpmvDot) ? grid : 0;
}

// CSR-stream variant: a block owns RB consecutive rows; its threads load the
// block's nonzeros with coalesced loads, multiply by the gathered entries and
// park the products in LDS; then 256/RB lanes per row add the row's products.
constexpr int kStreamCap = AMG_STREAM_CAP;   // products staged per pass (16 KB of LDS)

template <class T, int RB, int OP, bool VEC4, bool IDX16>
__global__ __launch_bounds__(kBlock) void stream_kernel(CsrT<T> a, const T* __restrict__ g,
                                                        const T* u, const T* __restrict__ dinv,
                                                        T omega, T* y, T* y2,
                                                        DotTarget dot, int nblk) {
    constexpr int W2 = kBlock / RB;
    __shared__ T prod[kStreamCap];
    const int lb = xcd_logical_block();
    const int lane = threadIdx.x & (W2 - 1);
    double contrib = 0.0;
    for (int lblk = lb; lblk < nblk; lblk += gridDim.x) {
        const int blk = a.rev ? nblk - 1 - lblk : lblk;
        const int r0 = blk * RB;
        const int r1 = min(r0 + RB, a.rows);
        const int p0 = a.rp[r0], p1 = a.rp[r1];
        const int cb = IDX16 ? a.cbase[blk] : 0;
        const int r = r0 + (int)threadIdx.x / W2;
        const bool act = r < r1;
        const int rb = act ? a.rp[r] : 0, re = act ? a.rp[r + 1] : 0;
        T ui = T(0), gi = T(0), di = T(0);
        if (act && lane == 0) {
            if constexpr (OP != kSpmv && OP != kSpmvDot && OP != kSpmvScale) ui = u[r];
            if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kSpmvDot) gi = g[r];
            if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kZeroJacobiResid || OP == kSpmvScale)
                di = dinv[r];
        }
        T s = T(0);
        for (int c0 = p0; c0 < p1; c0 += kStreamCap) {
            const int c1 = min(c0 + kStreamCap, p1);
            if constexpr (VEC4) {
                // 4 entries per lane from the 16-byte aligned pack holding them;
                // the arrays carry spare entries so that the last pack is
                // readable, entries outside [c0, c1) are skipped
                const int base = c0 & ~3;
#pragma unroll
                for (int k = 0; k < (kStreamCap + 3) / (4 * kBlock) + 1; ++k) {
                    const int q = base + 4 * (k * kBlock + (int)threadIdx.x);
                    if (q < c1) {
                        int jj[4];
                        if constexpr (IDX16) {
                            // entries of the pack outside the block are skipped below
                            const v4u16 cj = stream_ld(reinterpret_cast<const v4u16*>(a.ci16 + q));
                            jj[0] = cb + cj.x; jj[1] = cb + cj.y; jj[2] = cb + cj.z; jj[3] = cb + cj.w;
                        } else {
                            const v4i cj = stream_ld(reinterpret_cast<const v4i*>(a.ci + q));
                            jj[0] = cj.x; jj[1] = cj.y; jj[2] = cj.z; jj[3] = cj.w;
                        }
                        T vv[4];
                        if constexpr (sizeof(T) == 8) {
                            const v2d v01 = stream_ld(reinterpret_cast<const v2d*>(a.v + q));
                            const v2d v23 = stream_ld(reinterpret_cast<const v2d*>(a.v + q + 2));
                            vv[0] = v01.x; vv[1] = v01.y; vv[2] = v23.x; vv[3] = v23.y;
                        } else {
                            const v4f v0123 = stream_ld(reinterpret_cast<const v4f*>(a.v + q));
                            vv[0] = v0123.x; vv[1] = v0123.y; vv[2] = v0123.z; vv[3] = v0123.w;
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int p = q + e;
                            if (p >= c0 && p < c1) {
                                const int j = jj[e];
                                T gj;
                                if constexpr (OP == kZeroJacobiResid) gj = omega * (dinv[j] * u[j]);
                                else gj = g[j];
                                prod[p - c0] = vv[e] * gj;
                            }
                        }
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < kStreamCap / kBlock; ++k) {
                    const int p = c0 + k * kBlock + (int)threadIdx.x;
                    if (p < c1) {
                        const int j = load_col<IDX16>(a, p, cb);
                        T gj;
                        if constexpr (OP == kZeroJacobiResid) gj = omega * (dinv[j] * u[j]);
                        else gj = g[j];
                        prod[p - c0] = stream_ld(a.v + p) * gj;
                    }
                }
            }
            __syncthreads();
            const int lo = max(rb, c0), hi = min(re, c1);
            for (int p = lo + lane; p < hi; p += W2) s += prod[p - c0];
            __syncthreads();
        }
        s = sub_sum<W2>(s);
        if (act && lane == 0) {
            if constexpr (OP == kSpmv) {
                y[r] = s;
            } else if constexpr (OP == kSpmvAdd) {
                y[r] = ui + s;
            } else if constexpr (OP == kResid || OP == kResidNorm) {
                const T rr = ui - s;
                y[r] = rr;
                if constexpr (OP == kResidNorm) contrib += (double)rr * (double)rr;
            } else if constexpr (OP == kJacobi || OP == kJacobiDot) {
                const T xn = gi + omega * di * (ui - s);
                y[r] = xn;
                if constexpr (OP == kJacobiDot) contrib += (double)ui * (double)xn;
            } else if constexpr (OP == kZeroJacobiResid) {
                y2[r] = omega * (di * ui);
                y[r] = ui - s;
            } else if constexpr (OP == kSpmvDot) {
                y[r] = s;
                contrib += (double)gi * (double)s;
            } else if constexpr (OP == kSpmvScale) {
                y[r] = s;
                y2[r] = omega * (di * s);
            }
        }
    }
    if constexpr (op_has_dot<OP>()) store_block_partial(contrib, dot.partials, lb);
}

// Software-pipelined form of stream_kernel for scalar loads.  A block's next
// row block is staged one pass ahead: its row pointers are requested before
// the current gathers and the first chunk of its column indices and values
// before the current reduction, so the matrix stream keeps running across
// the two barriers of each pass (on gfx950 a workgroup barrier waits for LDS
// traffic only, not for outstanding global loads).
// Measured on the 128^3 hierarchy's level-1 operator (19.6M nonzeros): staging
// two entries per thread is 8% faster than the unpipelined kernel; staging 1,
// 3 or 4 is between (4 costs occupancy: 64 registers).
#ifndef AMG_PIPE
#define AMG_PIPE 1
#endif
#ifndef AMG_PIPE_E
#define AMG_PIPE_E 2
#endif
template <class T, int RB, int OP, bool IDX16>
__global__ __launch_bounds__(kBlock) void stream_pipe_kernel(CsrT<T> a, const T* __restrict__ g,
                                                             const T* u, const T* __restrict__ dinv,
                                                             T omega, T* y, T* y2, DotTarget dot, int nblk) {
    constexpr int W2 = kBlock / RB;
    constexpr int E = kStreamCap / kBlock;     // entries per thread of a full chunk
    constexpr int PE = AMG_PIPE_E < E ? AMG_PIPE_E : E;   // of which staged one pass ahead
    __shared__ T prod[kStreamCap];
    const int lb = xcd_logical_block();
    const int lane = threadIdx.x & (W2 - 1);
    const int rsub = (int)threadIdx.x / W2;
    double contrib = 0.0;
    auto meta = [&](int lbk, int& q0, int& q1, int& rr, bool& ac, int& qb, int& qe, int& cbb) {
        const int b = a.rev ? nblk - 1 - lbk : lbk;
        const int r0 = b * RB;
        const int r1 = min(r0 + RB, a.rows);
        q0 = a.rp[r0];
        q1 = a.rp[r1];
        cbb = IDX16 ? a.cbase[b] : 0;
        rr = r0 + rsub;
        ac = rr < r1;
        qb = ac ? a.rp[rr] : 0;
        qe = ac ? a.rp[rr + 1] : 0;
    };
    auto stage = [&](int q0, int q1, int cbb, int (&jj)[PE], T (&vv)[PE]) {
        const int c1 = min(q1, q0 + kStreamCap);
#pragma unroll
        for (int k = 0; k < PE; ++k) {
            const int p = q0 + k * kBlock + (int)threadIdx.x;
            const bool ok = p < c1;
            jj[k] = ok ? load_col<IDX16>(a, p, cbb) : 0;
            vv[k] = ok ? stream_ld(a.v + p) : T(0);
        }
    };
    auto gather = [&](int j) -> T {
        if constexpr (OP == kZeroJacobiResid) return omega * (dinv[j] * u[j]);
        else return g[j];
    };
    int p0 = 0, p1 = 0, r = 0, rb = 0, re = 0, cb = 0;
    bool act = false;
    int jc[PE];
    T vc[PE];
    int blk = lb;
    if (blk < nblk) {
        meta(blk, p0, p1, r, act, rb, re, cb);
        stage(p0, p1, cb, jc, vc);
    }
    for (; blk < nblk; blk += gridDim.x) {
        const int nb = blk + gridDim.x;
        int np0 = 0, np1 = 0, nr = 0, nrb = 0, nre = 0, ncb = 0;
        bool nact = false;
        if (nb < nblk) meta(nb, np0, np1, nr, nact, nrb, nre, ncb);
        T ui = T(0), gi = T(0), di = T(0);
        if (act && lane == 0) {
            if constexpr (OP != kSpmv && OP != kSpmvDot && OP != kSpmvScale) ui = u[r];
            if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kSpmvDot) gi = g[r];
            if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kZeroJacobiResid || OP == kSpmvScale)
                di = dinv[r];
        }
        const int c1 = min(p1, p0 + kStreamCap);
        T gk[PE];
#pragma unroll
        for (int k = 0; k < PE; ++k) {
            const int p = p0 + k * kBlock + (int)threadIdx.x;
            gk[k] = p < c1 ? gather(jc[k]) : T(0);
        }
        int jn[PE];
        T vn[PE];
        if (nb < nblk) {
            stage(np0, np1, ncb, jn, vn);
        } else {
#pragma unroll
            for (int k = 0; k < PE; ++k) {
                jn[k] = 0;
                vn[k] = T(0);
            }
        }
#pragma unroll
        for (int k = 0; k < PE; ++k) {
            const int p = p0 + k * kBlock + (int)threadIdx.x;
            if (p < c1) prod[p - p0] = vc[k] * gk[k];
        }
        // entries of the first chunk beyond the staged ones
#pragma unroll
        for (int k = PE; k < E; ++k) {
            const int p = p0 + k * kBlock + (int)threadIdx.x;
            if (p < c1) prod[p - p0] = stream_ld(a.v + p) * gather(load_col<IDX16>(a, p, cb));
        }
        __syncthreads();
        T s = T(0);
        {
            const int lo = max(rb, p0), hi = min(re, c1);
            for (int p = lo + lane; p < hi; p += W2) s += prod[p - p0];
        }
        __syncthreads();
        // rows of this block beyond the first chunk
        for (int c0 = p0 + kStreamCap; c0 < p1; c0 += kStreamCap) {
            const int cc1 = min(c0 + kStreamCap, p1);
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int p = c0 + k * kBlock + (int)threadIdx.x;
                if (p < cc1) prod[p - c0] = stream_ld(a.v + p) * gather(load_col<IDX16>(a, p, cb));
            }
            __syncthreads();
            const int lo = max(rb, c0), hi = min(re, cc1);
            for (int p = lo + lane; p < hi; p += W2) s += prod[p - c0];
            __syncthreads();
        }
        s = sub_sum<W2>(s);
        if (act && lane == 0) {
            if constexpr (OP == kSpmv) {
                y[r] = s;
            } else if constexpr (OP == kSpmvAdd) {
                y[r] = ui + s;
            } else if constexpr (OP == kResid || OP == kResidNorm) {
                const T rr = ui - s;
                y[r] = rr;
                if constexpr (OP == kResidNorm) contrib += (double)rr * (double)rr;
            } else if constexpr (OP == kJacobi || OP == kJacobiDot) {
                const T xn = gi + omega * di * (ui - s);
                y[r] = xn;
                if constexpr (OP == kJacobiDot) contrib += (double)ui * (double)xn;
            } else if constexpr (OP == kZeroJacobiResid) {
                y2[r] = omega * (di * ui);
                y[r] = ui - s;
            } else if constexpr (OP == kSpmvDot) {
                y[r] = s;
                contrib += (double)gi * (double)s;
            } else if constexpr (OP == kSpmvScale) {
                y[r] = s;
                y2[r] = omega * (di * s);
            }
        }
        p0 = np0;
        p1 = np1;
        cb = ncb;
        r = nr;
        act = nact;
        rb = nrb;
        re = nre;
#pragma unroll
        for (int k = 0; k < PE; ++k) {
            jc[k] = jn[k];
            vc[k] = vn[k];
        }
    }
    if constexpr (op_has_dot<OP>()) store_block_partial(contrib, dot.partials, lb);
}

template <class T, int RB, bool VEC4, bool IDX16>
void launch_stream_rbi(RowOp op, const CsrT<T>& a, const T* g, const T* u, const T* dinv,
                       T omega, T* y, T* y2, DotTarget dot, int nblk, int grid, hipStream_t st) {
    switch (op) {
#define AMG_STREAM_CASE(OPV)                                                                      \
    case OPV:                                                                                     \
        if (AMG_PIPE && !VEC4)                                                                    \
            launch_row_kernel(stream_pipe_kernel<T, RB, OPV, IDX16>, dim3(grid), dim3(kBlock), st, a, g, u, \
                              dinv, omega, y, y2, dot, nblk);                                     \
        else                                                                                      \
            launch_row_kernel(stream_kernel<T, RB, OPV, VEC4, IDX16>, dim3(grid), dim3(kBlock), st, a, g, u, \
                              dinv, omega, y, y2, dot, nblk);                                     \
        break;
        AMG_STREAM_CASE(kSpmv)
        AMG_STREAM_CASE(kSpmvAdd)
        AMG_STREAM_CASE(kResid)
        AMG_STREAM_CASE(kResidNorm)
        AMG_STREAM_CASE(kJacobi)
        AMG_STREAM_CASE(kJacobiDot)
        AMG_STREAM_CASE(kZeroJacobiResid)
        AMG_STREAM_CASE(kSpmvDot)
        AMG_STREAM_CASE(kSpmvScale)
#undef AMG_STREAM_CASE
        default: break;
    }
}

// Alternating the direction of consecutive passes over one operator lets a
// pass start on the part of the operator the previous pass left in the
// Infinity Cache.
#ifndef AMG_STREAM_ALTERNATE
#define AMG_STREAM_ALTERNATE 1
#endif

template <class T, int RB, bool VEC4>
int launch_stream_rb(RowOp op, const CsrT<T>& a_in, const T* g, const T* u, const T* dinv,
                     T omega, T* y, T* y2, DotTarget dot, hipStream_t st) {
    const int nblk = std::max(1, (a_in.rows + RB - 1) / RB);
    const int grid = round_up8(std::min(nblk, std::min(kRowGridCap, AMG_STREAM_GRID_CAP)));
    CsrT<T> a = a_in;
    // a dot product's per-workgroup partials depend on which row blocks a
    // workgroup visits: those launches keep the ascending order
    if (!AMG_STREAM_ALTERNATE || op == kResidNorm || op == kJacobiDot || op == kSpmvDot) a.rev = 0;
    if (a.ci16 && a.idx_rb == RB)
        launch_stream_rbi<T, RB, VEC4, true>(op, a, g, u, dinv, omega, y, y2, dot, nblk, grid, st);
    else launch_stream_rbi<T, RB, VEC4, false>(op, a, g, u, dinv, omega, y, y2, dot, nblk, grid, st);
    return (op == kResidNorm || op == kJacobiDot || op == kSpmvDot) ? grid : 0;
}


// ---- SELL-64 row kernel ------------------------------------------------------
// One wavefront per slice of 64 consecutive rows, one lane per row.  Entry k
// of every row of a slice is one contiguous stretch (256 bytes of column
// indices, 512 of values), and a lane requests its whole row (U entries, the
// slice width rounded up) before it forms a product: no LDS staging and no
// barriers, and each lane has U independent gathers in flight.  Entries
// beyond the slice width re-read the last one (same cache line, no extra
// traffic) and are masked out; padding inside the width carries value 0.  A
// lane sums its row in ascending column order.  Rows wider than U are taken
// U entries at a time.
#ifndef AMG_SELL
#define AMG_SELL 1
#endif
// one workgroup per four slices, up to 65,536 workgroups (16.7M rows; larger
// operators loop): the hardware hands out the workgroups as others finish.
// Measured on 3D Poisson 192^3, against 2,048, 4,096 and 8,192 workgroups
// looping over the slices: A_1 Jacobi sweep 195 -> 171 us, A_0 residual 152
// -> 140 us (back to back); no change at 128^3.
#ifndef AMG_SELL_GRID_CAP
#define AMG_SELL_GRID_CAP 65536
#endif
constexpr int kSellRows = 64;
constexpr int kSellSlicesPerBlock = kBlock / kSellRows;

template <bool NT, class T>
__device__ __forceinline__ T sell_ld(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// IDXW: bytes per column index read, 4 (sl_col), 2 (sl_base + sl_col16) or 1
// (the slice's offset table, sl_idx8)
template <class T, int U, int OP, bool NT, int IDXW>
__global__ __launch_bounds__(kBlock) void sell_kernel(CsrT<T> a, const T* __restrict__ g, const T* u,
                                                      const T* __restrict__ dinv, T omega, T* y, T* y2,
                                                      DotTarget dot, int nslices) {
    const int lb = xcd_logical_block();
    const int wv = (int)threadIdx.x / kSellRows;
    const int lane = (int)threadIdx.x & (kSellRows - 1);
    const int nblocks = (nslices + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock;
    double contrib = 0.0;
    // a workgroup takes blocks of four slices, in descending block order when
    // a.rev; with one block per workgroup a dot product's partial goes to the
    // block's own index, so it is the same in both orders
    int pidx = lb;
    for (int lblk = lb; lblk < nblocks; lblk += gridDim.x) {
        const int blk = a.rev ? nblocks - 1 - lblk : lblk;
        if (nblocks <= (int)gridDim.x) pidx = blk;
        const int sl = blk * kSellSlicesPerBlock + wv;
        if (sl >= nslices) continue;
        const int o0 = a.sl_off[sl];
        const int w = (a.sl_off[sl + 1] - o0) / kSellRows;
        const int cb = IDXW == 2 ? a.sl_base[sl] : 0;
        const int tabv = IDXW == 1 ? a.sl_tab[sl * kSellRows + lane] : 0;
        const int r = sl * kSellRows + lane;
        const bool act = r < a.rows;
        T ui = T(0), gi = T(0), di = T(0);
        if (act) {
            if constexpr (OP != kSpmv && OP != kSpmvDot && OP != kSpmvScale) ui = u[r];
            if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kSpmvDot) gi = g[r];
            if constexpr (OP == kJacobi || OP == kJacobiDot || OP == kZeroJacobiResid || OP == kSpmvScale)
                di = dinv[r];
        }
        T acc = T(0);
        for (int k0 = 0; k0 < w; k0 += U) {
            int jj[U];
            T vv[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int p = o0 + min(k0 + k, w - 1) * kSellRows + lane;
                if constexpr (IDXW == 1) {
                    const int d = __shfl(tabv, (int)sell_ld<NT>(a.sl_idx8 + p), 64);
                    jj[k] = act ? r + d : 0;
                } else if constexpr (IDXW == 2) {
                    jj[k] = cb + (int)sell_ld<NT>(a.sl_col16 + p);
                } else {
                    jj[k] = sell_ld<NT>(a.sl_col + p);
                }
                vv[k] = sell_ld<NT>(a.sl_val + p);
            }
            T gg[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int j = jj[k];
                if constexpr (OP == kZeroJacobiResid) gg[k] = omega * (dinv[j] * u[j]);
                else gg[k] = g[j];
            }
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (k0 + k < w) acc += vv[k] * gg[k];
        }
        if (act) {
            if constexpr (OP == kSpmv) {
                y[r] = acc;
            } else if constexpr (OP == kSpmvAdd) {
                y[r] = ui + acc;
            } else if constexpr (OP == kResid || OP == kResidNorm) {
                const T rr = ui - acc;
                y[r] = rr;
                if constexpr (OP == kResidNorm) contrib += (double)rr * (double)rr;
            } else if constexpr (OP == kJacobi || OP == kJacobiDot) {
                const T xn = gi + omega * di * (ui - acc);
                y[r] = xn;
                if constexpr (OP == kJacobiDot) contrib += (double)ui * (double)xn;
            } else if constexpr (OP == kZeroJacobiResid) {
                y2[r] = omega * (di * ui);
                y[r] = ui - acc;
            } else if constexpr (OP == kSpmvDot) {
                y[r] = acc;
                contrib += (double)gi * (double)acc;
            } else if constexpr (OP == kSpmvScale) {
                y[r] = acc;
                y2[r] = omega * (di * acc);
            }
        }
    }
    if constexpr (op_has_dot<OP>()) store_block_partial(contrib, dot.partials, pidx);
}

// Two residuals of one operator in one pass over its SELL-64 copy:
// y = u - A g and y2 = u2 - A g2 with the block partials of ||y2||^2.  Each
// entry is loaded once and both vectors gathered; every row is summed in the
// order sell_kernel sums it and the partials go to the same indices, so both
// results are those of the kResid and kResidNorm launches bit for bit.
template <int U, bool NT, int IDXW>
__global__ __launch_bounds__(kBlock) void sell_dual_resid_kernel(CsrView a, const double* __restrict__ g,
                                                                 const double* u, double* y,
                                                                 const double* __restrict__ g2,
                                                                 const double* u2, double* y2, DotTarget dot,
                                                                 int nslices) {
    const int lb = xcd_logical_block();
    const int wv = (int)threadIdx.x / kSellRows;
    const int lane = (int)threadIdx.x & (kSellRows - 1);
    const int nblocks = (nslices + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock;
    double contrib = 0.0;
    int pidx = lb;
    for (int lblk = lb; lblk < nblocks; lblk += gridDim.x) {
        const int blk = a.rev ? nblocks - 1 - lblk : lblk;
        if (nblocks <= (int)gridDim.x) pidx = blk;
        const int sl = blk * kSellSlicesPerBlock + wv;
        if (sl >= nslices) continue;
        const int o0 = a.sl_off[sl];
        const int w = (a.sl_off[sl + 1] - o0) / kSellRows;
        const int cb = IDXW == 2 ? a.sl_base[sl] : 0;
        const int tabv = IDXW == 1 ? a.sl_tab[sl * kSellRows + lane] : 0;
        const int r = sl * kSellRows + lane;
        const bool act = r < a.rows;
        double ui = 0.0, u2i = 0.0;
        if (act) {
            ui = u[r];
            u2i = u2[r];
        }
        double acc = 0.0, acc2 = 0.0;
        for (int k0 = 0; k0 < w; k0 += U) {
            int jj[U];
            double vv[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int p = o0 + min(k0 + k, w - 1) * kSellRows + lane;
                if constexpr (IDXW == 1) {
                    const int d = __shfl(tabv, (int)sell_ld<NT>(a.sl_idx8 + p), 64);
                    jj[k] = act ? r + d : 0;
                } else if constexpr (IDXW == 2) {
                    jj[k] = cb + (int)sell_ld<NT>(a.sl_col16 + p);
                } else {
                    jj[k] = sell_ld<NT>(a.sl_col + p);
                }
                vv[k] = sell_ld<NT>(a.sl_val + p);
            }
            double gg[U], gg2[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                gg[k] = g[jj[k]];
                gg2[k] = g2[jj[k]];
            }
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (k0 + k < w) {
                    acc += vv[k] * gg[k];
                    acc2 += vv[k] * gg2[k];
                }
        }
        if (act) {
            y[r] = ui - acc;
            const double rr = u2i - acc2;
            y2[r] = rr;
            contrib += rr * rr;
        }
    }
    store_block_partial(contrib, dot.partials, pidx);
}

// Matrices larger than this stream their entries with non-temporal loads:
// they cannot stay in the 256 MB Infinity Cache between passes, and the
// entries then do not displace the gathered vectors; smaller ones are loaded
// normally so that a later pass can find them there.
#ifndef AMG_SELL_NT_BYTES
#define AMG_SELL_NT_BYTES (256ll << 20)
#endif

int sell_grid(int rows) {
    const int nslices = (rows + kSellRows - 1) / kSellRows;
    const int blocks = (nslices + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock;
    return round_up8(std::max(1, std::min(blocks, (int)AMG_SELL_GRID_CAP)));
}

template <class T, int U>
int launch_sell_u(RowOp op, const CsrT<T>& a_in, const T* g, const T* u, const T* dinv, T omega, T* y, T* y2,
                  DotTarget dot, hipStream_t st) {
    const int nslices = (a_in.rows + kSellRows - 1) / kSellRows;
    const int grid = sell_grid(a_in.rows);
    CsrT<T> a = a_in;
    // a dot product's partials are independent of the order only with one
    // block of four slices per workgroup
    const bool dot_op = op == kResidNorm || op == kJacobiDot || op == kSpmvDot;
    if (!AMG_STREAM_ALTERNATE || (dot_op && (nslices + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock > grid))
        a.rev = 0;
    const int iw = a.sl_idx8 ? 1 : a.sl_col16 ? 2 : 4;
    const long long entries = (long long)a.rows * (long long)(a.mean_row + 0.5);
    const bool nt = entries * (long long)(sizeof(T) + iw) > (long long)AMG_SELL_NT_BYTES;
    switch (op) {
#define AMG_SELL_LAUNCH(OPV, NTV, IW)                                                                    \
    launch_row_kernel(sell_kernel<T, U, OPV, NTV, IW>, dim3(grid), dim3(kBlock), st, a, g, u, dinv, omega, y, \
                      y2, dot, nslices)
#define AMG_SELL_CASE(OPV)                                                                             \
    case OPV:                                                                                          \
        if constexpr (sizeof(T) == 4 && op_has_dot<OPV>()) break;   /* the FP32 cycle forms no dots */ \
        if (iw == 1) {                                                                                 \
            if (nt) AMG_SELL_LAUNCH(OPV, true, 1);                                                     \
            else AMG_SELL_LAUNCH(OPV, false, 1);                                                       \
        } else if (iw == 2) {                                                                          \
            if (nt) AMG_SELL_LAUNCH(OPV, true, 2);                                                     \
            else AMG_SELL_LAUNCH(OPV, false, 2);                                                       \
        } else {                                                                                       \
            if (nt) AMG_SELL_LAUNCH(OPV, true, 4);                                                     \
            else AMG_SELL_LAUNCH(OPV, false, 4);                                                       \
        }                                                                                              \
        break;
        AMG_SELL_CASE(kSpmv)
        AMG_SELL_CASE(kSpmvAdd)
        AMG_SELL_CASE(kResid)
        AMG_SELL_CASE(kResidNorm)
        AMG_SELL_CASE(kJacobi)
        AMG_SELL_CASE(kJacobiDot)
        AMG_SELL_CASE(kZeroJacobiResid)
        AMG_SELL_CASE(kSpmvDot)
        AMG_SELL_CASE(kSpmvScale)
#undef AMG_SELL_CASE
#undef AMG_SELL_LAUNCH
        default: break;
    }
    return (op == kResidNorm || op == kJacobiDot || op == kSpmvDot) ? grid : 0;
}

template <int U>
int launch_sell_dual_u(const CsrView& a_in, const double* g, const double* u, double* y, const double* g2,
                       const double* u2, double* y2, DotTarget dot, hipStream_t st) {
    const int nslices = (a_in.rows + kSellRows - 1) / kSellRows;
    const int grid = sell_grid(a_in.rows);
    CsrView a = a_in;
    // as for every launch that forms a dot product (launch_sell_u)
    if (!AMG_STREAM_ALTERNATE || (nslices + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock > grid) a.rev = 0;
    const int iw = a.sl_idx8 ? 1 : a.sl_col16 ? 2 : 4;
    const long long entries = (long long)a.rows * (long long)(a.mean_row + 0.5);
    const bool nt = entries * (long long)(sizeof(double) + iw) > (long long)AMG_SELL_NT_BYTES;
#define AMG_DUAL_LAUNCH(NTV, IW)                                                                       \
    launch_row_kernel(sell_dual_resid_kernel<U, NTV, IW>, dim3(grid), dim3(kBlock), st, a, g, u, y, g2, u2, y2, \
                      dot, nslices)
    if (iw == 1) {
        if (nt) AMG_DUAL_LAUNCH(true, 1);
        else AMG_DUAL_LAUNCH(false, 1);
    } else if (iw == 2) {
        if (nt) AMG_DUAL_LAUNCH(true, 2);
        else AMG_DUAL_LAUNCH(false, 2);
    } else {
        if (nt) AMG_DUAL_LAUNCH(true, 4);
        else AMG_DUAL_LAUNCH(false, 4);
    }
#undef AMG_DUAL_LAUNCH
    return grid;
}


template <class T>
int launch_sell(RowOp op, const CsrT<T>& a, const T* g, const T* u, const T* dinv, T omega, T* y, T* y2,
                DotTarget dot, hipStream_t st) {
    const int w = a.sl_maxw;
    if (w <= 8) return launch_sell_u<T, 8>(op, a, g, u, dinv, omega, y, y2, dot, st);
    if (w <= 12) return launch_sell_u<T, 12>(op, a, g, u, dinv, omega, y, y2, dot, st);
    if (w <= 16) return launch_sell_u<T, 16>(op, a, g, u, dinv, omega, y, y2, dot, st);
    if (w <= 20) return launch_sell_u<T, 20>(op, a, g, u, dinv, omega, y, y2, dot, st);
    if (w <= 24) return launch_sell_u<T, 24>(op, a, g, u, dinv, omega, y, y2, dot, st);
    return launch_sell_u<T, 32>(op, a, g, u, dinv, omega, y, y2, dot, st);
}

// one wavefront per slice: 64 x the longest row
__global__ __launch_bounds__(kBlock) void sell_width_kernel(int rows, const int32_t* __restrict__ rp,
                                                            int32_t* __restrict__ width64) {
    const int nslices = (rows + kSellRows - 1) / kSellRows;
    const int sl = blockIdx.x * kSellSlicesPerBlock + (int)threadIdx.x / kSellRows;
    if (sl >= nslices) return;
    const int r = sl * kSellRows + ((int)threadIdx.x & (kSellRows - 1));
    int len = r < rows ? rp[r + 1] - rp[r] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
    if (((int)threadIdx.x & (kSellRows - 1)) == 0) width64[sl] = len * kSellRows;
}

__global__ __launch_bounds__(kBlock) void sell_fill_kernel(int rows, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           const int32_t* __restrict__ off,
                                                           int32_t* __restrict__ col, double* __restrict__ val) {
    const int nslices = (rows + kSellRows - 1) / kSellRows;
    const int sl = blockIdx.x * kSellSlicesPerBlock + (int)threadIdx.x / kSellRows;
    if (sl >= nslices) return;
    const int lane = (int)threadIdx.x & (kSellRows - 1);
    const int r = sl * kSellRows + lane;
    const int o0 = off[sl];
    const int w = (off[sl + 1] - o0) / kSellRows;
    const int b = r < rows ? rp[r] : 0;
    const int len = r < rows ? rp[r + 1] - b : 0;
    // padding repeats the row's last column (an empty row: the row's own
    // index, a valid column of these operators, which have at least as many
    // columns as rows)
    const int last = len > 0 ? ci[b + len - 1] : (r < rows ? r : 0);
    for (int k = 0; k < w; ++k) {
        const int p = o0 + k * kSellRows + lane;
        col[p] = k < len ? ci[b + k] : last;
        val[p] = k < len ? v[b + k] : 0.0;
    }
}

// one wavefront per slice: the slice's distinct offsets column - row in
// order of first appearance (entry slot by slot, lanes in order), added one
// at a time from the lowest lane that misses; then each entry's position
__global__ __launch_bounds__(kBlock) void sell_dictionary_kernel(int rows, const int32_t* __restrict__ off,
                                                                 const int32_t* __restrict__ col,
                                                                 uint8_t* __restrict__ idx8,
                                                                 int32_t* __restrict__ tab, int* wide) {
    __shared__ int table[kSellSlicesPerBlock][kSellRows];
    const int nslices = (rows + kSellRows - 1) / kSellRows;
    const int wv = (int)threadIdx.x / kSellRows;
    const int sl = blockIdx.x * kSellSlicesPerBlock + wv;
    if (sl >= nslices) return;
    const int lane = (int)threadIdx.x & (kSellRows - 1);
    const int r = sl * kSellRows + lane;
    const bool act = r < rows;
    const int o0 = off[sl];
    const int w = (off[sl + 1] - o0) / kSellRows;
    table[wv][lane] = 0;
    int cnt = 0;
    bool overflow = false;
    for (int k = 0; k < w && !overflow; ++k) {
        const int p = o0 + k * kSellRows + lane;
        const int d = act ? col[p] - r : 0;
        int pos = act ? -1 : 0;
        for (int t = 0; t < cnt && pos < 0; ++t)
            if (table[wv][t] == d) pos = t;
        for (;;) {
            const unsigned long long miss = __ballot(pos < 0);
            if (!miss) break;
            if (cnt == kSellRows) {
                overflow = true;
                break;
            }
            const int dl = __shfl(d, __ffsll((long long)miss) - 1, 64);
            if (lane == 0) table[wv][cnt] = dl;
            if (pos < 0 && d == dl) pos = cnt;
            ++cnt;
        }
        idx8[p] = overflow ? (uint8_t)0 : (uint8_t)pos;
    }
    if (lane == 0 && overflow) atomicAdd(wide, 1);
    tab[sl * kSellRows + lane] = table[wv][lane];
}

// one wavefront per slice: smallest and largest column by shuffles, then
// the 16-bit offsets
__global__ __launch_bounds__(kBlock) void sell_compress_kernel(int rows, const int32_t* __restrict__ off,
                                                               const int32_t* __restrict__ col,
                                                               uint16_t* __restrict__ col16,
                                                               int32_t* __restrict__ base, int* wide) {
    const int nslices = (rows + kSellRows - 1) / kSellRows;
    const int sl = blockIdx.x * kSellSlicesPerBlock + (int)threadIdx.x / kSellRows;
    if (sl >= nslices) return;
    const int lane = (int)threadIdx.x & (kSellRows - 1);
    const int o0 = off[sl], o1 = off[sl + 1];
    int mn = INT_MAX, mx = INT_MIN;
    for (int p = o0 + lane; p < o1; p += kSellRows) {
        mn = min(mn, col[p]);
        mx = max(mx, col[p]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, 64));
        mx = max(mx, __shfl_xor(mx, o, 64));
    }
    const bool fits = o1 == o0 || (int64_t)mx - (int64_t)mn <= 65535;
    if (lane == 0) {
        base[sl] = o1 > o0 ? mn : 0;
        if (!fits) atomicAdd(wide, 1);
    }
    for (int p = o0 + lane; p < o1; p += kSellRows) col16[p] = fits ? (uint16_t)(col[p] - mn) : (uint16_t)0;
}

// ---- vector kernels --------------------------------------------------------

constexpr int kVecGrid = 2048;

int vec_grid(int n) { return std::max(1, std::min(kVecGrid, (n + kBlock - 1) / kBlock)); }

__global__ __launch_bounds__(kBlock) void cg_update_xr_kernel(int n, double* __restrict__ x,
                                                              double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ q,
                                                              const double* scal, int i_num,
                                                              int i_den, double* flag, DotTarget dot,
                                                              const double* __restrict__ dinv,
                                                              double omega, double* __restrict__ zs,
                                                              float* __restrict__ r32,
                                                              const float* __restrict__ dinv32,
                                                              float* __restrict__ zs32) {
    const double num = scal[i_num], den = scal[i_den];
    const bool ok = den > 0.0 && std::isfinite(den);
    double contrib = 0.0;
    if (ok) {
        const double alpha = num / den;
        const float omega32 = (float)omega;
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
            x[i] = x[i] + alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            if (zs) zs[i] = omega * (dinv[i] * ri);
            if (r32) {
                const float rf = (float)ri;
                r32[i] = rf;
                if (zs32) zs32[i] = omega32 * (dinv32[i] * rf);
            }
            contrib += ri * ri;
        }
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        *flag = 1.0;
    }
    store_block_partial(contrib, dot.partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void cg_update_p_kernel(int n, double* __restrict__ p,
                                                             const double* __restrict__ z,
                                                             const double* scal, int i_num, int i_den) {
    const double beta = scal[i_num] / scal[i_den];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(kBlock) void scaled_copy_kernel(int n, double* __restrict__ y,
                                                             const double* __restrict__ dinv,
                                                             const double* __restrict__ x, double omega) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        y[i] = omega * (dinv[i] * x[i]);
}

__global__ __launch_bounds__(kBlock) void copy_kernel(int n, double* __restrict__ y,
                                                      const double* __restrict__ x) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = x[i];
}

__global__ __launch_bounds__(kBlock) void fill_u8_kernel(int64_t n, uint8_t* p, uint8_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(int64_t n, unsigned* p, unsigned v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void narrow_kernel(int64_t n, float* __restrict__ y,
                                                        const double* __restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = (float)x[i];
}

// y = (double) x, dot += u . y   (the FP32 preconditioner output entering FP64 CG)
__global__ __launch_bounds__(kBlock) void widen_dot_kernel(int n, double* __restrict__ y,
                                                           const float* __restrict__ x,
                                                           const double* __restrict__ u, DotTarget dot) {
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double v = (double)x[i];
        y[i] = v;
        s += u[i] * v;
    }
    store_block_partial(s, dot.partials, blockIdx.x);
}

// x += (double) e   (iterative refinement with an FP32 correction)
__global__ __launch_bounds__(kBlock) void add_widened_kernel(int n, double* __restrict__ x,
                                                             const float* __restrict__ e) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) x[i] = x[i] + (double)e[i];
}

template <class T>
__global__ __launch_bounds__(kBlock) void scaled_copy_t_kernel(int n, T* __restrict__ y,
                                                               const T* __restrict__ dinv,
                                                               const T* __restrict__ x, T omega) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        y[i] = omega * (dinv[i] * x[i]);
}

template <class T>
__global__ __launch_bounds__(kBlock) void copy_t_kernel(int n, T* __restrict__ y, const T* __restrict__ x) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = x[i];
}

template <class T>
__global__ __launch_bounds__(kBlock) void fill_t_kernel(int64_t n, T* p, T v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// y = Ainv b with the FP64 inverse of the coarsest operator; FP32 in and out
__global__ __launch_bounds__(kBlock) void dense_matvec_mixed_kernel(int n, const double* __restrict__ ainv,
                                                                    const float* __restrict__ b,
                                                                    float* __restrict__ y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    const double* row = ainv + (size_t)i * n;
    for (int j = 0; j < n; ++j) s += row[j] * (double)b[j];
    y[i] = (float)s;
}

__global__ __launch_bounds__(kBlock) void fill_f64_kernel(int64_t n, double* p, double v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void dot_kernel(int n, const double* __restrict__ a,
                                                     const double* __restrict__ b, DotTarget dot) {
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) s += a[i] * b[i];
    store_block_partial(s, dot.partials, blockIdx.x);
}

// Start from x0 = 0: x = 0, r = b (the residual of the zero vector) and the
// block partials of ||b||^2.
__global__ __launch_bounds__(kBlock) void zero_guess_start_kernel(int n, const double* __restrict__ b,
                                                                  double* __restrict__ x, double* __restrict__ r,
                                                                  DotTarget dot) {
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        s += bi * bi;
    }
    store_block_partial(s, dot.partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void dense_matvec_kernel(int n, const double* __restrict__ ainv,
                                                              const double* __restrict__ b,
                                                              double* __restrict__ y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    const double* row = ainv + (size_t)i * n;
    for (int j = 0; j < n; ++j) s += row[j] * b[j];
    y[i] = s;
}

__global__ __launch_bounds__(kBlock) void inverse_diagonal_kernel(CsrView a, double* __restrict__ dinv,
                                                                  float* __restrict__ dinv32) {
    constexpr int W = 8;
    const int i = blockIdx.x * (kBlock / W) + threadIdx.x / W;
    const int lane = threadIdx.x & (W - 1);
    double d = 0.0;
    if (i < a.rows)
        for (int p = a.rp[i] + lane; p < a.rp[i + 1]; p += W)
            if (a.ci[p] == i) d = a.v[p];
    d = sub_sum<W>(d);          // exactly one lane holds the diagonal
    if (i < a.rows && lane == 0) {
        dinv[i] = 1.0 / d;
        if (dinv32) dinv32[i] = (float)(1.0 / d);
    }
}

// ---- sparsification kernels --------------------------------------------------

__device__ __forceinline__ int find_in_row(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                           int row, int col) {
    int lo = rp[row], hi = rp[row + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = ci[mid];
        if (c == col) return mid;
        if (c < col) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// One wave per coarse row I, lanes over the entries l of the fine row c(I):
// every (I, J) with J in P's row l is marked together with (J, I).  The marks
// form a set (idempotent byte stores), so the lanes need no order.
constexpr int kMarkGridCap = 65536;

__global__ __launch_bounds__(kBlock) void mark_minimal_pattern_kernel(
    int nc, const int32_t* __restrict__ c_points, const int32_t* __restrict__ afine_rp,
    const int32_t* __restrict__ afine_ci, const int32_t* __restrict__ p_rp,
    const int32_t* __restrict__ p_ci, const int32_t* __restrict__ ac_rp,
    const int32_t* __restrict__ ac_ci, uint8_t* in_m, int* missing) {
    constexpr int kWaves = kBlock / 64;
    const int lane = threadIdx.x & 63;
    for (int I = blockIdx.x * kWaves + (int)(threadIdx.x >> 6); I < nc; I += gridDim.x * kWaves) {
        const int f = c_points[I];
        for (int p = afine_rp[f] + lane; p < afine_rp[f + 1]; p += 64) {
            const int l = afine_ci[p];
            for (int q = p_rp[l]; q < p_rp[l + 1]; ++q) {
                const int J = p_ci[q];
                const int a = find_in_row(ac_rp, ac_ci, I, J);
                const int b = find_in_row(ac_rp, ac_ci, J, I);
                if (a < 0 || b < 0) {
                    *missing = 1;
                    continue;
                }
                in_m[a] = 1;
                in_m[b] = 1;
            }
        }
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void row_max_kernel(CsrView a, double* __restrict__ m) {
    const int row = blockIdx.x * (kBlock / W) + threadIdx.x / W;
    const int lane = threadIdx.x & (W - 1);
    double mx = 0.0;
    if (row < a.rows)
        for (int p = a.rp[row] + lane; p < a.rp[row + 1]; p += W)
            if (a.ci[p] != row) mx = fmax(mx, fabs(a.v[p]));
    mx = sub_max<W>(mx);
    if (row < a.rows && lane == 0) m[row] = mx;
}

template <int W>
__device__ __forceinline__ void keep_count_rows(const CsrView& a, const uint8_t* __restrict__ in_m,
                                                const double* __restrict__ m, double gamma,
                                                uint8_t* __restrict__ keep, int32_t* __restrict__ cnt,
                                                int32_t* __restrict__ bsum, int blk) {
    const int row = blk * (kBlock / W) + threadIdx.x / W;
    const int lane = threadIdx.x & (W - 1);
    int c = 0;
    if (row < a.rows) {
        // fl(gamma * m_i): one rounding, compared as is (no contraction is possible in a compare)
        const double ti = gamma * m[row];
        for (int p = a.rp[row] + lane; p < a.rp[row + 1]; p += W) {
            const int j = a.ci[p];
            const double av = fabs(a.v[p]);
            const double tj = gamma * m[j];
            const bool k = (j == row) || in_m[p] || av >= ti || av >= tj;
            keep[p] = k ? 1 : 0;
            c += k ? 1 : 0;
        }
    }
    c = sub_sum_int<W>(c);
    if (row < a.rows && lane == 0) cnt[row] = c;
    if (bsum) {
        // the block's kept entries (its kBlock / W <= 64 rows added by one wave)
        __shared__ int rows_c[kBlock / W];
        if (lane == 0) rows_c[threadIdx.x / W] = row < a.rows ? c : 0;
        __syncthreads();
        if (threadIdx.x < 64) {
            int v = (int)threadIdx.x < kBlock / W ? rows_c[threadIdx.x] : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (threadIdx.x == 0) bsum[blk] = v;
        }
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void keep_count_kernel(CsrView a, const uint8_t* __restrict__ in_m,
                                                            const double* __restrict__ m, double gamma,
                                                            uint8_t* __restrict__ keep,
                                                            int32_t* __restrict__ cnt,
                                                            int32_t* __restrict__ bsum) {
    keep_count_rows<W>(a, in_m, m, gamma, keep, cnt, bsum, blockIdx.x);
}

// The first position of each row in the compacted operator: the block's
// offset (the exclusive scan of the blocks' kept counts, boff) plus the
// kept counts of the block's earlier rows (a shuffle scan over its <= 64
// rows); the row pointers of the compacted operator are written here too.
template <int W>
__device__ __forceinline__ void compact_lump_rows(const CsrView& a, const uint8_t* __restrict__ keep,
                                                  const int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ boff,
                                                  int32_t* __restrict__ new_rp, int32_t* __restrict__ new_ci,
                                                  double* __restrict__ new_v, double* __restrict__ dinv,
                                                  float* __restrict__ new_v32, float* __restrict__ dinv32,
                                                  int blk) {
    constexpr int R = kBlock / W;   // rows per block
    __shared__ int row_out[R];
    const int row = blk * R + threadIdx.x / W;
    const int lane = threadIdx.x & (W - 1);
    if (threadIdx.x < 64) {
        const int r = blk * R + (int)threadIdx.x;
        const int c = ((int)threadIdx.x < R && r < a.rows) ? cnt[r] : 0;
        int incl = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if ((int)threadIdx.x >= off) incl += t;
        }
        if ((int)threadIdx.x < R) {
            const int o = boff[blk] + incl - c;
            row_out[threadIdx.x] = o;
            if (r < a.rows) new_rp[r] = o;
            if (r == a.rows - 1) new_rp[a.rows] = o + c;
        }
    }
    __syncthreads();
    const int shift = (threadIdx.x & 63) & ~(W - 1);
    const unsigned long long lanes_below = (lane == 0) ? 0ull : ((1ull << lane) - 1ull);
    double dropped = 0.0, diag = 0.0;
    int diag_pos = -1;
    int written = 0;
    const int beg = row < a.rows ? a.rp[row] : 0;
    const int end = row < a.rows ? a.rp[row + 1] : 0;
    const int out0 = row < a.rows ? row_out[threadIdx.x / W] : 0;
    for (int base = beg; base < end; base += W) {
        const int p = base + lane;
        bool k = false;
        int j = -1;
        double v = 0.0;
        if (p < end) {
            j = a.ci[p];
            v = a.v[p];
            k = keep[p] != 0;
        }
        unsigned long long bits = __ballot(k);
        bits = (W == 64) ? bits : ((bits >> shift) & ((1ull << (W & 63)) - 1ull));
        if (k) {
            const int w = out0 + written + __popcll(bits & lanes_below);
            new_ci[w] = j;
            new_v[w] = v;
            if (new_v32) new_v32[w] = (float)v;
            if (j == row) { diag_pos = w; diag = v; }
        } else if (p < end && j != row) {
            dropped += v;
        }
        written += __popcll(bits);
    }
    dropped = sub_sum<W>(dropped);
    if (diag_pos >= 0) {
        const double d = diag + dropped;
        new_v[diag_pos] = d;
        dinv[row] = 1.0 / d;
        if (new_v32) {
            new_v32[diag_pos] = (float)d;
            dinv32[row] = (float)(1.0 / d);
        }
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void compact_lump_kernel(CsrView a, const uint8_t* __restrict__ keep,
                                                              const int32_t* __restrict__ cnt,
                                                              const int32_t* __restrict__ boff,
                                                              int32_t* __restrict__ new_rp,
                                                              int32_t* __restrict__ new_ci,
                                                              double* __restrict__ new_v,
                                                              double* __restrict__ dinv,
                                                              float* __restrict__ new_v32,
                                                              float* __restrict__ dinv32) {
    compact_lump_rows<W>(a, keep, cnt, boff, new_rp, new_ci, new_v, dinv, new_v32, dinv32, blockIdx.x);
}

// Several small levels in one launch each (64 lanes a row): block b belongs to
// the last level whose first block is <= b, and runs that level's rows as
// the per-level kernels do.
__device__ __forceinline__ int merged_level(const SparsifyLevels& L) {
    int li = 0;
    for (int k = 1; k < L.count; ++k)
        if ((int)blockIdx.x >= L.lv[k].block0) li = k;
    return li;
}

__global__ __launch_bounds__(kBlock) void keep_count_merged_kernel(SparsifyLevels L) {
    const SparsifyLevel& v = L.lv[merged_level(L)];
    keep_count_rows<64>(v.a, v.in_m, v.m, v.gamma, v.keep, v.cnt, v.bsum, (int)blockIdx.x - v.block0);
}

__global__ __launch_bounds__(kBlock) void compact_lump_merged_kernel(SparsifyLevels L) {
    const SparsifyLevel& v = L.lv[merged_level(L)];
    compact_lump_rows<64>(v.a, v.keep, v.cnt, v.bsum, v.new_rp, v.new_ci, v.new_v, v.dinv, v.new_v32, v.dinv32,
                          (int)blockIdx.x - v.block0);
}

// Inverse of the dense coarsest operator (n <= kDenseInvMax) by Gauss-Jordan
// elimination with partial pivoting in LDS, one block.  *singular = 1 if a
// pivot is zero.  Per column c, three steps between barriers: the pivot row
// (one wave, a DPP maximum and a ballot), then the scaled pivot row
// P = M[pr] / d (and V's), the multipliers F[i] = M[i][c] and the row swap,
// then every element M[i][j] -= F[i] P[j] (V likewise), row c = P and column
// c zeroed.  The operations on every element are those of the textbook order
// (swap, scale row c, eliminate with the scaled row, zero column c).
constexpr int kDenseInvMax = 64;
constexpr int kDenseInvThreads = 1024;
constexpr int kDenseInvPerThread = kDenseInvMax * kDenseInvMax / kDenseInvThreads;

// The largest unsigned 64-bit value of the wave, in every lane: an inclusive
// maximum scan within each row of 16 lanes (DPP row_shr 1, 2, 4, 8), then
// row_bcast 15 and 31 carry the row maxima up to lane 63, which is read
// back.  A lane whose DPP source does not exist receives 0, the identity.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
    const unsigned l2 = (unsigned)__builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
    const unsigned h2 = (unsigned)__builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
    return ((unsigned long long)h2 << 32) | l2;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    unsigned long long t;
    t = dpp_u64<0x111, 0xf>(v); v = t > v ? t : v;   // row_shr:1
    t = dpp_u64<0x112, 0xf>(v); v = t > v ? t : v;   // row_shr:2
    t = dpp_u64<0x114, 0xf>(v); v = t > v ? t : v;   // row_shr:4
    t = dpp_u64<0x118, 0xf>(v); v = t > v ? t : v;   // row_shr:8
    t = dpp_u64<0x142, 0xa>(v); v = t > v ? t : v;   // row_bcast:15 into rows 1, 3
    t = dpp_u64<0x143, 0xc>(v); v = t > v ? t : v;   // row_bcast:31 into rows 2, 3
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

__global__ __launch_bounds__(kDenseInvThreads) void dense_invert_kernel(CsrView a, double* __restrict__ inv,
                                                                        int* singular) {
    __shared__ double M[kDenseInvMax][kDenseInvMax + 1];
    __shared__ double V[kDenseInvMax][kDenseInvMax + 1];
    __shared__ double P[kDenseInvMax], PV[kDenseInvMax], F[kDenseInvMax];
    __shared__ int piv;
    __shared__ double pivd;
    const int n = a.rows;
    for (int t = threadIdx.x; t < n * n; t += kDenseInvThreads) {
        const int i = t / n, j = t % n;
        M[i][j] = 0.0;
        V[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kDenseInvThreads)
        for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) M[i][a.ci[p]] = a.v[p];
    // the elements this thread updates, (row, column) in row-major order
    int ei[kDenseInvPerThread], ej[kDenseInvPerThread];
#pragma unroll
    for (int q = 0; q < kDenseInvPerThread; ++q) {
        const int e = (int)threadIdx.x + q * kDenseInvThreads;
        ei[q] = e < n * n ? e / n : -1;
        ej[q] = e < n * n ? e % n : 0;
    }
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        if (threadIdx.x < 64) {
            // pivot: the first row i >= c of largest |M[i][c]| (a NaN never
            // wins, except at row c, where the scan starts), found by one wave:
            // lane l holds row c + l (n <= 64) with the key 0 (no candidate) or
            // the magnitude's bit pattern + 1, which orders non-negative
            // doubles as their values; the wave's largest key, then the lowest
            // lane holding it
            const int i = c + (int)threadIdx.x;
            unsigned long long key = 0ull;
            if (i < n) {
                const double m = fabs(M[i][c]);
                if (m == m) key = (unsigned long long)__double_as_longlong(m) + 1ull;
                else if (i == c) key = (unsigned long long)__double_as_longlong(HUGE_VAL) + 1ull;
            }
            const unsigned long long hits = __ballot(key == wave_max_u64(key));
            const int best = c + (__ffsll((long long)hits) - 1);
            if (threadIdx.x == 0) {
                piv = best;
                pivd = M[best][c];
                if (M[best][c] == 0.0) *singular = 1;
            }
        }
        __syncthreads();
        const int pr = piv;
        const double d = pivd;
        const int t = threadIdx.x;
        if (t < n) {
            // column t of the pivot row, scaled; the old row c moves to row pr
            const double mp = M[pr][t], vp = V[pr][t];
            P[t] = mp / d;
            PV[t] = vp / d;
            if (pr != c) {
                M[pr][t] = M[c][t];
                V[pr][t] = V[c][t];
            }
        } else if (t >= 64 && t - 64 < n) {
            // multiplier of row i after the swap
            const int i = t - 64;
            F[i] = (i == pr) ? M[c][c] : M[i][c];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kDenseInvPerThread; ++q) {
            const int i = ei[q], j = ej[q];
            if (i < 0) continue;
            if (i == c) {
                M[c][j] = P[j];
                V[c][j] = PV[j];
            } else {
                const double f = F[i];
                if (j == c) M[i][c] = 0.0;
                else M[i][j] -= f * P[j];
                V[i][j] -= f * PV[j];
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < n * n; t += kDenseInvThreads) inv[t] = V[t / n][t % n];
}

// Single-workgroup tail of the V-cycle (see kernels.hpp).  Rows are handled
// by 8-lane subgroups; every step ends with a workgroup barrier, which also
// makes the step's writes visible to the next step.  The cycle runs either on
// the arrays in memory (LDS = false) or on copies in LDS (LDS = true), whose
// generic pointers tail_ld / tail_st turn into LDS addresses so that the
// accesses are LDS instructions rather than flat ones (a flat access counts
// against the LDS wait counter as well and keeps the next LDS access waiting
// for it).
constexpr int kTailBlock = 1024;
constexpr int kTailW = 8;

template <bool LDS, class U>
__device__ __forceinline__ U tail_ld(const U* p, int i) {
    if constexpr (LDS) return ((const __attribute__((address_space(3))) U*)p)[i];
    else return p[i];
}

template <bool LDS, class U>
__device__ __forceinline__ void tail_st(U* p, int i, U v) {
    if constexpr (LDS) ((__attribute__((address_space(3))) U*)p)[i] = v;
    else p[i] = v;
}

template <class T, int OPT, bool LDS>
__device__ __forceinline__ void tail_rows(const TailCsr<T>& a, const T* __restrict__ g,
                                          const T* u, const T* __restrict__ dinv,
                                          T omega, T* y, T* y2) {
    // OPT 0: y = u - A g        (residual)
    // OPT 1: y = A g, y2 = omega dinv y   (restriction writing the prescaled sweep)
    // OPT 2: y = A g            (restriction onto the coarsest level)
    // OPT 3: y = u + A g        (interpolation and correction, in place)
    // OPT 4: y = g + omega dinv (u - A g)   (post-smoothing sweep)
    const int lane = threadIdx.x & (kTailW - 1);
    for (int row = threadIdx.x / kTailW; row < a.rows; row += kTailBlock / kTailW) {
        const int end = tail_ld<LDS>(a.rp, row + 1);
        int p = tail_ld<LDS>(a.rp, row) + lane;
        T s = T(0);
        // four entries' loads issued before their products are summed (in
        // entry order, as the one-entry loop below does)
        for (; p + 3 * kTailW < end; p += 4 * kTailW) {
            int c[4];
            T v[4], x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = tail_ld<LDS>(a.ci, p + q * kTailW);
                v[q] = tail_ld<LDS>(a.v, p + q * kTailW);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = tail_ld<LDS>(g, c[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q) s += v[q] * x[q];
        }
        for (; p < end; p += kTailW) s += tail_ld<LDS>(a.v, p) * tail_ld<LDS>(g, tail_ld<LDS>(a.ci, p));
        s = sub_sum<kTailW>(s);
        if (lane == 0) {
            if constexpr (OPT == 0) tail_st<LDS>(y, row, tail_ld<LDS>(u, row) - s);
            else if constexpr (OPT == 1) {
                tail_st<LDS>(y, row, s);
                tail_st<LDS>(y2, row, omega * (tail_ld<LDS>(dinv, row) * s));
            } else if constexpr (OPT == 2) tail_st<LDS>(y, row, s);
            else if constexpr (OPT == 3) tail_st<LDS>(y, row, tail_ld<LDS>(u, row) + s);
            else
                tail_st<LDS>(y, row, tail_ld<LDS>(g, row) +
                                         omega * tail_ld<LDS>(dinv, row) * (tail_ld<LDS>(u, row) - s));
        }
    }
}

template <class T, bool LDS>
__device__ __forceinline__ void tail_cycle(const TailArgs<T>& t) {
    const int last = t.count - 1;
    for (int k = 0; k < last; ++k) {
        const TailLevel<T>& L = t.lv[k];
        tail_rows<T, 0, LDS>(L.A, L.x, L.b, nullptr, t.omega, L.r, nullptr);
        __syncthreads();
        const TailLevel<T>& N = t.lv[k + 1];
        if (k + 1 < last) tail_rows<T, 1, LDS>(L.R, L.r, nullptr, N.dinv, t.omega, N.b, N.x);
        else tail_rows<T, 2, LDS>(L.R, L.r, nullptr, nullptr, t.omega, N.b, nullptr);
        __syncthreads();
    }
    {
        const TailLevel<T>& C = t.lv[last];
        const int n = C.A.rows;
        for (int i = threadIdx.x; i < n; i += kTailBlock) {
            double s = 0.0;
            for (int j = 0; j < n; ++j)
                s += tail_ld<LDS>(t.coarse_inv, i * n + j) * (double)tail_ld<LDS>(C.b, j);
            tail_st<LDS>(C.x, i, (T)s);
        }
        __syncthreads();
    }
    for (int k = last - 1; k >= 0; --k) {
        const TailLevel<T>& L = t.lv[k];
        const T* xc = (k + 1 == last) ? t.lv[k + 1].x : t.lv[k + 1].xt;
        tail_rows<T, 3, LDS>(L.P, xc, L.x, nullptr, t.omega, L.x, nullptr);
        __syncthreads();
        tail_rows<T, 4, LDS>(L.A, L.x, L.b, L.dinv, t.omega, L.xt, nullptr);
        __syncthreads();
    }
}

template <class T>
__global__ __launch_bounds__(kTailBlock) void coarse_tail_kernel(TailArgs<T> t) {
    tail_cycle<T, false>(t);
}

// The staged tail: the host lays the arrays out in LDS (every array on a
// 16-byte boundary, level by level A's row pointers, columns and values,
// dinv, b, x, xt, r, then R's and P's arrays; last the coarsest inverse) and
// lists the runs of 4-byte words to copy there, cut into chunks of 64 words
// (one wave-wide load each) numbered in one flat order.
constexpr int kTailLdsLevels = 6;
constexpr int kTailLdsSegs = 10 * kTailLdsLevels + 3;
constexpr int kTailWaves = kTailBlock / 64;
struct TailSeg {
    const uint32_t* src;
    uint32_t begin;        // the run's first chunk in the flat order
    uint32_t words;
    uint32_t dst;          // its byte offset in LDS
};
struct TailLdsOff {        // byte offsets in LDS of one level's arrays
    uint32_t a_rp, a_ci, a_v, dinv, b, x, xt, r, r_rp, r_ci, r_v, p_rp, p_ci, p_v;
};
template <class T>
struct TailLdsArgs {
    TailArgs<T> t;         // the arrays in memory
    TailLdsOff off[kTailLdsLevels];
    uint32_t inv_off;
    uint32_t chunks;       // chunks copied; wave w takes the w-th of kTailWaves equal ranges
    int nseg;
    int wave_seg[kTailWaves];            // the run holding each wave's first chunk
    TailSeg seg[kTailLdsSegs + 1];       // closed by a run that begins at chunks
};

inline size_t tail_align(size_t b) { return (b + 15) & ~(size_t)15; }

// Fills a's layout and copy list; returns the LDS bytes the layout takes.
template <class T>
size_t tail_lds_plan(const TailArgs<T>& t, TailLdsArgs<T>& a) {
    a.t = t;
    size_t off = 0;
    uint32_t chunks = 0;
    int count = 0;
    auto place = [&](const void* src, size_t bytes) {
        const uint32_t at = (uint32_t)off;
        if (src && bytes) {
            const uint32_t words = (uint32_t)(bytes / 4);
            a.seg[count++] = TailSeg{static_cast<const uint32_t*>(src), chunks, words, at};
            chunks += (words + 63) / 64;
        }
        off += tail_align(bytes);
        return at;
    };
    for (int k = 0; k < t.count; ++k) {
        const TailLevel<T>& G = t.lv[k];
        TailLdsOff& o = a.off[k];
        const size_t n = (size_t)G.A.rows;
        o.a_rp = place(G.A.rp, (n + 1) * 4);
        o.a_ci = place(G.A.ci, (size_t)G.A.cap * 4);
        o.a_v = place(G.A.v, (size_t)G.A.cap * sizeof(T));
        o.dinv = place(G.dinv, n * sizeof(T));
        o.b = place(k == 0 ? G.b : nullptr, n * sizeof(T));
        o.x = place(k == 0 ? G.x : nullptr, n * sizeof(T));
        o.xt = place(nullptr, n * sizeof(T));
        o.r = place(nullptr, n * sizeof(T));
        o.r_rp = o.r_ci = o.r_v = o.p_rp = o.p_ci = o.p_v = 0;
        if (k + 1 < t.count) {
            o.r_rp = place(G.R.rp, ((size_t)G.R.rows + 1) * 4);
            o.r_ci = place(G.R.ci, (size_t)G.R.cap * 4);
            o.r_v = place(G.R.v, (size_t)G.R.cap * sizeof(T));
            o.p_rp = place(G.P.rp, ((size_t)G.P.rows + 1) * 4);
            o.p_ci = place(G.P.ci, (size_t)G.P.cap * 4);
            o.p_v = place(G.P.v, (size_t)G.P.cap * sizeof(T));
        }
    }
    const size_t nl = (size_t)t.lv[t.count - 1].A.rows;
    a.inv_off = place(t.coarse_inv, nl * nl * 8);
    a.seg[count] = TailSeg{nullptr, chunks, 0, 0};
    a.nseg = count;
    a.chunks = chunks;
    const uint32_t per = (chunks + kTailWaves - 1) / kTailWaves;
    for (int w = 0, si = 0; w < kTailWaves; ++w) {
        const uint32_t c = (uint32_t)w * per;
        while (si + 1 < count && c >= a.seg[si + 1].begin) ++si;
        a.wave_seg[w] = si;
    }
    return off;
}

template <class T>
__global__ __launch_bounds__(kTailBlock) void coarse_tail_lds_kernel(TailLdsArgs<T> a) {
    extern __shared__ __align__(16) unsigned char tail_smem[];
    // the arguments with their pointers redirected into LDS, and the copy list
    // closed by a run that starts at the end
    __shared__ __align__(16) unsigned char args_raw[sizeof(TailArgs<T>)];
    __shared__ TailSeg segs[kTailLdsSegs + 1];
    TailArgs<T>& s = *reinterpret_cast<TailArgs<T>*>(args_raw);
    const TailArgs<T>& t = a.t;
    const int tid = threadIdx.x;
    if (tid < t.count) {
        const TailLevel<T>& G = t.lv[tid];
        const TailLdsOff& o = a.off[tid];
        TailLevel<T> L;
        L.A = TailCsr<T>{reinterpret_cast<const int32_t*>(tail_smem + o.a_rp),
                         reinterpret_cast<const int32_t*>(tail_smem + o.a_ci),
                         reinterpret_cast<const T*>(tail_smem + o.a_v), G.A.rows, G.A.cap};
        L.R = TailCsr<T>{reinterpret_cast<const int32_t*>(tail_smem + o.r_rp),
                         reinterpret_cast<const int32_t*>(tail_smem + o.r_ci),
                         reinterpret_cast<const T*>(tail_smem + o.r_v), G.R.rows, G.R.cap};
        L.P = TailCsr<T>{reinterpret_cast<const int32_t*>(tail_smem + o.p_rp),
                         reinterpret_cast<const int32_t*>(tail_smem + o.p_ci),
                         reinterpret_cast<const T*>(tail_smem + o.p_v), G.P.rows, G.P.cap};
        L.dinv = reinterpret_cast<const T*>(tail_smem + o.dinv);
        L.b = reinterpret_cast<T*>(tail_smem + o.b);
        L.x = reinterpret_cast<T*>(tail_smem + o.x);
        L.xt = reinterpret_cast<T*>(tail_smem + o.xt);
        L.r = reinterpret_cast<T*>(tail_smem + o.r);
        s.lv[tid] = L;
    }
    if (tid == 0) {
        s.count = t.count;
        s.coarse_inv = reinterpret_cast<const double*>(tail_smem + a.inv_off);
        s.omega = t.omega;
    }
    if (tid <= a.nseg) segs[tid] = a.seg[tid];
    __syncthreads();
    // the copy: each wave takes a range of chunks and loads each straight
    // into LDS with one wave-wide load, none waited for until the end
    {
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        const uint32_t per = (a.chunks + kTailWaves - 1) / kTailWaves;
        uint32_t c = (uint32_t)wave * per;
        const uint32_t cend = min(a.chunks, c + per);
        int si = a.wave_seg[wave];
        while (c < cend) {
            const uint32_t next = __builtin_amdgcn_readfirstlane(segs[si + 1].begin);
            if (c >= next) {
                ++si;
                continue;
            }
            const uint32_t begin = __builtin_amdgcn_readfirstlane(segs[si].begin);
            const uint32_t words = __builtin_amdgcn_readfirstlane(segs[si].words);
            const uint32_t dst = __builtin_amdgcn_readfirstlane(segs[si].dst);
            const uint32_t* src = segs[si].src;
            for (const uint32_t stop = min(next, cend); c < stop; ++c) {
                const uint32_t w = (c - begin) * 64;
                if (w + lane < words)
                    __builtin_amdgcn_global_load_lds(
                        (const __attribute__((address_space(1))) void*)(src + w + lane),
                        (__attribute__((address_space(3))) void*)(tail_smem + dst + w * 4), 4, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    tail_cycle<T, true>(s);
    const int n0 = t.lv[0].A.rows;
    const T* xt = s.lv[0].xt;
    for (int i = tid; i < n0; i += kTailBlock) t.lv[0].xt[i] = tail_ld<true>(xt, i);
}

// exclusive scan: 1024 items per block in pass 1 and 3
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_exclusive_scan_int(int v, int* lds, int* total) {
    // Hillis-Steele over the block in LDS
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const int t = threadIdx.x >= o ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += t;
        __syncthreads();
    }
    const int incl = lds[threadIdx.x];
    *total = lds[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void scan_pass1_kernel(int n, const int32_t* __restrict__ cnt,
                                                            int32_t* __restrict__ bsum) {
    __shared__ int lds[kBlock];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += (base + k < n) ? cnt[base + k] : 0;
    int tot;
    block_exclusive_scan_int(s, lds, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void scan_pass2_kernel(int nb, int32_t* bsum) {
    __shared__ int lds[1024];
    const int per = (nb + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(nb, lo + per);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += bsum[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int t = threadIdx.x >= o ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += t;
        __syncthreads();
    }
    int run = lds[threadIdx.x] - s;
    for (int i = lo; i < hi; ++i) {
        const int v = bsum[i];
        bsum[i] = run;
        run += v;
    }
}

// in-place exclusive scans of several arrays, one workgroup of 1,024 threads
// each (every thread a contiguous range)
__global__ __launch_bounds__(1024) void scan_jobs_kernel(ScanJobs jobs) {
    __shared__ int lds[1024];
    int32_t* data = jobs.data[blockIdx.x];
    const int nb = jobs.n[blockIdx.x];
    const int per = (nb + 1023) / 1024;
    const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += data[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int t = threadIdx.x >= o ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += t;
        __syncthreads();
    }
    int run = lds[threadIdx.x] - s;
    for (int i = lo; i < hi; ++i) {
        const int v = data[i];
        data[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kBlock) void scan_pass3_kernel(int n, const int32_t* __restrict__ cnt,
                                                            const int32_t* __restrict__ boff,
                                                            int32_t* __restrict__ out) {
    __shared__ int lds[kBlock];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? cnt[base + k] : 0;
        s += v[k];
    }
    int tot;
    int run = block_exclusive_scan_int(s, lds, &tot) + boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
        if (base + k == n - 1) out[n] = run;
    }
}

// rows per block: the largest power of two whose mean nonzero count fits one pass
int stream_rows_per_block(double mean) {
    int rb = 256;
    while (rb > 16 && rb * mean > AMG_STREAM_FILL * kStreamCap) rb /= 2;
    return rb;
}

// The LDS-staged kernel wins on the large operators with rows of up to a few
// dozen entries (measured on the 128^3 hierarchy: A_0, A_1, P_0, R_0, R_1 and
// the sparsified level 2); with longer rows or too few row blocks to fill 256
// CUs the subgroup kernel wins.
template <class T>
bool use_stream_kernel(const CsrT<T>& a) {
#if AMG_USE_STREAM >= 0
    return AMG_USE_STREAM != 0;
#else
    const int rb = stream_rows_per_block(a.mean_row);
    return a.mean_row <= AMG_STREAM_MAX_ROW && (a.rows + rb - 1) / rb >= 1024;
#endif
}

// 16-byte packed loads pay off on the operators with the shortest rows
// (measured: A_0, P_l, R_0 gain 5-8%; the 19-point A_1 loses).
template <class T, bool VEC4>
int launch_stream_v(RowOp op, const CsrT<T>& a, const T* g, const T* u, const T* dinv,
                    T omega, T* y, T* y2, DotTarget dot, hipStream_t st) {
    switch (stream_rows_per_block(a.mean_row)) {
        case 256: return launch_stream_rb<T, 256, VEC4>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 128: return launch_stream_rb<T, 128, VEC4>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 64: return launch_stream_rb<T, 64, VEC4>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 32: return launch_stream_rb<T, 32, VEC4>(op, a, g, u, dinv, omega, y, y2, dot, st);
        default: return launch_stream_rb<T, 16, VEC4>(op, a, g, u, dinv, omega, y, y2, dot, st);
    }
}

template <class T>
int launch_stream_any(RowOp op, const CsrT<T>& a, const T* g, const T* u, const T* dinv,
                      T omega, T* y, T* y2, DotTarget dot, hipStream_t st) {
#if AMG_VEC4 >= 0
    constexpr bool kForce = AMG_VEC4 != 0;
    if (kForce) return launch_stream_v<T, true>(op, a, g, u, dinv, omega, y, y2, dot, st);
    return launch_stream_v<T, false>(op, a, g, u, dinv, omega, y, y2, dot, st);
#else
    if (a.mean_row <= 10.0) return launch_stream_v<T, true>(op, a, g, u, dinv, omega, y, y2, dot, st);
    return launch_stream_v<T, false>(op, a, g, u, dinv, omega, y, y2, dot, st);
#endif
}

}  // namespace

// Lanes per row: the power of two nearest (in log scale) to AMG_WIDTH_SCALE
// times the mean row length, i.e. about two nonzeros per lane.  Measured on
// the Poisson hierarchies this beats one nonzero per lane (more subgroups
// and shuffles per byte) and four (fewer independent loads per wavefront).
int pick_width(double mean) {
    const double t = std::max(mean * AMG_WIDTH_SCALE, 1.0);
    int w = 1 << (int)std::lround(std::log2(t));
    return std::max(AMG_MIN_WIDTH, std::min(64, w));
}

int max_row_launch_blocks() { return std::max(kRowGridCap, (int)AMG_SELL_GRID_CAP); }

int row_launch_blocks(int rows, int width) {
    const int rpb = kBlock / width;
    const int R = width <= 16 ? AMG_RIF : 1;
    const int ntiles = std::max(1, (rows + rpb - 1) / rpb);
    return round_up8(std::min((ntiles + R - 1) / R, kRowGridCap));
}

template <class T>
int launch_row_op_t(RowOp op, int width, const CsrT<T>& a, const T* g, const T* u,
                    const T* dinv, T omega, T* y, T* y2, DotTarget dot, hipStream_t st) {
    if (AMG_SELL && a.sl_off) return launch_sell(op, a, g, u, dinv, omega, y, y2, dot, st);
    if (use_stream_kernel(a)) return launch_stream_any(op, a, g, u, dinv, omega, y, y2, dot, st);
    switch (width) {
        case 1: return launch_row_w<T, 1>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 2: return launch_row_w<T, 2>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 4: return launch_row_w<T, 4>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 8: return launch_row_w<T, 8>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 16: return launch_row_w<T, 16>(op, a, g, u, dinv, omega, y, y2, dot, st);
        case 32: return launch_row_w<T, 32>(op, a, g, u, dinv, omega, y, y2, dot, st);
        default: return launch_row_w<T, 64>(op, a, g, u, dinv, omega, y, y2, dot, st);
    }
}

int launch_row_op(RowOp op, int width, const CsrView& a, const double* g, const double* u,
                  const double* dinv, double omega, double* y, double* y2, DotTarget dot,
                  hipStream_t st) {
    return launch_row_op_t<double>(op, width, a, g, u, dinv, omega, y, y2, dot, st);
}

void launch_row_op(RowOp op, int width, const CsrView32& a, const float* g, const float* u,
                   const float* dinv, float omega, float* y, float* y2, hipStream_t st) {
    launch_row_op_t<float>(op, width, a, g, u, dinv, omega, y, y2, DotTarget{nullptr, nullptr}, st);
}

void launch_dot_finish(const DotTarget& dot, int nparts, hipStream_t st) { finish_dot(dot, nparts, st); }

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}

bool clear_launch_events() {
    const bool pending = t_ev_start != nullptr;
    t_ev_start = t_ev_stop = nullptr;
    return pending;
}

void launch_cg_update_xr(int n, double* x, double* r, const double* p, const double* q,
                         const double* scal, int i_num, int i_den, double* flag, DotTarget dot,
                         const double* dinv, double omega, double* zs, float* r32,
                         const float* dinv32, float* zs32, hipStream_t st) {
    hipLaunchKernelGGL(cg_update_xr_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, x, r, p, q,
                       scal, i_num, i_den, flag, dot, dinv, omega, zs, r32, dinv32, zs32);
    finish_dot(dot, vec_grid(n), st);
}

void launch_cg_update_p(int n, double* p, const double* z, const double* scal, int i_num,
                        int i_den, hipStream_t st) {
    hipLaunchKernelGGL(cg_update_p_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, p, z, scal,
                       i_num, i_den);
}

void launch_scaled_copy(int n, double* y, const double* dinv, const double* x, double omega,
                        hipStream_t st) {
    hipLaunchKernelGGL(scaled_copy_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, y, dinv, x, omega);
}

__global__ __launch_bounds__(256) void publish_scalars_kernel(int n, const double* __restrict__ scal,
                                                            double* host, uint32_t* flag, uint32_t seq,
                                                            const int* extra) {
    for (int i = threadIdx.x; i < n; i += 256) host[i] = scal[i];
    if (threadIdx.x == 0) host[n] = extra ? (double)*extra : 0.0;
    // every thread's writes reach the system before the workgroup's flag
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish_scalars(int n, const double* scal, double* host, uint32_t* flag, uint32_t seq,
                            const int* extra, hipStream_t st) {
    hipLaunchKernelGGL(publish_scalars_kernel, dim3(1), dim3(256), 0, st, n, scal, host, flag, seq, extra);
}

void launch_copy(int n, double* y, const double* x, hipStream_t st) {
    hipLaunchKernelGGL(copy_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, y, x);
}

void launch_fill_u8(int64_t n, uint8_t* p, uint8_t v, hipStream_t st) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(fill_u8_kernel, dim3(g), dim3(kBlock), 0, st, n, p, v);
}

void launch_fill_u32(int64_t n, unsigned* p, unsigned v, hipStream_t st) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(fill_u32_kernel, dim3(g), dim3(kBlock), 0, st, n, p, v);
}

void launch_narrow(int64_t n, float* y, const double* x, hipStream_t st) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(narrow_kernel, dim3(g), dim3(kBlock), 0, st, n, y, x);
}

void launch_widen_dot(int n, double* y, const float* x, const double* u, DotTarget dot, hipStream_t st) {
    hipLaunchKernelGGL(widen_dot_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, y, x, u, dot);
    finish_dot(dot, vec_grid(n), st);
}

void launch_add_widened(int n, double* x, const float* e, hipStream_t st) {
    hipLaunchKernelGGL(add_widened_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, x, e);
}

void launch_scaled_copy(int n, float* y, const float* dinv, const float* x, float omega, hipStream_t st) {
    hipLaunchKernelGGL(scaled_copy_t_kernel<float>, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, y, dinv, x, omega);
}

void launch_copy(int n, float* y, const float* x, hipStream_t st) {
    hipLaunchKernelGGL(copy_t_kernel<float>, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, y, x);
}

void launch_fill_f32(int64_t n, float* p, float v, hipStream_t st) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(fill_t_kernel<float>, dim3(g), dim3(kBlock), 0, st, n, p, v);
}

void launch_dense_matvec(int n, const double* ainv, const float* b, float* y, hipStream_t st) {
    hipLaunchKernelGGL(dense_matvec_mixed_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n,
                       ainv, b, y);
}

void launch_fill_f64(int64_t n, double* p, double v, hipStream_t st) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(fill_f64_kernel, dim3(g), dim3(kBlock), 0, st, n, p, v);
}

void launch_dot(int n, const double* a, const double* b, DotTarget dot, hipStream_t st) {
    hipLaunchKernelGGL(dot_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, a, b, dot);
    finish_dot(dot, vec_grid(n), st);
}

int launch_sell_dual_resid(const CsrView& a, const double* g, const double* u, double* y, const double* g2,
                           const double* u2, double* y2, DotTarget dot, hipStream_t st) {
    if (!AMG_SELL || !a.sl_off) return 0;
    const int w = a.sl_maxw;
    if (w <= 8) return launch_sell_dual_u<8>(a, g, u, y, g2, u2, y2, dot, st);
    if (w <= 12) return launch_sell_dual_u<12>(a, g, u, y, g2, u2, y2, dot, st);
    if (w <= 16) return launch_sell_dual_u<16>(a, g, u, y, g2, u2, y2, dot, st);
    if (w <= 20) return launch_sell_dual_u<20>(a, g, u, y, g2, u2, y2, dot, st);
    if (w <= 24) return launch_sell_dual_u<24>(a, g, u, y, g2, u2, y2, dot, st);
    return launch_sell_dual_u<32>(a, g, u, y, g2, u2, y2, dot, st);
}

void launch_zero_guess_start(int n, const double* b, double* x, double* r, DotTarget dot, hipStream_t st) {
    hipLaunchKernelGGL(zero_guess_start_kernel, dim3(vec_grid(n)), dim3(kBlock), 0, st, n, b, x, r, dot);
    finish_dot(dot, vec_grid(n), st);
}

int vector_launch_blocks(int n) { return vec_grid(n); }

void launch_dense_matvec(int n, const double* ainv, const double* b, double* y, hipStream_t st) {
    hipLaunchKernelGGL(dense_matvec_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n,
                       ainv, b, y);
}

void launch_inverse_diagonal(const CsrView& a, double* dinv, float* dinv32, hipStream_t st) {
    hipLaunchKernelGGL(inverse_diagonal_kernel, dim3((a.rows + kBlock / 8 - 1) / (kBlock / 8)), dim3(kBlock),
                       0, st, a, dinv, dinv32);
}

void launch_mark_minimal_pattern(int nc, const int32_t* c_points, const int32_t* afine_rp,
                                 const int32_t* afine_ci, const int32_t* p_rp,
                                 const int32_t* p_ci, const int32_t* ac_rp, const int32_t* ac_ci,
                                 uint8_t* in_m, int* missing, hipStream_t st) {
    if (nc <= 0) return;
    const int grid = std::min((nc + kBlock / 64 - 1) / (kBlock / 64), kMarkGridCap);
    hipLaunchKernelGGL(mark_minimal_pattern_kernel, dim3(grid), dim3(kBlock), 0, st, nc, c_points, afine_rp,
                       afine_ci, p_rp, p_ci, ac_rp, ac_ci, in_m, missing);
}

#define AMG_WIDTH_SWITCH(width, KERNEL, ...)                                                   \
    do {                                                                                       \
        switch (width) {                                                                       \
            case 4: hipLaunchKernelGGL(KERNEL<4>, dim3((a.rows + kBlock / 4 - 1) / (kBlock / 4)), dim3(kBlock), 0, st, __VA_ARGS__); break;    \
            case 8: hipLaunchKernelGGL(KERNEL<8>, dim3((a.rows + kBlock / 8 - 1) / (kBlock / 8)), dim3(kBlock), 0, st, __VA_ARGS__); break;    \
            case 16: hipLaunchKernelGGL(KERNEL<16>, dim3((a.rows + kBlock / 16 - 1) / (kBlock / 16)), dim3(kBlock), 0, st, __VA_ARGS__); break; \
            case 32: hipLaunchKernelGGL(KERNEL<32>, dim3((a.rows + kBlock / 32 - 1) / (kBlock / 32)), dim3(kBlock), 0, st, __VA_ARGS__); break; \
            default: hipLaunchKernelGGL(KERNEL<64>, dim3((a.rows + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, st, __VA_ARGS__); break; \
        }                                                                                      \
    } while (0)

void launch_row_max(int width, const CsrView& a, double* m, hipStream_t st) {
    if (a.rows <= 0) return;
    AMG_WIDTH_SWITCH(width, row_max_kernel, a, m);
}

void launch_keep_count(int width, const CsrView& a, const uint8_t* in_m, const double* m,
                       double gamma, uint8_t* keep, int32_t* cnt, int32_t* bsum, hipStream_t st) {
    if (a.rows <= 0) return;
    AMG_WIDTH_SWITCH(width, keep_count_kernel, a, in_m, m, gamma, keep, cnt, bsum);
}

int keep_count_blocks(int width, int rows) {
    const int w = width == 4 || width == 8 || width == 16 || width == 32 ? width : 64;
    const int r = kBlock / w;
    return (rows + r - 1) / r;
}

void launch_keep_count_merged(SparsifyLevels& L, hipStream_t st) {
    int b = 0;
    for (int k = 0; k < L.count; ++k) {
        L.lv[k].block0 = b;
        b += keep_count_blocks(64, L.lv[k].a.rows);
    }
    if (L.count > 0 && b > 0) hipLaunchKernelGGL(keep_count_merged_kernel, dim3(b), dim3(kBlock), 0, st, L);
}

void launch_compact_lump_merged(SparsifyLevels& L, hipStream_t st) {
    int b = 0;
    for (int k = 0; k < L.count; ++k) {
        L.lv[k].block0 = b;
        b += keep_count_blocks(64, L.lv[k].a.rows);
    }
    if (L.count > 0 && b > 0) hipLaunchKernelGGL(compact_lump_merged_kernel, dim3(b), dim3(kBlock), 0, st, L);
}

void launch_scan_jobs(const ScanJobs& jobs, hipStream_t st) {
    if (jobs.count <= 0) return;
    hipLaunchKernelGGL(scan_jobs_kernel, dim3(jobs.count), dim3(1024), 0, st, jobs);
}

void launch_compact_lump(int width, const CsrView& a, const uint8_t* keep, const int32_t* cnt,
                         const int32_t* boff, int32_t* new_rp, int32_t* new_ci, double* new_v, double* dinv,
                         float* new_v32, float* dinv32, hipStream_t st) {
    if (a.rows <= 0) return;
    AMG_WIDTH_SWITCH(width, compact_lump_kernel, a, keep, cnt, boff, new_rp, new_ci, new_v, dinv, new_v32,
                     dinv32);
}

int dense_invert_max() { return kDenseInvMax; }

// Dynamic LDS the staged tail may take: the device's limit per workgroup less
// the kernel's static LDS (its arguments and copy list); 0 if the limit
// cannot be read or raised.
template <class T>
size_t tail_lds_limit() {
    static const size_t limit = [] {
        int dev = 0, per_block = 0;
        hipFuncAttributes fa{};
        const void* k = reinterpret_cast<const void*>(coarse_tail_lds_kernel<T>);
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            hipFuncGetAttributes(&fa, k) != hipSuccess || (size_t)per_block <= fa.sharedSizeBytes)
            return (size_t)0;
        const size_t dyn = (size_t)per_block - fa.sharedSizeBytes;
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess) return (size_t)0;
        return dyn;
    }();
    return limit;
}

template <class T>
void launch_coarse_tail_t(const TailArgs<T>& t, hipStream_t st) {
    if (t.count <= kTailLdsLevels) {
        TailLdsArgs<T> a;
        const size_t bytes = tail_lds_plan(t, a);
        if (bytes <= tail_lds_limit<T>()) {
            hipLaunchKernelGGL(coarse_tail_lds_kernel<T>, dim3(1), dim3(kTailBlock), bytes, st, a);
            return;
        }
    }
    hipLaunchKernelGGL(coarse_tail_kernel<T>, dim3(1), dim3(kTailBlock), 0, st, t);
}

void launch_coarse_tail(const TailArgs<double>& t, hipStream_t st) { launch_coarse_tail_t<double>(t, st); }

void launch_coarse_tail(const TailArgs<float>& t, hipStream_t st) { launch_coarse_tail_t<float>(t, st); }

void launch_dense_invert(const CsrView& a, double* inv, int* singular, hipStream_t st) {
    hipLaunchKernelGGL(dense_invert_kernel, dim3(1), dim3(kDenseInvThreads), 0, st, a, inv, singular);
}

// one wavefront per row block: its smallest and largest column by shuffles,
// then the offsets
__global__ __launch_bounds__(kBlock) void compress_index_kernel(int rows, int rb, const int32_t* __restrict__ rp,
                                                                const int32_t* __restrict__ ci,
                                                                uint16_t* __restrict__ ci16,
                                                                int32_t* __restrict__ cbase, int* wide) {
    const int nblk = (rows + rb - 1) / rb;
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (kBlock / 64);
    for (int b = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); b < nblk; b += nwaves) {
        const int r0 = b * rb, r1 = min(r0 + rb, rows);
        const int p0 = rp[r0], p1 = rp[r1];
        int mn = INT_MAX, mx = INT_MIN;
        for (int p = p0 + lane; p < p1; p += 64) {
            mn = min(mn, ci[p]);
            mx = max(mx, ci[p]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, __shfl_xor(mn, o, 64));
            mx = max(mx, __shfl_xor(mx, o, 64));
        }
        const bool fits = p1 == p0 || (int64_t)mx - (int64_t)mn <= 65535;
        if (lane == 0) {
            cbase[b] = p1 > p0 ? mn : 0;
            if (!fits) atomicAdd(wide, 1);
        }
        for (int p = p0 + lane; p < p1; p += 64) ci16[p] = fits ? (uint16_t)(ci[p] - mn) : (uint16_t)0;
    }
}

int64_t scan_scratch_ints(int n) { return (int64_t)(n + kScanTile - 1) / kScanTile + 1; }

void launch_compress_index(int rows, int rb, const int32_t* rp, const int32_t* ci, uint16_t* ci16,
                           int32_t* cbase, int* wide, hipStream_t st) {
    const int nblk = (rows + rb - 1) / rb;
    const int grid = std::max(1, std::min((nblk + 3) / 4, 8192));
    hipLaunchKernelGGL(compress_index_kernel, dim3(grid), dim3(kBlock), 0, st, rows, rb, rp, ci, ci16, cbase,
                       wide);
}

int stream_block_rows(const CsrView& a) { return use_stream_kernel(a) ? stream_rows_per_block(a.mean_row) : 0; }

// SELL-64 copies only for rows of at most this mean length: on the 128^3
// Galerkin level 2 (rows of 34 entries) the SELL kernel's zero-guess residual
// took 31.4 us against 27.8 us for the subgroup kernel.
#ifndef AMG_SELL_MAX_ROW
#define AMG_SELL_MAX_ROW 24.0
#endif
bool sell_candidate(const CsrView& a) {
    return AMG_SELL && a.mean_row <= AMG_SELL_MAX_ROW && use_stream_kernel(a);
}

int sell_slices(int rows) { return (rows + kSellRows - 1) / kSellRows; }

void launch_sell_widths(int rows, const int32_t* rp, int32_t* width64, hipStream_t st) {
    const int blocks = std::max(1, (sell_slices(rows) + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock);
    hipLaunchKernelGGL(sell_width_kernel, dim3(blocks), dim3(kBlock), 0, st, rows, rp, width64);
}

void launch_sell_dictionary(int rows, const int32_t* off, const int32_t* col, uint8_t* idx8, int32_t* tab,
                            int* wide, hipStream_t st) {
    const int blocks = std::max(1, (sell_slices(rows) + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock);
    hipLaunchKernelGGL(sell_dictionary_kernel, dim3(blocks), dim3(kBlock), 0, st, rows, off, col, idx8, tab, wide);
}

void launch_sell_compress(int rows, const int32_t* off, const int32_t* col, uint16_t* col16, int32_t* base,
                          int* wide, hipStream_t st) {
    const int blocks = std::max(1, (sell_slices(rows) + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock);
    hipLaunchKernelGGL(sell_compress_kernel, dim3(blocks), dim3(kBlock), 0, st, rows, off, col, col16, base, wide);
}

void launch_sell_fill(int rows, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* off,
                      int32_t* col, double* val, hipStream_t st) {
    const int blocks = std::max(1, (sell_slices(rows) + kSellSlicesPerBlock - 1) / kSellSlicesPerBlock);
    hipLaunchKernelGGL(sell_fill_kernel, dim3(blocks), dim3(kBlock), 0, st, rows, rp, ci, v, off, col, val);
}

void launch_exclusive_scan(int n, const int32_t* cnt, int32_t* out, int32_t* scratch,
                           hipStream_t st) {
    const int nb = std::max(1, (n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(scan_pass1_kernel, dim3(nb), dim3(kBlock), 0, st, n, cnt, scratch);
    hipLaunchKernelGGL(scan_pass2_kernel, dim3(1), dim3(1024), 0, st, nb, scratch);
    hipLaunchKernelGGL(scan_pass3_kernel, dim3(nb), dim3(kBlock), 0, st, n, cnt, scratch, out);
}

}  // namespace amg355
