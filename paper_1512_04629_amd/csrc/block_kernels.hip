// Multi-right-hand-side kernels of the V-cycle (gfx950, wave64).
//
// K columns row-interleaved: the K values that a row gathers from row j of a
// block are one contiguous run of K * sizeof(T) bytes.  A row is served by
// K * sizeof(T) / 16 lanes, each holding 16 bytes of columns (4 FP32 or 2
// FP64), so that every gather is a 16-byte load and the matrix entries of the
// row (column index and value, same address in those lanes) are read once for
// all K columns.  Bandwidth-bound like the single-vector kernels: per nonzero
// 8 (FP32) or 12 (FP64) bytes of matrix against K values of gathered vector,
// most of which come from cache because neighbouring rows share columns.
#include "block_kernels.hpp"

#include <algorithm>

namespace amg355 {
namespace {

constexpr int kBlk = 256;
constexpr int kXcd = 8;          // accelerator complex dies, each with its own L2
constexpr int kGridCap = 4096;   // row tiles beyond this many workgroups are looped over

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

template <class T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = v4f;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = v2d;
    static constexpr int n = 2;
};

// workgroups go to the dies round-robin; give each die a contiguous range of
// row tiles so that the rows it gathers for stay in its L2 (grid multiple of 8)
__device__ __forceinline__ int logical_block() {
    const int per = gridDim.x / kXcd;
    return (blockIdx.x % kXcd) * per + blockIdx.x / kXcd;
}

int round8(int b) { return (b + kXcd - 1) / kXcd * kXcd; }

// The row tiles one workgroup handles.  AMG_BLK_RANGES = 1: each die walks
// one contiguous range of tiles for the whole launch (its workgroups move
// through the range together), so the rows a tile gathers from one grid plane
// away were gathered by the same die shortly before and can still be in its
// L2; 0 (default): the dies interleave, each taking a contiguous slice of
// every step.  Measured on the 16-column 192^3 hierarchy: within 2% either
// way; non-temporal matrix loads (AMG_BLK_NT) are 30% slower.
#ifndef AMG_BLK_RANGES
#define AMG_BLK_RANGES 0
#endif
// AMG_BLK_NT = 1: column indices and values are loaded non-temporally, so
// that the streamed matrix does not evict the gathered block from L2.
#ifndef AMG_BLK_NT
#define AMG_BLK_NT 0
#endif
struct TileWalk {
    int t, end, stride;
};

__device__ __forceinline__ TileWalk tile_walk(int ntiles) {
#if AMG_BLK_RANGES
    const int x = blockIdx.x % kXcd, per = gridDim.x / kXcd;
    const int lo = (int)((long long)ntiles * x / kXcd), hi = (int)((long long)ntiles * (x + 1) / kXcd);
    return TileWalk{lo + (int)blockIdx.x / kXcd, hi, per};
#else
    return TileWalk{logical_block(), ntiles, (int)gridDim.x};
#endif
}

template <class T>
__device__ __forceinline__ T mat_ld(const T* p) {
#if AMG_BLK_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <class VT, class T>
__device__ __forceinline__ VT ld16(const T* p) {
    return *reinterpret_cast<const VT*>(p);
}

template <class VT, class T>
__device__ __forceinline__ void st16(T* p, const VT& v) {
    *reinterpret_cast<VT*>(p) = v;
}

// acc[0..V) += (double) v
__device__ __forceinline__ void add_to_fp64(double* acc, const v4f& v) {
    v2d a = ld16<v2d>(acc), b = ld16<v2d>(acc + 2);
    a.x += (double)v.x;
    a.y += (double)v.y;
    b.x += (double)v.z;
    b.y += (double)v.w;
    st16(acc, a);
    st16(acc + 2, b);
}

__device__ __forceinline__ void add_to_fp64(double* acc, const v2d& v) {
    v2d a = ld16<v2d>(acc);
    a += v;
    st16(acc, a);
}

// s = sum_p a_ip G[j_p, c0 .. c0+V) over the row [beg, end).  The row's
// LPR lanes (one per 16 bytes of columns) each load one entry of the row,
// and the entries are handed round the group with lane shuffles: one column
// index and one value load per lane for up to LPR entries, where loading
// each entry in every lane of the group would cost an index and a value
// load per entry (the kernels are bound by the count of vector memory
// instructions, the gathers included, more than by their bytes).  Entries
// at even and odd positions of the row go to two accumulators, added at the
// end, with two gathers in flight (the chunks of LPR entries start at even
// positions; a row of one lane takes its entries two at a time).  With
// DIAG, *gd receives G[i, c0 .. c0+V) from the gather of the row's diagonal
// entry (loaded if the row has none), so a sweep does not load its own x_i
// again.
template <class T, int K, bool DIAG>
struct RowAcc {
    using VT = typename Vec16<T>::type;
    VT s0{}, s1{}, dg{};
    bool found = false;
    // entry (j, v) at an even (odd = false) or odd position of the row
    __device__ __forceinline__ void add(bool odd, int j, T v, const VT& gj, int i) {
        if (odd) s1 += v * gj;
        else s0 += v * gj;
        if constexpr (DIAG) {
            if (j == i) dg = gj;
            found = found || j == i;
        }
    }
};

template <class T, int K, bool DIAG = false>
__device__ __forceinline__ typename Vec16<T>::type row_gather_sum(const CsrT<T>& a, const T* __restrict__ g,
                                                                  int beg, int end, int c0, int i = 0,
                                                                  typename Vec16<T>::type* gd = nullptr) {
    using VT = typename Vec16<T>::type;
    constexpr int LPR = K / Vec16<T>::n;
    RowAcc<T, K, DIAG> acc;
    if constexpr (LPR == 1) {
        // a lane per row (4 FP32 columns): its own loads, two entries a step
        int p = beg;
        for (; p + 1 < end; p += 2) {
            const int j0 = mat_ld(a.ci + p), j1 = mat_ld(a.ci + p + 1);
            const T v0 = mat_ld(a.v + p), v1 = mat_ld(a.v + p + 1);
            const VT g0 = ld16<VT>(g + j0 * K + c0);
            const VT g1 = ld16<VT>(g + j1 * K + c0);
            acc.add(false, j0, v0, g0, i);
            acc.add(true, j1, v1, g1, i);
        }
        if (p < end) {
            const int j0 = mat_ld(a.ci + p);
            acc.add(false, j0, mat_ld(a.v + p), ld16<VT>(g + j0 * K + c0), i);
        }
    } else {
        const int q = threadIdx.x & (LPR - 1);
        for (int p = beg; p < end; p += LPR) {
            const int qq = min(p + q, end - 1);
            const int myj = mat_ld(a.ci + qq);
            const T myv = mat_ld(a.v + qq);
            const int cnt = min(LPR, end - p);
            int k = 0;
            for (; k + 1 < cnt; k += 2) {
                const int j0 = __shfl(myj, k, LPR), j1 = __shfl(myj, k + 1, LPR);
                const T v0 = __shfl(myv, k, LPR), v1 = __shfl(myv, k + 1, LPR);
                const VT g0 = ld16<VT>(g + j0 * K + c0);
                const VT g1 = ld16<VT>(g + j1 * K + c0);
                acc.add(false, j0, v0, g0, i);
                acc.add(true, j1, v1, g1, i);
            }
            if (k < cnt) {
                const int j0 = __shfl(myj, k, LPR);
                acc.add(false, j0, __shfl(myv, k, LPR), ld16<VT>(g + j0 * K + c0), i);
            }
        }
    }
    if constexpr (DIAG) *gd = acc.found ? acc.dg : ld16<VT>(g + i * K + c0);
    return acc.s0 + acc.s1;
}

template <class T, int K, int OP>
__global__ __launch_bounds__(kBlk) void block_row_kernel(CsrT<T> a, const T* __restrict__ g, const T* u,
                                                         const T* __restrict__ dinv, T omega, T* y,
                                                         T* __restrict__ y2, double* acc, int ntiles,
                                                         const double* __restrict__ live) {
    using VT = typename Vec16<T>::type;
    constexpr int V = Vec16<T>::n;
    constexpr int LPR = K / V;          // lanes per row
    constexpr int RPT = kBlk / LPR;     // rows per tile
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * V;
    // columns past the live prefix are left as they are; their lanes still
    // load and hand round their rows' entries (gathering the first columns)
    const bool dead = live && c0 >= (int)*live;
    for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
        const int i = t * RPT + sub;
        if (i >= a.rows) break;
        constexpr bool kSweep = OP == kBJacobi || OP == kBJacobiAccum;
        VT gi;
        const VT s = row_gather_sum<T, K, kSweep>(a, g, a.rp[i], a.rp[i + 1], dead ? 0 : c0, i, &gi);
        if (dead) continue;
        const int o = i * K + c0;
        if constexpr (OP == kBSpmv) {
            st16(y + o, s);
        } else if constexpr (OP == kBSpmvScale) {
            st16(y + o, s);
            st16(y2 + o, omega * (dinv[i] * s));
        } else if constexpr (OP == kBSpmvAdd) {
            st16(y + o, ld16<VT>(u + o) + s);
        } else if constexpr (OP == kBResid) {
            st16(y + o, ld16<VT>(u + o) - s);
        } else {
            const VT xn = gi + omega * dinv[i] * (ld16<VT>(u + o) - s);
            if constexpr (OP == kBJacobi) st16(y + o, xn);
            else add_to_fp64(acc + o, xn);
        }
    }
}

// Per-column sums over a workgroup.  Each thread holds V consecutive columns
// c0..c0+V-1 of its rows; threads holding the same columns are LPR = K / V
// lanes apart.  Writes partials[lb * K + c] (fixed reduction order).
template <int K, int V>
__device__ __forceinline__ void store_column_partials(double (&v)[V], double* __restrict__ partials, int lb) {
    constexpr int LPR = K / V;
    __shared__ double lds[kBlk / 64][K];
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] += __shfl_xor(v[e], off, 64);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane < LPR)
#pragma unroll
        for (int e = 0; e < V; ++e) lds[w][lane * V + e] = v[e];
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double tot = lds[0][threadIdx.x];
#pragma unroll
        for (int k = 1; k < kBlk / 64; ++k) tot += lds[k][threadIdx.x];
        partials[lb * K + threadIdx.x] = tot;
    }
}

// r = b - A x in FP64 for K columns; rt = (T) r, zt = omega dinvt rt, and r
// itself when r64 is not null; per workgroup partial sums of r_c^2 per
// column into partials[lb * K + c]
template <class T, int K>
__global__ __launch_bounds__(kBlk) void block_outer_kernel(CsrView a, const double* __restrict__ x,
                                                           const double* __restrict__ b,
                                                           const T* __restrict__ dinvt, T omega,
                                                           T* __restrict__ rt, T* __restrict__ zt,
                                                           double* __restrict__ r64,
                                                           double* __restrict__ partials, int ntiles,
                                                           const double* __restrict__ live) {
    constexpr int LPR = K / 2;
    constexpr int RPT = kBlk / LPR;
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * 2;
    const bool dead = live && c0 >= (int)*live;   // see block_row_kernel
    double n0 = 0.0, n1 = 0.0;
    for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
        const int i = t * RPT + sub;
        if (i >= a.rows) break;
        const v2d s = row_gather_sum<double, K>(a, x, a.rp[i], a.rp[i + 1], dead ? 0 : c0);
        if (dead) continue;
        const int o = i * K + c0;
        const v2d r = ld16<v2d>(b + o) - s;
        n0 += r.x * r.x;
        n1 += r.y * r.y;
        if (r64) st16(r64 + o, r);
        const T d = dinvt[i];
        const T r0 = (T)r.x, r1 = (T)r.y;
        rt[o] = r0;
        rt[o + 1] = r1;
        zt[o] = omega * (d * r0);
        zt[o + 1] = omega * (d * r1);
    }
    double nn[2] = {n0, n1};
    store_column_partials<K, 2>(nn, partials, lb);
}

// out[c] = sum over workgroups of partials[b * K + c], in a fixed order: one
// workgroup of kFinishThreads; thread t takes column t % K and the partials
// b = t / K + S m (S = kFinishThreads / K), into four accumulators (m mod 4)
// so that four loads are in flight; the four are added, then the S threads
// of a column in order (the ones in a wave with shuffles, then the waves).
constexpr int kFinishThreads = 1024;

template <int K>
__global__ __launch_bounds__(kFinishThreads) void block_norm_finish_kernel(int nparts,
                                                                           const double* __restrict__ partials,
                                                                           double* __restrict__ out) {
    constexpr int S = kFinishThreads / K;
    constexpr int W = kFinishThreads / 64;
    __shared__ double wsum[W][K];
    const int c = threadIdx.x % K;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = threadIdx.x / K;
    for (; b + 3 * S < nparts; b += 4 * S) {
        a0 += partials[b * K + c];
        a1 += partials[(b + S) * K + c];
        a2 += partials[(b + 2 * S) * K + c];
        a3 += partials[(b + 3 * S) * K + c];
    }
    if (b < nparts) a0 += partials[b * K + c];
    if (b + S < nparts) a1 += partials[(b + S) * K + c];
    if (b + 2 * S < nparts) a2 += partials[(b + 2 * S) * K + c];
    double v = (a0 + a1) + (a2 + a3);
    // lanes of one wave holding the same column are K apart
#pragma unroll
    for (int off = K; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane < K) wsum[w][lane] = v;
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double t = wsum[0][threadIdx.x];
#pragma unroll
        for (int k = 1; k < W; ++k) t += wsum[k][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// q = A p (FP64) with per-column partials of p_c . q_c
template <int K>
__global__ __launch_bounds__(kBlk) void block_spmv_dot_kernel(CsrView a, const double* __restrict__ p,
                                                              double* __restrict__ q,
                                                              double* __restrict__ partials, int ntiles,
                                                              const double* __restrict__ live) {
    constexpr int LPR = K / 2;
    constexpr int RPT = kBlk / LPR;
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * 2;
    const bool dead = live && c0 >= (int)*live;   // see block_row_kernel
    double d[2] = {0.0, 0.0};
    for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
        const int i = t * RPT + sub;
        if (i >= a.rows) break;
        v2d pi;
        const v2d s = row_gather_sum<double, K, true>(a, p, a.rp[i], a.rp[i + 1], dead ? 0 : c0, i, &pi);
        if (dead) continue;
        const int o = i * K + c0;
        st16(q + o, s);
        d[0] += pi.x * s.x;
        d[1] += pi.y * s.y;
    }
    store_column_partials<K, 2>(d, partials, lb);
}

// Per-column CG update of x and r (FP64): alpha_c = scal[i_num+c] /
// scal[i_den+c] for the columns with scal[i_act+c] != 0; a column whose
// denominator is not positive and finite is left unchanged and sets flags[c] = 1.
// Also rt = (T) r, zt = omega dinvt rt (the preconditioner's right-hand side
// and first sweep) and partials of |r_c|^2.
template <class T, int K>
__global__ __launch_bounds__(kBlk) void block_cg_xr_kernel(int n, double* __restrict__ x, double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ scal, int i_num, int i_den,
                                                           int i_act, double* flags, const T* __restrict__ dinvt,
                                                           T omega, T* __restrict__ rt, T* __restrict__ zt,
                                                           double* __restrict__ partials, int ntiles,
                                                           const double* __restrict__ live) {
    constexpr int LPR = K / 2;
    constexpr int RPT = kBlk / LPR;
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * 2;
    const int nt = (live && c0 >= (int)*live) ? 0 : ntiles;
    double alpha[2];
    bool upd[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const double num = scal[i_num + c0 + e], den = scal[i_den + c0 + e];
        const bool act = scal[i_act + c0 + e] != 0.0;
        const bool ok = den > 0.0 && isfinite(den);
        upd[e] = act && ok;
        alpha[e] = upd[e] ? num / den : 0.0;
        if (act && !ok && blockIdx.x == 0 && threadIdx.x < LPR) flags[c0 + e] = 1.0;
    }
    double nr[2] = {0.0, 0.0};
    for (TileWalk w = tile_walk(nt); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
        const int i = t * RPT + sub;
        if (i >= n) break;
        const int o = i * K + c0;
        v2d xi = ld16<v2d>(x + o), ri = ld16<v2d>(r + o);
        if (upd[0] || upd[1]) {
            // frozen columns keep x and r bit for bit (p may hold anything there)
            const v2d pi = ld16<v2d>(p + o), qi = ld16<v2d>(q + o);
            if (upd[0]) {
                xi.x = xi.x + alpha[0] * pi.x;
                ri.x = ri.x - alpha[0] * qi.x;
            }
            if (upd[1]) {
                xi.y = xi.y + alpha[1] * pi.y;
                ri.y = ri.y - alpha[1] * qi.y;
            }
            st16(x + o, xi);
            st16(r + o, ri);
        }
        nr[0] += ri.x * ri.x;
        nr[1] += ri.y * ri.y;
        const T d = dinvt[i];
        const T r0 = (T)ri.x, r1 = (T)ri.y;
        rt[o] = r0;
        rt[o + 1] = r1;
        zt[o] = omega * (d * r0);
        zt[o + 1] = omega * (d * r1);
    }
    store_column_partials<K, 2>(nr, partials, lb);
}

// p = z + beta_c p with beta_c = scal[i_num+c] / scal[i_den+c] for the
// columns with scal[i_act+c] != 0; p = z (a fresh start) in every column if
// restart_all, else in the columns with scal[i_restart+c] != 0
template <class Z, int K>
__global__ __launch_bounds__(kBlk) void block_cg_p_kernel(int n, double* __restrict__ p,
                                                          const Z* __restrict__ z,
                                                          const double* __restrict__ scal, int i_num, int i_den,
                                                          int i_act, int i_restart, int restart_all,
                                                          const double* __restrict__ live) {
    constexpr int LPR = K / 2;
    constexpr int RPT = kBlk / LPR;
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * 2;
    if (live && c0 >= (int)*live) return;
    double beta[2];
    bool upd[2], fresh[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        fresh[e] = restart_all || (i_restart >= 0 && scal[i_restart + c0 + e] != 0.0);
        upd[e] = fresh[e] || scal[i_act + c0 + e] != 0.0;
        beta[e] = fresh[e] ? 0.0 : scal[i_num + c0 + e] / scal[i_den + c0 + e];
    }
    if (!upd[0] && !upd[1]) return;
    const int ntiles = (n + RPT - 1) / RPT;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int i = t * RPT + sub;
        if (i >= n) break;
        const int o = i * K + c0;
        v2d zi;
        zi.x = (double)z[o];      // the preconditioned residual, widened exactly
        zi.y = (double)z[o + 1];
        v2d pi = ld16<v2d>(p + o);
        if (upd[0]) pi.x = fresh[0] ? zi.x : zi.x + beta[0] * pi.x;
        if (upd[1]) pi.y = fresh[1] ? zi.y : zi.y + beta[1] * pi.y;
        st16(p + o, pi);
    }
}

// A fresh start of the columns with scal[i_load+c] != 0: x_c = 0, r_c = b_c,
// rt_c = (T) b_c, zt_c = omega dinvt rt_c (the first sweep of the cycle), and
// per-workgroup partials of |b_c|^2 (same row partition and order as the
// outer residual, whose norm of b - A 0 they reproduce)
template <class T, int K>
__global__ __launch_bounds__(kBlk) void block_load_kernel(int n, const double* __restrict__ scal, int i_load,
                                                          const double* __restrict__ b, double* __restrict__ x,
                                                          double* __restrict__ r, const T* __restrict__ dinvt,
                                                          T omega, T* __restrict__ rt, T* __restrict__ zt,
                                                          double* __restrict__ partials, int ntiles) {
    constexpr int LPR = K / 2;
    constexpr int RPT = kBlk / LPR;
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * 2;
    const bool ld0 = scal[i_load + c0] != 0.0, ld1 = scal[i_load + c0 + 1] != 0.0;
    double nn[2] = {0.0, 0.0};
    if (ld0 || ld1) {
        for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
            const int i = t * RPT + sub;
            if (i >= n) break;
            const int o = i * K + c0;
            const v2d bi = ld16<v2d>(b + o);
            const T d = dinvt[i];
            if (ld0) {
                x[o] = 0.0;
                r[o] = bi.x;
                nn[0] += bi.x * bi.x;
                const T b0 = (T)bi.x;
                rt[o] = b0;
                zt[o] = omega * (d * b0);
            }
            if (ld1) {
                x[o + 1] = 0.0;
                r[o + 1] = bi.y;
                nn[1] += bi.y * bi.y;
                const T b1 = (T)bi.y;
                rt[o + 1] = b1;
                zt[o + 1] = omega * (d * b1);
            }
        }
    }
    store_column_partials<K, 2>(nn, partials, lb);
}

// column c of a K-wide block to / from a plain vector
__global__ __launch_bounds__(kBlk) void block_column_in_kernel(int n, int k, int c, const double* __restrict__ v,
                                                               double* __restrict__ blk) {
    for (int i = blockIdx.x * kBlk + threadIdx.x; i < n; i += gridDim.x * kBlk) blk[(size_t)i * k + c] = v[i];
}

__global__ __launch_bounds__(kBlk) void block_column_out_kernel(int n, int k, int c, const double* __restrict__ blk,
                                                                double* __restrict__ v) {
    for (int i = blockIdx.x * kBlk + threadIdx.x; i < n; i += gridDim.x * kBlk) v[i] = blk[(size_t)i * k + c];
}

// Last level-0 sweep of the preconditioner: z = G + omega dinv (U - A G) in
// the cycle's precision, with per-column partials of r64_c . (double) z_c
template <class T, int K>
__global__ __launch_bounds__(kBlk) void block_sweep_dot_kernel(CsrT<T> a, const T* __restrict__ g,
                                                               const T* __restrict__ u,
                                                               const T* __restrict__ dinv, T omega,
                                                               T* __restrict__ zt,
                                                               const double* __restrict__ r64,
                                                                     double* __restrict__ partials, int ntiles,
                                                                     const double* __restrict__ live) {
    using VT = typename Vec16<T>::type;
    constexpr int V = Vec16<T>::n;
    constexpr int LPR = K / V;
    constexpr int RPT = kBlk / LPR;
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * V;
    const bool dead = live && c0 >= (int)*live;   // see block_row_kernel
    double d[V];
#pragma unroll
    for (int e = 0; e < V; ++e) d[e] = 0.0;
    for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
        const int i = t * RPT + sub;
        if (i >= a.rows) break;
        VT gi;
        const VT s = row_gather_sum<T, K, true>(a, g, a.rp[i], a.rp[i + 1], dead ? 0 : c0, i, &gi);
        if (dead) continue;
        const int o = i * K + c0;
        const VT xn = gi + omega * dinv[i] * (ld16<VT>(u + o) - s);
        st16(zt + o, xn);
#pragma unroll
        for (int e = 0; e < V; e += 2) {
            const v2d re = ld16<v2d>(r64 + o + e);
            d[e] += re.x * (double)xn[e];
            d[e + 1] += re.y * (double)xn[e + 1];
        }
    }
    store_column_partials<K, V>(d, partials, lb);
}

// zt = x with partials of r64_c . (double) x_c (a cycle without post-smoothing)
template <class T, int K>
__global__ __launch_bounds__(kBlk) void block_copy_dot_kernel(int n, const T* __restrict__ x,
                                                              T* __restrict__ zt,
                                                              const double* __restrict__ r64,
                                                               double* __restrict__ partials, int ntiles,
                                                               const double* __restrict__ live) {
    constexpr int LPR = K / 2;
    constexpr int RPT = kBlk / LPR;
    const int lb = logical_block();
    const int sub = threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * 2;
    const int nt = (live && c0 >= (int)*live) ? 0 : ntiles;
    double d[2] = {0.0, 0.0};
    for (TileWalk w = tile_walk(nt); w.t < w.end; w.t += w.stride) {
        const int t = w.t;
        const int i = t * RPT + sub;
        if (i >= n) break;
        const int o = i * K + c0;
        const T x0 = x[o], x1 = x[o + 1];
        zt[o] = x0;
        zt[o + 1] = x1;
        const v2d re = ld16<v2d>(r64 + o);
        d[0] += re.x * (double)x0;
        d[1] += re.y * (double)x1;
    }
    store_column_partials<K, 2>(d, partials, lb);
}

// Device-side bookkeeping of the batch slots after an iteration (one
// workgroup): for every active column, count the iteration and stop the
// column when its residual meets the tolerance (||r|| <= rtol ||b||), its CG
// denominator broke down, the residual is not finite, or maxit is reached.
// A column loaded in this iteration (scal[i_load+c] != 0, i_load >= 0) first
// takes its |b|^2 from scal[i_new+c] into scal[i_nr0+c] and has its counter
// reset; with a zero right-hand side it stops at once with x = 0.  State per
// column: scal[i_stat+c] = 0 running, 1 converged, 2 maxit reached,
// 3 breakdown; scal[i_rel+c] = ||r|| / ||b|| after the iteration.
__global__ __launch_bounds__(64) void block_converge_kernel(int k, double* __restrict__ scal, int i_act,
                                                            int i_norm, int i_nr0, int i_flag, int i_iter,
                                                            int i_stat, int i_rel, int i_load, int i_new,
                                                            double rtol, int maxit) {
    const int c = threadIdx.x;
    if (c >= k || scal[i_act + c] == 0.0) return;
    if (i_load >= 0 && scal[i_load + c] != 0.0) {
        scal[i_nr0 + c] = scal[i_new + c];
        scal[i_iter + c] = 0.0;
        scal[i_stat + c] = 0.0;
    }
    const double n0 = sqrt(scal[i_nr0 + c]);
    if (n0 == 0.0) {
        scal[i_act + c] = 0.0;
        scal[i_stat + c] = 1.0;
        scal[i_rel + c] = 0.0;
        return;
    }
    const double it = scal[i_iter + c] + 1.0;
    scal[i_iter + c] = it;
    const double nr = sqrt(scal[i_norm + c]);
    double stat = 0.0;
    if (scal[i_flag + c] != 0.0 || !isfinite(nr) || !isfinite(n0)) stat = 3.0;
    else if (nr <= rtol * n0) stat = 1.0;
    else if (it >= (double)maxit) stat = 2.0;
    scal[i_rel + c] = nr / n0;
    if (stat != 0.0) {
        scal[i_stat + c] = stat;
        scal[i_act + c] = 0.0;
    }
}

template <class T>
__global__ __launch_bounds__(kBlk) void block_dense_kernel(int n, int k, const double* __restrict__ ainv,
                                                           const T* __restrict__ b, T* __restrict__ y,
                                                           const double* __restrict__ live) {
    const int idx = blockIdx.x * kBlk + threadIdx.x;
    if (idx >= n * k) return;
    const int i = idx / k, c = idx % k;
    if (live && c >= (int)*live) return;
    const double* row = ainv + (size_t)i * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += row[j] * (double)b[j * k + c];
    y[idx] = (T)s;
}

template <class T>
__global__ __launch_bounds__(kBlk) void block_accumulate_kernel(int64_t count, double* __restrict__ x,
                                                                const T* __restrict__ e) {
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlk)
        x[i] = x[i] + (double)e[i];
}

__global__ __launch_bounds__(kBlk) void block_pack_kernel(int n, int nrhs, int k, const double* __restrict__ src,
                                                          double* __restrict__ dst) {
    const int64_t total = (int64_t)n * k;
    for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total; q += (int64_t)gridDim.x * kBlk) {
        const int64_t i = q / k;
        const int c = (int)(q % k);
        dst[q] = c < nrhs ? src[i * nrhs + c] : 0.0;
    }
}

__global__ __launch_bounds__(kBlk) void block_unpack_kernel(int n, int nrhs, int k, const double* __restrict__ src,
                                                            double* __restrict__ dst) {
    const int64_t total = (int64_t)n * nrhs;
    for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total; q += (int64_t)gridDim.x * kBlk) {
        const int64_t i = q / nrhs;
        const int c = (int)(q % nrhs);
        dst[q] = src[i * k + c];
    }
}

int elem_grid(int64_t count) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (count + kBlk - 1) / kBlk));
}

template <class T, int K>
void block_op_k(BlockOp op, const CsrT<T>& a, const T* g, const T* u, const T* dinv, T omega, T* y, T* y2,
                double* acc, const double* live, hipStream_t st) {
    constexpr int LPR = K / Vec16<T>::n;
    constexpr int RPT = kBlk / LPR;
    const int ntiles = std::max(1, (a.rows + RPT - 1) / RPT);
    const int grid = round8(std::min(ntiles, kGridCap));
    switch (op) {
#define AMG_BLOCK_CASE(OPV)                                                                             \
    case OPV:                                                                                           \
        hipLaunchKernelGGL((block_row_kernel<T, K, OPV>), dim3(grid), dim3(kBlk), 0, st, a, g, u, dinv, \
                           omega, y, y2, acc, ntiles, live);                                            \
        break;
        AMG_BLOCK_CASE(kBSpmv)
        AMG_BLOCK_CASE(kBSpmvScale)
        AMG_BLOCK_CASE(kBSpmvAdd)
        AMG_BLOCK_CASE(kBResid)
        AMG_BLOCK_CASE(kBJacobi)
        AMG_BLOCK_CASE(kBJacobiAccum)
#undef AMG_BLOCK_CASE
        default: break;
    }
}

template <class T>
void block_op(BlockOp op, int k, const CsrT<T>& a, const T* g, const T* u, const T* dinv, T omega, T* y,
              T* y2, double* acc, const double* live, hipStream_t st) {
    if (k == 4) block_op_k<T, 4>(op, a, g, u, dinv, omega, y, y2, acc, live, st);
    else if (k == 8) block_op_k<T, 8>(op, a, g, u, dinv, omega, y, y2, acc, live, st);
    else block_op_k<T, 16>(op, a, g, u, dinv, omega, y, y2, acc, live, st);
}

// launch shape of the kernels that give a row K * 8 / 16 lanes (FP64 columns)
template <int K>
int fp64_tiles(int rows) {
    constexpr int RPT = kBlk / (K / 2);
    return std::max(1, (rows + RPT - 1) / RPT);
}

template <int K>
void finish(int grid, const ColumnDots& dot, hipStream_t st) {
    hipLaunchKernelGGL((block_norm_finish_kernel<K>), dim3(1), dim3(kFinishThreads), 0, st, grid, dot.partials,
                       dot.result);
}

// calls f.template operator()<K>() with the compile-time width
template <class F>
void with_width(int k, F&& f) {
    if (k == 4) f.template operator()<4>();
    else if (k == 8) f.template operator()<8>();
    else f.template operator()<16>();
}

template <class T>
void outer(int k, const CsrView& a, const double* x, const double* b, const T* dinvt, T omega, T* rt, T* zt,
           double* r64, ColumnDots dot, const double* live, hipStream_t st) {
    with_width(k, [&]<int K>() {
        const int ntiles = fp64_tiles<K>(a.rows);
        const int grid = round8(std::min(ntiles, kGridCap));
        hipLaunchKernelGGL((block_outer_kernel<T, K>), dim3(grid), dim3(kBlk), 0, st, a, x, b, dinvt, omega, rt,
                           zt, r64, dot.partials, ntiles, live);
        finish<K>(grid, dot, st);
    });
}

template <class T>
void cg_xr(int n, int k, double* x, double* r, const double* p, const double* q, const double* scal, int i_num,
           int i_den, int i_act, double* flags, const T* dinvt, T omega, T* rt, T* zt, ColumnDots norms,
           const double* live, hipStream_t st) {
    with_width(k, [&]<int K>() {
        const int ntiles = fp64_tiles<K>(n);
        const int grid = round8(std::min(ntiles, kGridCap));
        hipLaunchKernelGGL((block_cg_xr_kernel<T, K>), dim3(grid), dim3(kBlk), 0, st, n, x, r, p, q, scal, i_num,
                           i_den, i_act, flags, dinvt, omega, rt, zt, norms.partials, ntiles, live);
        finish<K>(grid, norms, st);
    });
}

template <class T>
void sweep_dot(int k, const CsrT<T>& a, const T* g, const T* u, const T* dinv, T omega, T* zt,
               const double* r64, ColumnDots dot, const double* live, hipStream_t st) {
    with_width(k, [&]<int K>() {
        constexpr int RPT = kBlk / (K / Vec16<T>::n);
        const int ntiles = std::max(1, (a.rows + RPT - 1) / RPT);
        const int grid = round8(std::min(ntiles, kGridCap));
        hipLaunchKernelGGL((block_sweep_dot_kernel<T, K>), dim3(grid), dim3(kBlk), 0, st, a, g, u, dinv,
                           omega, zt, r64, dot.partials, ntiles, live);
        finish<K>(grid, dot, st);
    });
}

template <class T>
void copy_dot(int n, int k, const T* x, T* zt, const double* r64, ColumnDots dot, const double* live,
              hipStream_t st) {
    with_width(k, [&]<int K>() {
        const int ntiles = fp64_tiles<K>(n);
        const int grid = round8(std::min(ntiles, kGridCap));
        hipLaunchKernelGGL((block_copy_dot_kernel<T, K>), dim3(grid), dim3(kBlk), 0, st, n, x, zt, r64,
                           dot.partials, ntiles, live);
        finish<K>(grid, dot, st);
    });
}

}  // namespace

int block_width(int nrhs) { return nrhs <= 4 ? 4 : (nrhs <= 8 ? 8 : 16); }

int block_partials_needed() { return kGridCap * 16; }

void launch_block_op(BlockOp op, int k, const CsrT<double>& a, const double* g, const double* u,
                     const double* dinv, double omega, double* y, double* y2, double* acc, hipStream_t st,
                     const double* live) {
    block_op<double>(op, k, a, g, u, dinv, omega, y, y2, acc, live, st);
}

void launch_block_op(BlockOp op, int k, const CsrT<float>& a, const float* g, const float* u,
                     const float* dinv, float omega, float* y, float* y2, double* acc, hipStream_t st,
                     const double* live) {
    block_op<float>(op, k, a, g, u, dinv, omega, y, y2, acc, live, st);
}

void launch_block_outer_residual(int k, const CsrView& a, const double* x, const double* b,
                                 const double* dinvt, double omega, double* rt, double* zt, double* r64,
                                 ColumnDots norms2, hipStream_t st, const double* live) {
    outer<double>(k, a, x, b, dinvt, omega, rt, zt, r64, norms2, live, st);
}

void launch_block_outer_residual(int k, const CsrView& a, const double* x, const double* b,
                                 const float* dinvt, float omega, float* rt, float* zt, double* r64,
                                 ColumnDots norms2, hipStream_t st, const double* live) {
    outer<float>(k, a, x, b, dinvt, omega, rt, zt, r64, norms2, live, st);
}

void launch_block_spmv_dot(int k, const CsrView& a, const double* p, double* q, ColumnDots dot, hipStream_t st,
                           const double* live) {
    with_width(k, [&]<int K>() {
        const int ntiles = fp64_tiles<K>(a.rows);
        const int grid = round8(std::min(ntiles, kGridCap));
        hipLaunchKernelGGL((block_spmv_dot_kernel<K>), dim3(grid), dim3(kBlk), 0, st, a, p, q, dot.partials,
                           ntiles, live);
        finish<K>(grid, dot, st);
    });
}

void launch_block_cg_update_xr(int n, int k, double* x, double* r, const double* p, const double* q,
                               const double* scal, int i_num, int i_den, int i_act, double* flags,
                               const double* dinvt, double omega, double* rt, double* zt, ColumnDots norms,
                               hipStream_t st, const double* live) {
    cg_xr<double>(n, k, x, r, p, q, scal, i_num, i_den, i_act, flags, dinvt, omega, rt, zt, norms, live, st);
}

void launch_block_cg_update_xr(int n, int k, double* x, double* r, const double* p, const double* q,
                               const double* scal, int i_num, int i_den, int i_act, double* flags,
                               const float* dinvt, float omega, float* rt, float* zt, ColumnDots norms,
                               hipStream_t st, const double* live) {
    cg_xr<float>(n, k, x, r, p, q, scal, i_num, i_den, i_act, flags, dinvt, omega, rt, zt, norms, live, st);
}

template <class Z>
void cg_p(int n, int k, double* p, const Z* z, const double* scal, int i_num, int i_den, int i_act, int i_restart,
          bool restart_all, hipStream_t st, const double* live) {
    with_width(k, [&]<int K>() {
        const int grid = std::min(fp64_tiles<K>(n), kGridCap);
        hipLaunchKernelGGL((block_cg_p_kernel<Z, K>), dim3(grid), dim3(kBlk), 0, st, n, p, z, scal, i_num, i_den,
                           i_act, i_restart, restart_all ? 1 : 0, live);
    });
}

void launch_block_cg_update_p(int n, int k, double* p, const double* z, const double* scal, int i_num,
                              int i_den, int i_act, int i_restart, bool restart_all, hipStream_t st,
                              const double* live) {
    cg_p<double>(n, k, p, z, scal, i_num, i_den, i_act, i_restart, restart_all, st, live);
}

void launch_block_cg_update_p(int n, int k, double* p, const float* z, const double* scal, int i_num,
                              int i_den, int i_act, int i_restart, bool restart_all, hipStream_t st,
                              const double* live) {
    cg_p<float>(n, k, p, z, scal, i_num, i_den, i_act, i_restart, restart_all, st, live);
}

template <class T>
void load_columns(int n, int k, const double* scal, int i_load, const double* b, double* x, double* r,
                  const T* dinvt, T omega, T* rt, T* zt, ColumnDots norms, hipStream_t st) {
    with_width(k, [&]<int K>() {
        const int ntiles = fp64_tiles<K>(n);
        const int grid = round8(std::min(ntiles, kGridCap));
        hipLaunchKernelGGL((block_load_kernel<T, K>), dim3(grid), dim3(kBlk), 0, st, n, scal, i_load, b, x, r,
                           dinvt, omega, rt, zt, norms.partials, ntiles);
        finish<K>(grid, norms, st);
    });
}

void launch_block_load_columns(int n, int k, const double* scal, int i_load, const double* b, double* x,
                               double* r, const double* dinvt, double omega, double* rt, double* zt,
                               ColumnDots norms, hipStream_t st) {
    load_columns<double>(n, k, scal, i_load, b, x, r, dinvt, omega, rt, zt, norms, st);
}

void launch_block_load_columns(int n, int k, const double* scal, int i_load, const double* b, double* x,
                               double* r, const float* dinvt, float omega, float* rt, float* zt,
                               ColumnDots norms, hipStream_t st) {
    load_columns<float>(n, k, scal, i_load, b, x, r, dinvt, omega, rt, zt, norms, st);
}

void launch_block_converge(int k, double* scal, int i_act, int i_norm, int i_nr0, int i_flag, int i_iter, int i_stat,
                           int i_rel, int i_load, int i_new, double rtol, int maxit, hipStream_t st) {
    hipLaunchKernelGGL(block_converge_kernel, dim3(1), dim3(64), 0, st, k, scal, i_act, i_norm, i_nr0, i_flag,
                       i_iter, i_stat, i_rel, i_load, i_new, rtol, maxit);
}

void launch_block_column_in(int n, int k, int c, const double* v, double* blk, hipStream_t st) {
    hipLaunchKernelGGL(block_column_in_kernel, dim3(elem_grid(n)), dim3(kBlk), 0, st, n, k, c, v, blk);
}

void launch_block_column_out(int n, int k, int c, const double* blk, double* v, hipStream_t st) {
    hipLaunchKernelGGL(block_column_out_kernel, dim3(elem_grid(n)), dim3(kBlk), 0, st, n, k, c, blk, v);
}

void launch_block_sweep_dot(int k, const CsrT<double>& a, const double* g, const double* u, const double* dinv,
                            double omega, double* zt, const double* r64, ColumnDots dot, hipStream_t st,
                            const double* live) {
    sweep_dot<double>(k, a, g, u, dinv, omega, zt, r64, dot, live, st);
}

void launch_block_sweep_dot(int k, const CsrT<float>& a, const float* g, const float* u, const float* dinv,
                            float omega, float* zt, const double* r64, ColumnDots dot, hipStream_t st,
                            const double* live) {
    sweep_dot<float>(k, a, g, u, dinv, omega, zt, r64, dot, live, st);
}

void launch_block_copy_dot(int n, int k, const double* x, double* zt, const double* r64, ColumnDots dot,
                           hipStream_t st, const double* live) {
    copy_dot<double>(n, k, x, zt, r64, dot, live, st);
}

void launch_block_copy_dot(int n, int k, const float* x, float* zt, const double* r64, ColumnDots dot,
                           hipStream_t st, const double* live) {
    copy_dot<float>(n, k, x, zt, r64, dot, live, st);
}

void launch_block_dense_matvec(int n, int k, const double* ainv, const double* b, double* y,
                               hipStream_t st, const double* live) {
    hipLaunchKernelGGL(block_dense_kernel<double>, dim3((n * k + kBlk - 1) / kBlk), dim3(kBlk), 0, st, n, k,
                       ainv, b, y, live);
}

void launch_block_dense_matvec(int n, int k, const double* ainv, const float* b, float* y, hipStream_t st,
                               const double* live) {
    hipLaunchKernelGGL(block_dense_kernel<float>, dim3((n * k + kBlk - 1) / kBlk), dim3(kBlk), 0, st, n, k,
                       ainv, b, y, live);
}

void launch_block_accumulate(int64_t count, double* x, const float* e, hipStream_t st) {
    hipLaunchKernelGGL(block_accumulate_kernel<float>, dim3(elem_grid(count)), dim3(kBlk), 0, st, count, x, e);
}

void launch_block_accumulate(int64_t count, double* x, const double* e, hipStream_t st) {
    hipLaunchKernelGGL(block_accumulate_kernel<double>, dim3(elem_grid(count)), dim3(kBlk), 0, st, count, x, e);
}

void launch_block_pack(int n, int nrhs, int k, const double* src, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(block_pack_kernel, dim3(elem_grid((int64_t)n * k)), dim3(kBlk), 0, st, n, nrhs, k, src,
                       dst);
}

void launch_block_unpack(int n, int nrhs, int k, const double* src, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(block_unpack_kernel, dim3(elem_grid((int64_t)n * nrhs)), dim3(kBlk), 0, st, n, nrhs, k,
                       src, dst);
}

}  // namespace amg355
