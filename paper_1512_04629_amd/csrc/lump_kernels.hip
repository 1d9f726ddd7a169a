// Strong-neighbour lumping kernels: every sum and share in the order the
// definition fixes (ascending columns; shares of a target in ascending order
// of their source entry), contraction off.  The threshold and the copy run
// one wave per row; the shares a workgroup per row with the row staged in
// LDS, the denominators the same or, on levels of short rows, a wave per row
// with its own stage (rows longer than the stage, and a launch forced to it,
// one wave per row without a stage).
#include "lump_kernels.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>

#pragma clang fp contract(off)

namespace amg355 {

namespace {

constexpr int kLB = 256;
constexpr int kWaves = kLB / 64;
constexpr int kWideCap = 256;   // row entries a workgroup stages in LDS (15 KB: eight workgroups a CU)
// below this mean row length, on levels with enough rows to fill the device
// with waves, the denominators run a wave per row with its own LDS stage
// (measured on 3D Poisson: faster at 174,772 and 27,542 rows of 34 and 57
// entries, slower at 129 rows of 65 and from 108 entries a row)
constexpr double kDenWaveMeanRow = 80.0;
constexpr int kDenWaveMinRows = 16384;

int wave_grid_of(int n) { return std::max(1, std::min((n + kWaves - 1) / kWaves, 65536)); }

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

// one wave per row i (kWaves per workgroup), lanes over the row's entries
#define WAVE_ROW_LOOP(i, n)                                                                         \
    for (int i = blockIdx.x * kWaves + (int)(threadIdx.x >> 6); i < (n); i += gridDim.x * kWaves)

// one wave per row: the kept entries of each 64-entry chunk go to the next
// free places in order (ballot, count of the lower lanes' kept entries)
__global__ void __launch_bounds__(kLB) compact_copy_kernel(int n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           const uint8_t* __restrict__ keep,
                                                           const int32_t* __restrict__ new_rp,
                                                           int32_t* __restrict__ new_ci, double* __restrict__ new_v) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1;
    WAVE_ROW_LOOP(i, n) {
        const int ie = rp[i + 1];
        int w = new_rp[i];
        for (int p0 = rp[i]; p0 < ie; p0 += 64) {
            const int p = p0 + lane;
            const bool kp = p < ie && keep[p];
            const uint64_t mask = __ballot(kp);
            if (kp) {
                const int at = w + __popcll(mask & below);
                new_ci[at] = ci[p];
                new_v[at] = v[p];
            }
            w += __popcll(mask);
        }
    }
}

// one wave per row: the largest -a_jm off the diagonal (a maximum, the same
// in any order)
__global__ void __launch_bounds__(kLB) lump_threshold_kernel(int n, const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ ci,
                                                             const double* __restrict__ v, double theta,
                                                             double* __restrict__ thr) {
    const int lane = threadIdx.x & 63;
    WAVE_ROW_LOOP(j, n) {
        double big = 0.0;
        for (int p = rp[j] + lane; p < rp[j + 1]; p += 64)
            if (ci[p] != j && -v[p] > big) big = -v[p];
        for (int o = 32; o > 0; o >>= 1) {
            const double other = __shfl_xor(big, o);
            if (other > big) big = other;
        }
        if (lane == 0) thr[j] = big > 0.0 ? theta * big : -1.0;
    }
}

// den of every dropped entry of row i, one wave: a lane per dropped entry;
// the strong neighbours m of j in ascending order are matched against the
// ascending columns of row i by a merge walk
__device__ inline void lump_den_row(int i, int lane, const int32_t* rp, const int32_t* ci, const double* v,
                                    const uint8_t* keep, const double* thr, double* den) {
    const int ib = rp[i], ie = rp[i + 1];
    for (int p = ib + lane; p < ie; p += 64) {
        const int j = ci[p];
        if (j == i || keep[p]) continue;
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

__global__ void __launch_bounds__(kLB) lump_den_kernel(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const uint8_t* __restrict__ keep,
                                                       const double* __restrict__ thr, double* __restrict__ den) {
    const int lane = threadIdx.x & 63;
    WAVE_ROW_LOOP(i, n) { lump_den_row(i, lane, rp, ci, v, keep, thr, den); }
}

// First position w in the ascending a[0..len) with a[w] >= col.
__device__ inline int lower_bound_lds(const int32_t* a, int len, int col) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Ordered sum of the lanes' x where has is set, in lane order, onto acc
// (the same value in every lane).
__device__ inline double ordered_add(double acc, bool has, double x) {
    for (uint64_t mask = __ballot(has); mask != 0; mask &= mask - 1) acc = acc + __shfl(x, __builtin_ctzll(mask));
    return acc;
}

// One workgroup per row i, its columns and keep flags staged in LDS; each
// wave takes a dropped entry (i,j) at a time, its lanes over the entries of
// row j (coalesced), and finds m among the staged columns by a binary search
// in LDS; the wave adds the terms in lane order, which is ascending m.  Rows
// longer than the stage take the one-wave path.
__global__ void __launch_bounds__(kLB) lump_den_wide_kernel(int n, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const double* __restrict__ v,
                                                            const uint8_t* __restrict__ keep,
                                                            const double* __restrict__ thr,
                                                            double* __restrict__ den) {
    __shared__ int32_t sc[kWideCap];
    __shared__ uint8_t sk[kWideCap];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int ib = rp[i], ie = rp[i + 1], len = ie - ib;
        if (len > kWideCap) {
            if (wave == 0) lump_den_row(i, lane, rp, ci, v, keep, thr, den);
            continue;
        }
        __syncthreads();   // the previous row's readers are done
        for (int t = threadIdx.x; t < len; t += kLB) {
            sc[t] = ci[ib + t];
            sk[t] = keep[ib + t];
        }
        __syncthreads();
        for (int u = wave; u < len; u += kWaves) {
            const int j = sc[u];
            if (j == i || sk[u]) continue;
            const int jb = rp[j], je = rp[j + 1];
            const double t = thr[j];
            double d = 0.0;
            for (int r0 = jb; r0 < je; r0 += 64) {
                const int r = r0 + lane;
                bool has = false;
                double a = 0.0;
                if (r < je && t > 0.0) {
                    const int m = ci[r];
                    a = v[r];
                    if (m != j && -a >= t) {
                        const int w = lower_bound_lds(sc, len, m);
                        has = w < len && sc[w] == m && sk[w];
                    }
                }
                d = ordered_add(d, has, fabs(a));
            }
            if (lane == 0) den[ib + u] = d;
        }
    }
}

// Short rows: the same per dropped entry, but one wave per row (each wave
// its own slice of LDS, so four rows of a workgroup are in flight at once);
// a row's stage is written and read by its own wave only.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(kLB) lump_den_wave_kernel(int n, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const double* __restrict__ v,
                                                            const uint8_t* __restrict__ keep,
                                                            const double* __restrict__ thr,
                                                            double* __restrict__ den) {
    __shared__ int32_t scw[kWaves][kWideCap];
    __shared__ uint8_t skw[kWaves][kWideCap];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int32_t* sc = scw[wave];
    uint8_t* sk = skw[wave];
    WAVE_ROW_LOOP(i, n) {
        const int ib = rp[i], ie = rp[i + 1], len = ie - ib;
        if (len > kWideCap) {
            lump_den_row(i, lane, rp, ci, v, keep, thr, den);
            continue;
        }
        wave_lds_sync();   // the previous row's reads are done
        for (int t = lane; t < len; t += 64) {
            sc[t] = ci[ib + t];
            sk[t] = keep[ib + t];
        }
        wave_lds_sync();
        for (int u = 0; u < len; ++u) {
            const int j = sc[u];
            if (j == i || sk[u]) continue;
            const int jb = rp[j], je = rp[j + 1];
            const double t = thr[j];
            double d = 0.0;
            for (int r0 = jb; r0 < je; r0 += 64) {
                const int r = r0 + lane;
                bool has = false;
                double a = 0.0;
                if (r < je && t > 0.0) {
                    const int m = ci[r];
                    a = v[r];
                    if (m != j && -a >= t) {
                        const int w = lower_bound_lds(sc, len, m);
                        has = w < len && sc[w] == m && sk[w];
                    }
                }
                d = ordered_add(d, has, fabs(a));
            }
            if (lane == 0) den[ib + u] = d;
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
__device__ inline void strong_lump_row(int k, int lane, const int32_t* rp, const int32_t* ci, const double* v,
                                       const uint8_t* keep, const double* thr, const double* den,
                                       const int32_t* hrp, const int32_t* hci, double* hv) {
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
    if (dk < 0) return;   // every operator stores its diagonal; never taken (uniform over the wave)
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
            acc = ordered_add(acc, has, c);
        }
    }
    if (lane == 0) hv[dk] = acc;
}

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
    WAVE_ROW_LOOP(k, n) { strong_lump_row(k, lane, rp, ci, v, keep, thr, den, hrp, hci, hv); }
}

// One workgroup per row k, row k of A (columns, values, keep flags,
// denominators, and the thresholds of its columns) staged in LDS.
// * (k,m), m > k, one wave each, its lanes over row m (coalesced): a lane
//   finds its column j in the staged row k by a binary search in LDS and
//   forms the share of dropped (k,j) (with a_jm read as a_mj); the wave adds
//   them in lane order, then, in a second pass, the shares of dropped (m,j)
//   (a_jk read as a_kj).  Every share needs j in row k, so its threshold is
//   a staged one.  Same terms, same order as the one-wave path.
// * the diagonal: the kept rows s of row k are laid end to end (offsets by a
//   scan), the workgroup computes kDiagPer x 256 consecutive entries' shares
//   at a time into LDS (a_kj by a binary search of the staged row k) and the
//   first wave adds them in order.
// Rows longer than the stage take the one-wave path.
constexpr int kDiagPer = 2;

// LB threads a workgroup: LB, or 1024 on levels too small to fill the
// device otherwise; eight waves a SIMD (at most 64 registers, no spills)
template <int LB>
__global__ void __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(8, 8))) strong_lump_wide_kernel(int n, const int32_t* __restrict__ rp,
                                                               const int32_t* __restrict__ ci,
                                                               const double* __restrict__ v,
                                                               const uint8_t* __restrict__ keep,
                                                               const double* __restrict__ thr,
                                                               const double* __restrict__ den,
                                                               const int32_t* __restrict__ hrp,
                                                               const int32_t* __restrict__ hci,
                                                               double* __restrict__ hv) {
    __shared__ int32_t kc[kWideCap];
    __shared__ double kv[kWideCap];
    __shared__ double kd[kWideCap];
    __shared__ double kt[kWideCap];         // thr of the columns of row k
    __shared__ uint8_t kk[kWideCap];
    __shared__ int32_t ks[kWideCap];        // the kept columns s of row k
    __shared__ int32_t sb[kWideCap];        // rp[s]
    __shared__ int32_t off[kWideCap + 1];   // their rows' offsets, end to end
    __shared__ double slot_c[kDiagPer * LB];
    __shared__ uint8_t slot_h[kDiagPer * LB];
    __shared__ int wsum[(LB / 64)];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const int kb = rp[k], ke = rp[k + 1], len = ke - kb;
        if (len > kWideCap) {
            if (wave == 0) strong_lump_row(k, lane, rp, ci, v, keep, thr, den, hrp, hci, hv);
            continue;
        }
        const int hb = hrp[k], he = hrp[k + 1], nk = he - hb;   // nk <= len
        __syncthreads();   // the previous row's readers are done
        for (int t = threadIdx.x; t < len; t += LB) {
            const int p = kb + t;
            const int j = ci[p];
            kc[t] = j;
            kv[t] = v[p];
            kk[t] = keep[p];
            kd[t] = keep[p] ? 0.0 : den[p];   // den is written for dropped entries only
            kt[t] = thr[j];
        }
        // kept columns and their row lengths, scanned end to end
        int carry = 0;
        for (int base = 0; base < nk; base += LB) {
            const int idx = base + (int)threadIdx.x;
            int x = 0;
            if (idx < nk) {
                const int s = hci[hb + idx];
                const int s0 = rp[s];
                ks[idx] = s;
                sb[idx] = s0;
                x = rp[s + 1] - s0;
            }
            int incl = x;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            if (lane == 63) wsum[wave] = incl;
            __syncthreads();
            int before = 0, total = 0;
            for (int w = 0; w < (LB / 64); ++w) {
                before += w < wave ? wsum[w] : 0;
                total += wsum[w];
            }
            if (idx < nk) off[idx] = carry + before + incl - x;
            carry += total;
            __syncthreads();   // wsum is reused
        }
        if (threadIdx.x == 0) off[nk] = carry;
        __syncthreads();
        const int dpos = lower_bound_lds(ks, nk, k);
        if (dpos >= nk || ks[dpos] != k) continue;   // every operator stores its diagonal; never taken
        const int dk = hb + dpos;
        // off-diagonals (k,m), m > k: a wave per target, its lanes over row m;
        // the terms of dropped (k,j) first, then those of dropped (m,j), each
        // in ascending j (lane order)
        // a target's loads: its start value, the bounds of row m's kept
        // columns, and the first 64 entries of row m (a kept entry's den is
        // never written and is not used)
        struct Target {
            int m, mb, me, hm0, hm1, j0;
            double acc, a0, d0;
            uint8_t kp0;
        };
        auto fetch = [&](int tt) {
            Target g;
            g.m = ks[tt - hb];
            g.mb = sb[tt - hb];
            g.me = g.mb + off[tt - hb + 1] - off[tt - hb];
            g.hm0 = hrp[g.m];
            g.hm1 = hrp[g.m + 1];
            g.acc = hv[tt];
            const int r0 = min(g.mb + lane, g.me - 1);
            g.j0 = ci[r0];
            g.a0 = v[r0];
            g.d0 = den[r0];
            g.kp0 = keep[r0];
            return g;
        };
        Target nxt{};
        if (dk + 1 + wave < he) nxt = fetch(dk + 1 + wave);
        for (int t = dk + 1 + wave; t < he; t += (LB / 64)) {
            const Target cur = nxt;
            // the first chunk of the mirror row, then the next target's
            // loads: both in flight while this target's shares are formed
            const int hidx = cur.hm0 + lane;
            const int hc0 = hidx < cur.hm1 ? hci[hidx] : -1;
            if (t + (LB / 64) < he) nxt = fetch(t + (LB / 64));
            const int m = cur.m, mb = cur.mb, me = cur.me, hm0 = cur.hm0, hm1 = cur.hm1, j0 = cur.j0;
            const double a0 = cur.a0, d0 = cur.d0;
            const uint8_t kp0 = cur.kp0;
            double acc = cur.acc;
            const int w0 = lower_bound_lds(kc, len, j0);
            const bool at0 = w0 < len && kc[w0] == j0;   // j0 in row k
            for (int c0 = mb; c0 < me; c0 += 64) {   // (k,j) dropped, (j,m) strong: a_jm read as a_mj
                int j = j0, w = w0;
                double ajm = a0;
                bool at = at0;
                if (c0 != mb) {
                    const int r = min(c0 + lane, me - 1);
                    j = ci[r];
                    ajm = v[r];
                    w = lower_bound_lds(kc, len, j);
                    at = w < len && kc[w] == j;
                }
                bool has = false;
                double c = 0.0;
                if (c0 + lane < me && at && j != k && !kk[w]) {
                    const double th = kt[w];
                    if (th > 0.0 && -ajm >= th) {
                        c = (fabs(ajm) / kd[w]) * kv[w];
                        has = true;
                    }
                }
                acc = ordered_add(acc, has, c);
            }
            for (int c0 = mb; c0 < me; c0 += 64) {   // (m,j) dropped, (j,k) strong: a_jk read as a_kj
                int j = j0, w = w0;
                double a = a0, d = d0;
                bool at = at0, kp = kp0 != 0;
                if (c0 != mb) {
                    const int q = min(c0 + lane, me - 1);
                    j = ci[q];
                    a = v[q];
                    d = den[q];
                    kp = keep[q] != 0;
                    w = lower_bound_lds(kc, len, j);
                    at = w < len && kc[w] == j;
                }
                bool has = false;
                double c = 0.0;
                if (c0 + lane < me && j != m && !kp && at) {
                    const double th = kt[w], akj = kv[w];
                    if (th > 0.0 && -akj >= th) {
                        c = (fabs(akj) / d) * a;
                        has = true;
                    }
                }
                acc = ordered_add(acc, has, c);
            }
            // (m,k): the same value; its position by a coalesced search of row m
            int tm = -1;
            for (int c0 = hm0; c0 < hm1 && tm < 0; c0 += 64) {
                const int idx = c0 + lane;
                const int col = c0 == hm0 ? hc0 : (idx < hm1 ? hci[idx] : -1);
                const uint64_t hit = __ballot(idx < hm1 && col == k);
                if (hit) tm = c0 + __builtin_ctzll(hit);
            }
            if (lane == 0) {
                hv[t] = acc;
                if (tm >= 0) hv[tm] = acc;   // always found: the kept pattern is symmetric
            }
        }
        // the diagonal
        double acc = hv[dk];
        const int total = off[nk];
        for (int g = 0; g < total; g += kDiagPer * LB) {
            int qq[kDiagPer], ss[kDiagPer];
#pragma unroll
            for (int e = 0; e < kDiagPer; ++e) {
                const int f = g + e * LB + (int)threadIdx.x;
                qq[e] = -1;
                ss[e] = 0;
                if (f < total) {
                    int lo = 0, hi = nk;   // off[lo] <= f < off[lo + 1]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (off[mid] <= f) lo = mid;
                        else hi = mid;
                    }
                    ss[e] = ks[lo];
                    qq[e] = sb[lo] + (f - off[lo]);
                }
            }
            int jj[kDiagPer];
            uint8_t kp[kDiagPer];
            double dd[kDiagPer], aa[kDiagPer];
#pragma unroll
            for (int e = 0; e < kDiagPer; ++e) {
                const int q = qq[e] < 0 ? kb : qq[e];   // a valid entry; unused when qq < 0
                jj[e] = ci[q];
                kp[e] = keep[q];
                dd[e] = den[q];
                aa[e] = v[q];
            }
#pragma unroll
            for (int e = 0; e < kDiagPer; ++e) {
                bool has = false;
                double c = 0.0;
                if (qq[e] >= 0 && !kp[e]) {
                    const int s = ss[e], j = jj[e];
                    const double d = dd[e];
                    if (j != s && s == k) {
                        if (d == 0.0) {
                            c = aa[e];   // no strong neighbour kept: the whole entry
                            has = true;
                        } else {
                            const double t = kt[qq[e] - kb], a = aa[e];   // the share to k itself, a_jk = a_kj
                            if (t > 0.0 && -a >= t) {
                                c = (fabs(a) / d) * a;
                                has = true;
                            }
                        }
                    } else if (j != s && d != 0.0) {
                        const int r = lower_bound_lds(kc, len, j);
                        if (r < len && kc[r] == j) {
                            const double t = kt[r], a = kv[r];
                            if (t > 0.0 && -a >= t) {
                                c = -((fabs(a) / d) * aa[e]);   // a - c == a + (-c) exactly
                                has = true;
                            }
                        }
                    }
                }
                slot_c[e * LB + threadIdx.x] = c;
                slot_h[e * LB + threadIdx.x] = has ? 1 : 0;
            }
            __syncthreads();
            if (wave == 0)
                for (int w = 0; w < kDiagPer * (LB / 64); ++w)
                    acc = ordered_add(acc, slot_h[w * 64 + lane] != 0, slot_c[w * 64 + lane]);
            __syncthreads();   // the slots are reused
        }
        if (threadIdx.x == 0) hv[dk] = acc;
    }
}

}  // namespace

void launch_compact_copy(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                         const int32_t* new_rp, int32_t* new_ci, double* new_v, hipStream_t st) {
    hipLaunchKernelGGL(compact_copy_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, new_rp,
                       new_ci, new_v);
}

void launch_lump_threshold(int n, const int32_t* rp, const int32_t* ci, const double* v, double theta,
                           double* thr, hipStream_t st) {
    hipLaunchKernelGGL(lump_threshold_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, theta, thr);
}

namespace {

bool use_wide(const LumpShapes& ls, double mean_row) { return mean_row >= ls.wide_mean_row; }

bool use_den_wave(const LumpShapes& ls, int n, double mean_row) {
    if (ls.den_wave_mean_row >= 0.0) return mean_row < ls.den_wave_mean_row;
    return n >= kDenWaveMinRows && mean_row < kDenWaveMeanRow;
}

int row_grid_of(int n) { return std::max(1, std::min(n, 65536)); }

}  // namespace

void launch_lump_den(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                     const double* thr, double* den, double mean_row, const LumpShapes& ls, hipStream_t st) {
    if (use_wide(ls, mean_row) && use_den_wave(ls, n, mean_row))
        hipLaunchKernelGGL(lump_den_wave_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr,
                           den);
    else if (use_wide(ls, mean_row))
        hipLaunchKernelGGL(lump_den_wide_kernel, dim3(row_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr,
                           den);
    else
        hipLaunchKernelGGL(lump_den_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr, den);
}

void launch_strong_lump(int n, const int32_t* rp, const int32_t* ci, const double* v, const uint8_t* keep,
                        const double* thr, const double* den, const int32_t* hrp, const int32_t* hci, double* hv,
                        double mean_row, const LumpShapes& ls, hipStream_t st) {
    if (use_wide(ls, mean_row) && n < ls.small_rows)
        hipLaunchKernelGGL(strong_lump_wide_kernel<1024>, dim3(row_grid_of(n)), dim3(1024), 0, st, n, rp, ci, v, keep,
                           thr, den, hrp, hci, hv);
    else if (use_wide(ls, mean_row))
        hipLaunchKernelGGL(strong_lump_wide_kernel<kLB>, dim3(row_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep,
                           thr, den, hrp, hci, hv);
    else
        hipLaunchKernelGGL(strong_lump_kernel, dim3(wave_grid_of(n)), dim3(kLB), 0, st, n, rp, ci, v, keep, thr, den,
                           hrp, hci, hv);
}

}  // namespace amg355
