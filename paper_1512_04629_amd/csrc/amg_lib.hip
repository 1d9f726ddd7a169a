// Device hierarchy, sparsification pipeline, V-cycle, outer iterations and
// the C ABI of libamg355.
//
//   setup       Section 2 (amg_setup) on the host, uploaded once; the
//               Galerkin operators A_l are retained on the device.
//   sparsify    Section 3 (sparse_hybrid_setup, Sparse Galerkin) with the
//               Algorithm 3 keep set and the diagonal lumping of Algorithm 3b,
//               entirely in device kernels (minimal pattern, row maxima, keep
//               flags, scan, compaction with lumping).
//   reintroduce Section 6 (adaptive_solve): gamma ladder on s levels and
//               re-sparsification from the retained A_l.
//   solve       Section 2 (amg_solve V-cycle), stationary or as the CG
//               preconditioner, with the windowed adaptive control of
//               Section 6.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/amg.h"
#include "block_kernels.hpp"
#include "host_setup.hpp"
#include "kernels.hpp"
#include "lump_kernels.hpp"
#include "relax_kernels.hpp"
#include "setup_kernels.hpp"

using namespace amg355;

namespace {

struct AmgFailure {
    amg_status status;
    std::string what;
};

#define HIP_CHECK(expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw AmgFailure{AMG_ERR_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)}; \
    } while (0)

constexpr int kMaxDenseCoarse = 4096;
// CSR index and value arrays carry this many spare entries so that kernels
// may read whole 16-byte packs at the end of a matrix
constexpr int kCsrPad = 4;

// device scalar slots
// Block solves use 16 slots per quantity: squared residual norms (S_BLOCK),
// r.z of two iterations (S_BRZ0, S_BRZ1), p.Ap (S_BPQ), active flags (S_BACT),
// load flags (S_BLOAD), the number of leading columns the block kernels
// compute (S_LIVE, one slot, right after the load flags so that one copy
// sets all three), |b|^2 of each batch slot (S_BNR0), breakdown flags
// (S_BFLAG), |b|^2 of freshly loaded columns (S_BNEW), and the batch slots'
// iteration counts, states and residual ratios (S_BITER, S_BSTAT, S_BREL).
enum : int { S_RZ0 = 0, S_RZ1 = 1, S_PQ = 2, S_NR2 = 3, S_FLAG = 4, S_NRT = 5, S_DOT = 6, S_BLOCK = 8,
             S_BRZ0 = 24, S_BRZ1 = 40, S_BPQ = 56, S_BACT = 72, S_BLOAD = 88, S_LIVE = 104, S_BNR0 = 112,
             S_BFLAG = 128, S_BNEW = 144, S_BITER = 160, S_BSTAT = 176, S_BREL = 192, S_COUNT = 208 };
constexpr int kMaxBlockRhs = 16;

struct DevMat {
    int rows = 0, cols = 0;
    int64_t nnz = 0;          // number of stored entries (valid when nnz_known)
    int64_t shape_nnz = 0;    // entry count the launch configuration is chosen for
    bool nnz_known = true;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* v = nullptr;
    int width = 8;
    // 16-bit column indices for the LDS-staged kernels (null: not built)
    uint16_t* ci16 = nullptr;
    int32_t* cbase = nullptr;
    int idx_rb = 0;
    // SELL-64 copy for the row operations (null: not built); its columns in
    // 32 bits (sl_col) or as 16-bit offsets from a base per slice
    int32_t* sl_off = nullptr;
    int32_t* sl_col = nullptr;
    double* sl_val = nullptr;
    int sl_maxw = 0;
    uint16_t* sl_col16 = nullptr;
    int32_t* sl_base = nullptr;
    uint8_t* sl_idx8 = nullptr;       // or 8-bit positions in a table of offsets per slice
    int32_t* sl_tab = nullptr;
    int64_t sl_cap = 0;               // entries the SELL-64 arrays hold
    float* sl_val32 = nullptr;        // FP32 values of the copy (FP32 cycle; built with the FP32 mirror)
    // direction of this operator's next cycle pass (flipped by every pass),
    // shared with the copies that alias the operator (Ah = A), so that
    // passes alternate whichever copy they go through
    std::shared_ptr<int> next_rev = std::make_shared<int>(0);
    CsrView view() const {
        return CsrView{rp, ci, v, rows, rows ? (double)shape_nnz / rows : 1.0, ci16, cbase, idx_rb, 0,
                       sl_off, sl_col, sl_val, sl_maxw, sl_col16, sl_base, sl_idx8, sl_tab};
    }
};

struct DevLevel {
    int n = 0;
    DevMat A;             // Galerkin operator (retained)
    DevMat Ah;            // operator the cycle uses: A while ah_alias, else Ahs
    bool ah_alias = true;
    DevMat Ahs;           // storage of the sparsified operator, capacity nnz(A)
    DevMat P, R;          // l < L
    int32_t* c_points = nullptr;  // fine index of each coarse point of level l+1
    int nc = 0;
    double* dinv = nullptr;       // 1 / diag(Ah)
    uint8_t* in_m = nullptr;      // minimal pattern flags (l >= 1)
    uint8_t* keep = nullptr;      // keep flags of the last sparsification
    int32_t* kcnt = nullptr;      // kept entries per row, and per block of the keep_count launch
    int32_t* kbsum = nullptr;     //   (regions of the handle's sp_cnt / sp_bsum)
    double* rowmax = nullptr;     // m_i of A
    double* lump_thr = nullptr;   // strong-neighbour lumping: strength thresholds of A's rows
    double* lump_den = nullptr;   //   and share denominators per dropped entry of A
    bool have_m = false;
    bool m_hybrid = false;        // in_m currently holds the Hybrid Galerkin pattern
    bool keep_valid = false;
    double gamma = 0.0;
    double *b = nullptr, *x = nullptr, *xt = nullptr, *r = nullptr;
    std::vector<int32_t> split;
    // FP32 mirror for the single-precision V-cycle (indices shared with the
    // FP64 operators; allocated on the first FP32 solve)
    float* A32 = nullptr;
    float* Ahs32 = nullptr;
    float* P32 = nullptr;
    float* R32 = nullptr;
    float* dinv32 = nullptr;
    float *b32 = nullptr, *x32 = nullptr, *xt32 = nullptr, *r32 = nullptr;
};

// work blocks of the multi-right-hand-side cycle in one precision: K-wide
// (row-interleaved) per level; rhs is the level-0 right-hand side of a
// correction cycle
template <class T>
struct BlockBufs {
    int k = 0;
    std::vector<T*> b, x, xt, r;
    T* rhs = nullptr;
};

struct ProfAcc {
    int64_t count = 0;
    double ms = 0.0;
};

struct PendingEvent {
    int kind, level;
    hipEvent_t start, stop;
};

}  // namespace

struct amg_batch_ctx;

struct amg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    amg_alloc_fn alloc_fn = nullptr;
    amg_free_fn free_fn = nullptr;
    void* user = nullptr;
    std::unordered_map<void*, size_t> blocks;
    amg_setup_params sp{};
    std::vector<DevLevel> lv;
    int nL = 0;
    double* coarse_inv = nullptr;
    double* scal = nullptr;
    double* partials = nullptr;
    int partial_cap = 0;
    double* pinned = nullptr;        // host-coherent: the scalar slots, then the readback sequence word
    double* pinned_dev = nullptr;    // its device address
    uint32_t* flag_host = nullptr;
    uint32_t* flag_dev = nullptr;
    uint32_t pub_seq = 0;
    int32_t* scan_scratch = nullptr;
    int32_t* cnt = nullptr;
    int32_t* sp_cnt = nullptr;    // every level's kcnt
    int32_t* sp_bsum = nullptr;   // every level's kbsum
    int* missing = nullptr;          // minimal-pattern and index-width checks
    int* singular = nullptr;         // zero pivot met by the device inversion of the coarsest operator
    double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr;
    double *xw = nullptr, *rt = nullptr;
    bool fp32 = false;
    float *cg_r32 = nullptr, *cg_z32 = nullptr;
    BlockBufs<double> blk64;
    BlockBufs<float> blk32;
    double* blk_partials = nullptr;
    double *blk_b = nullptr, *blk_x = nullptr;   // K-wide copies when nrhs is not a block width
    amg_batch_ctx* batch = nullptr;              // the continuous-batching engine, if any
    int method = AMG_SPARSE_GALERKIN;            // which finer operator the minimal pattern uses
    bool nongalerkin = false;                    // coarse operators sparsified during setup
    bool compact_idx = true;                     // 16-bit column indices where they fit
    int relax = AMG_RELAX_JACOBI;                // smoother of the V-cycle
    int lumping = AMG_LUMP_DIAGONAL;             // where sparsify puts dropped entries
    LumpShapes lump_shapes;                      // launch shapes of the strong-lumping kernels
    int gs_block = 64;                           // rows per block of hybrid Gauss-Seidel
    int bcg_k = 0;                               // block CG vectors (FP64, K wide)
    double *bcg_r = nullptr, *bcg_p = nullptr, *bcg_q = nullptr, *bcg_z = nullptr;
    int blk_pack_k = 0;
    std::string last_error;
    bool check_singular = false;   // a device inversion wrote h->singular, not read back yet
    bool profiling = false;
    int prof_kind = -1, prof_level = -1;
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<ProfAcc> prof;   // [kind * max_levels + level]
};

namespace {

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------
void* dalloc(amg_ctx* h, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (h->alloc_fn) {
        p = h->alloc_fn(bytes, (void*)h->stream, h->user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) throw AmgFailure{AMG_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    h->blocks[p] = bytes;
    return p;
}

template <class T>
T* dalloc_n(amg_ctx* h, int64_t n) {
    return static_cast<T*>(dalloc(h, sizeof(T) * (size_t)std::max<int64_t>(n, 1)));
}

void dfree(amg_ctx* h, void* p) {
    if (!p) return;
    auto it = h->blocks.find(p);
    size_t bytes = it == h->blocks.end() ? 0 : it->second;
    if (it != h->blocks.end()) h->blocks.erase(it);
    if (h->free_fn) h->free_fn(p, bytes, (void*)h->stream, h->user);
    else (void)hipFree(p);
}

void free_mat(amg_ctx* h, DevMat& m) {
    dfree(h, m.rp);
    dfree(h, m.ci);
    dfree(h, m.v);
    dfree(h, m.ci16);
    dfree(h, m.cbase);
    dfree(h, m.sl_off);
    dfree(h, m.sl_col);
    dfree(h, m.sl_val);
    dfree(h, m.sl_col16);
    dfree(h, m.sl_base);
    dfree(h, m.sl_idx8);
    dfree(h, m.sl_tab);
    dfree(h, m.sl_val32);
    m = DevMat{};
}

template <class T>
void upload(amg_ctx* h, T* dst, const T* src, int64_t n) {
    if (n > 0) HIP_CHECK(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)n, hipMemcpyHostToDevice, h->stream));
}

template <class T>
void download(amg_ctx* h, T* dst, const T* src, int64_t n) {
    if (n > 0) HIP_CHECK(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, h->stream));
}

void sync(amg_ctx* h) { HIP_CHECK(hipStreamSynchronize(h->stream)); }

void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw AmgFailure{AMG_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e)};
}

// launch shape of a matrix with nnz stored entries
void set_shape(DevMat& d, int64_t nnz) {
    d.nnz = nnz;
    d.nnz_known = true;
    d.shape_nnz = nnz;
    d.width = pick_width(d.rows ? (double)nnz / d.rows : 1.0);
}

DevMat upload_mat(amg_ctx* h, const HostCsr& m) {
    DevMat d;
    d.rows = m.rows;
    d.cols = m.cols;
    d.rp = dalloc_n<int32_t>(h, d.rows + 1);
    d.ci = dalloc_n<int32_t>(h, m.nnz() + kCsrPad);
    d.v = dalloc_n<double>(h, m.nnz() + kCsrPad);
    set_shape(d, m.nnz());
    upload(h, d.rp, m.ptr.data(), d.rows + 1);
    upload(h, d.ci, m.idx.data(), d.nnz);
    upload(h, d.v, m.val.data(), d.nnz);
    return d;
}

HostCsr download_mat(amg_ctx* h, const DevMat& d) {
    HostCsr m;
    m.rows = d.rows;
    m.cols = d.cols;
    m.ptr.resize(d.rows + 1);
    m.idx.resize(d.nnz);
    m.val.resize(d.nnz);
    download(h, m.ptr.data(), d.rp, d.rows + 1);
    download(h, m.idx.data(), d.ci, d.nnz);
    download(h, m.val.data(), d.v, d.nnz);
    sync(h);
    return m;
}

// ---------------------------------------------------------------------------
// profiling: events around launches of one kernel class on one level
// ---------------------------------------------------------------------------
// kernel_events: the scope holds one row-kernel launch, whose own start and
// end the events record (hipExtLaunchKernel); otherwise they are recorded on
// the stream around everything the scope launches
struct ProfScope {
    amg_ctx* h;
    int kind, level;
    hipEvent_t stop = nullptr;
    bool armed = false;
    ProfScope(amg_ctx* hh, int k, int l, bool kernel_events = false) : h(hh), kind(k), level(l) {
        if (!h->profiling) return;
        if ((h->prof_kind >= 0 && h->prof_kind != k) || (h->prof_level >= 0 && h->prof_level != l)) return;
        hipEvent_t start = take_event();
        stop = take_event();
        if (kernel_events) {
            set_launch_events(start, stop);
            armed = true;
        } else {
            HIP_CHECK(hipEventRecord(start, h->stream));
        }
        h->pending.push_back(PendingEvent{kind, level, start, stop});
    }
    ~ProfScope() {
        if (armed) {
            // a launch that did not take the events (none happens) leaves them unrecorded
            if (clear_launch_events()) {
                (void)hipEventRecord(h->pending.back().start, h->stream);
                (void)hipEventRecord(stop, h->stream);
            }
            return;
        }
        if (stop) (void)hipEventRecord(stop, h->stream);
    }
    hipEvent_t take_event() {
        if (!h->event_pool.empty()) {
            hipEvent_t e = h->event_pool.back();
            h->event_pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        return e;
    }
};

void prof_collect(amg_ctx* h) {
    if (h->pending.empty()) return;
    sync(h);
    const int ml = std::max(1, (int)h->lv.size());
    for (auto& pe : h->pending) {
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, pe.start, pe.stop));
        size_t idx = (size_t)pe.kind * ml + std::min(pe.level, ml - 1);
        if (idx < h->prof.size()) {
            h->prof[idx].count += 1;
            h->prof[idx].ms += ms;
        }
        h->event_pool.push_back(pe.start);
        h->event_pool.push_back(pe.stop);
    }
    h->pending.clear();
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
DotTarget dot_to(amg_ctx* h, int slot) { return DotTarget{h->partials, h->scal + slot}; }

void row_op(amg_ctx* h, int kind, int level, RowOp op, const DevMat& m, const double* g,
            const double* u, const double* dinv, double* y, double* y2, int dot_slot) {
    DotTarget dt = dot_slot >= 0 ? dot_to(h, dot_slot) : DotTarget{nullptr, nullptr};
    CsrView cv = m.view();
    cv.rev = *m.next_rev;
    *m.next_rev ^= 1;
    int nparts = 0;
    {
        // the events time the row kernel alone; the dot's finishing launch follows
        ProfScope ps(h, kind, level, true);
        nparts = launch_row_op(op, m.width, cv, g, u, dinv, h->sp.omega, y, y2, dt, h->stream);
        check_launch();
    }
    if (nparts > 0) {
        launch_dot_finish(dt, nparts, h->stream);
        check_launch();
    }
}

void row_op(amg_ctx* h, int kind, int level, RowOp op, const DevMat& m, const float* vals, const float* g,
            const float* u, const float* dinv, float* y, float* y2) {
    ProfScope ps(h, kind, level, true);
    // the SELL-64 copy's FP32 values are the same narrowed values in slice order
    const CsrView32 a32{m.rp, m.ci, vals, m.rows, m.view().mean_row, m.ci16, m.cbase, m.idx_rb, *m.next_rev,
                        m.sl_val32 ? m.sl_off : nullptr, m.sl_col, m.sl_val32, m.sl_maxw, m.sl_col16, m.sl_base,
                        m.sl_idx8, m.sl_tab};
    *m.next_rev ^= 1;
    launch_row_op(op, m.width, a32, g, u, dinv, (float)h->sp.omega, y, y2, h->stream);
    check_launch();
}

// ---------------------------------------------------------------------------
// coarse-level dense inverse (host factorization, applied by a device kernel)
// ---------------------------------------------------------------------------
bool dense_inverse(int n, std::vector<double>& a, std::vector<double>& inv) {
    // Cholesky A = L L^T, then inv = L^-T L^-1; Gauss-Jordan with partial
    // pivoting if a pivot is not positive.
    std::vector<double> L(a.size(), 0.0);
    bool spd = true;
    for (int j = 0; j < n && spd; ++j) {
        double d = a[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) { spd = false; break; }
        const double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = a[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    if (spd) {
        // columns of L^-1 by forward substitution, then inv = L^-T L^-1
        std::vector<double> Li((size_t)n * n, 0.0);
        for (int c = 0; c < n; ++c) {
            for (int i = c; i < n; ++i) {
                double t = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) t -= L[(size_t)i * n + k] * Li[(size_t)k * n + c];
                Li[(size_t)i * n + c] = t / L[(size_t)i * n + i];
            }
        }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int k = std::max(i, j); k < n; ++k) t += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
                inv[(size_t)i * n + j] = t;
            }
        return true;
    }
    std::vector<double> m = a;
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(m[(size_t)i * n + c]) > std::fabs(m[(size_t)piv * n + c])) piv = i;
        if (m[(size_t)piv * n + c] == 0.0) return false;
        if (piv != c)
            for (int j = 0; j < n; ++j) {
                std::swap(m[(size_t)c * n + j], m[(size_t)piv * n + j]);
                std::swap(inv[(size_t)c * n + j], inv[(size_t)piv * n + j]);
            }
        const double d = m[(size_t)c * n + c];
        for (int j = 0; j < n; ++j) { m[(size_t)c * n + j] /= d; inv[(size_t)c * n + j] /= d; }
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            const double f = m[(size_t)i * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                m[(size_t)i * n + j] -= f * m[(size_t)c * n + j];
                inv[(size_t)i * n + j] -= f * inv[(size_t)c * n + j];
            }
        }
    }
    return true;
}

// Number of stored entries of a sparsified operator: kept on the device by
// the scan and read back only when asked for.
int64_t operator_nnz(amg_ctx* h, DevMat& m) {
    if (!m.nnz_known) {
        int32_t total = 0;
        download(h, &total, m.rp + m.rows, 1);
        sync(h);
        m.nnz = total;
        m.nnz_known = true;
    }
    return m.nnz;
}

void refresh_coarse_inverse(amg_ctx* h) {
    DevLevel& c = h->lv.back();
    const int n = c.n;
    if (!h->coarse_inv || h->nL != n) {
        dfree(h, h->coarse_inv);
        h->coarse_inv = dalloc_n<double>(h, (int64_t)n * n);
    }
    h->nL = n;
    if (n <= dense_invert_max()) {
        // on the device, stream ordered after the operator it inverts
        launch_fill_u32(1, reinterpret_cast<unsigned*>(h->singular), 0u, h->stream);
        launch_dense_invert(c.Ah.view(), h->coarse_inv, h->singular, h->stream);
        check_launch();
        h->check_singular = true;
        return;
    }
    operator_nnz(h, c.Ah);
    HostCsr m = download_mat(h, c.Ah);
    std::vector<double> a((size_t)n * n, 0.0), inv;
    for (int i = 0; i < n; ++i)
        for (int p = m.ptr[i]; p < m.ptr[i + 1]; ++p) a[(size_t)i * n + m.idx[p]] = m.val[p];
    if (!dense_inverse(n, a, inv))
        throw AmgFailure{AMG_ERR_BAD_MATRIX, "coarsest operator is singular"};
    upload(h, h->coarse_inv, inv.data(), (int64_t)n * n);
    sync(h);
}

// ---------------------------------------------------------------------------
// sparsification (device)
// ---------------------------------------------------------------------------
void ensure_minimal_pattern(amg_ctx* h, int l) {
    DevLevel& c = h->lv[l];
    if (c.have_m) return;
    DevLevel& f = h->lv[l - 1];
    if (!c.in_m) c.in_m = dalloc_n<uint8_t>(h, c.A.nnz);
    if (!c.keep) c.keep = dalloc_n<uint8_t>(h, c.A.nnz);
    if (!c.rowmax) c.rowmax = dalloc_n<double>(h, c.n);
    {
        ProfScope ps(h, AMG_K_SPARSIFY, l);
        launch_fill_u8(c.A.nnz, c.in_m, 0, h->stream);
        launch_fill_u32(1, reinterpret_cast<unsigned*>(h->missing), 0u, h->stream);
        launch_mark_minimal_pattern(c.n, f.c_points, f.A.rp, f.A.ci, f.P.rp, f.P.ci, c.A.rp, c.A.ci,
                                    c.in_m, h->missing, h->stream);
        launch_row_max(c.A.width, c.A.view(), c.rowmax, h->stream);
        check_launch();
    }
    int missing = 0;
    download(h, &missing, h->missing, 1);
    sync(h);
    if (missing) throw AmgFailure{AMG_ERR_BAD_MATRIX, "minimal pattern of level " + std::to_string(l) + " is not inside the Galerkin pattern"};
    c.have_m = true;
}

// Minimal pattern of level l from the finer operator the method prescribes
// (Section 3, sparse_hybrid_setup): the Galerkin A_{l-1} (Sparse Galerkin)
// or the current sparsified \hat A_{l-1} (Hybrid Galerkin), asynchronously.
// The pattern of \hat A_{l-1} lies inside that of A_{l-1}, so this pattern
// lies inside the Sparse Galerkin one, which ensure_minimal_pattern checked.
void mark_minimal_pattern(amg_ctx* h, int l, bool hybrid) {
    ensure_minimal_pattern(h, l);
    DevLevel& c = h->lv[l];
    if (!hybrid && !c.m_hybrid) return;
    DevLevel& f = h->lv[l - 1];
    const DevMat& fine = hybrid ? f.Ah : f.A;
    ProfScope ps(h, AMG_K_SPARSIFY, l);
    launch_fill_u8(c.A.nnz, c.in_m, 0, h->stream);
    launch_mark_minimal_pattern(c.n, f.c_points, fine.rp, fine.ci, f.P.rp, f.P.ci, c.A.rp, c.A.ci, c.in_m,
                                h->missing, h->stream);
    check_launch();
    c.m_hybrid = hybrid;
}

// Rebuilds the sparsified operators of the given levels at the given
// tolerances, asynchronously on the handle's stream.  The storage of a
// sparsified operator is allocated once with the capacity of the Galerkin
// operator, so after the first call nothing is allocated and nothing waits
// for the device; any allocation happens before a level is modified.
// levels of at most this many rows are sparsified together, one launch for
// their keep flags and one for their compaction (their launches cost more
// than their work)
constexpr int kMergeRows = 8192;
bool merge_level(const DevLevel& c) { return c.n <= kMergeRows; }

void sparsify_levels(amg_ctx* h, const std::vector<std::pair<int, double>>& todo) {
    for (auto& t : todo) {
        DevLevel& c = h->lv[t.first];
        if (t.second == 0.0) continue;
        ensure_minimal_pattern(h, t.first);
        if (!c.Ahs.rp) {
            c.Ahs.rows = c.Ahs.cols = c.n;
            c.Ahs.rp = dalloc_n<int32_t>(h, c.n + 1);
            c.Ahs.ci = dalloc_n<int32_t>(h, c.A.nnz + kCsrPad);
            c.Ahs.v = dalloc_n<double>(h, c.A.nnz + kCsrPad);
            c.Ahs.shape_nnz = c.A.nnz;
            c.Ahs.width = c.A.width;
        }
        if (h->fp32 && !c.Ahs32) c.Ahs32 = dalloc_n<float>(h, c.A.nnz + kCsrPad);
        if (h->lumping == AMG_LUMP_STRONG && !c.lump_thr) {
            c.lump_thr = dalloc_n<double>(h, c.n);
            c.lump_den = dalloc_n<double>(h, c.A.nnz);
        }
    }
    bool coarse_changed = false;
    // Diagonal lumping in three steps over the levels: keep flags with row and
    // block counts (one launch per level), the scans of every level's block
    // counts (one launch), compaction (one launch per level, row pointers
    // from the block offsets).  A Hybrid Galerkin pattern needs the finer
    // operator this call has just rebuilt, so there the levels go one at a
    // time; strong-neighbour lumping keeps its own steps.
    const bool one_by_one = h->method == AMG_HYBRID_GALERKIN;
    size_t next = 0;
    while (next < todo.size()) {
        const size_t first = next;
        size_t last = one_by_one ? next + 1 : todo.size();
        ScanJobs jobs;
        SparsifyLevels merged;
        std::vector<char> in_merged(todo.size(), 0);
        for (size_t q = first; q < last; ++q) {
            const int l = todo[q].first;
            const double gamma = todo[q].second;
            DevLevel& c = h->lv[l];
            ProfScope ps(h, AMG_K_SPARSIFY, l);
            if (gamma == 0.0) {
                if (!c.ah_alias) {
                    c.Ah = c.A;
                    c.ah_alias = true;
                    launch_inverse_diagonal(c.A.view(), c.dinv, h->fp32 ? c.dinv32 : nullptr, h->stream);
                    if (l == (int)h->lv.size() - 1) coarse_changed = true;
                }
                c.gamma = 0.0;
                c.keep_valid = false;
                continue;
            }
            // levels are processed finest first, so a Hybrid pattern sees the
            // finer operator this call has just rebuilt
            mark_minimal_pattern(h, l, h->method == AMG_HYBRID_GALERKIN);
            if (h->lumping == AMG_LUMP_STRONG) {
                launch_keep_count(c.A.width, c.A.view(), c.in_m, c.rowmax, gamma, c.keep, c.kcnt, nullptr,
                                  h->stream);
                launch_exclusive_scan(c.n, c.kcnt, c.Ahs.rp, h->scan_scratch, h->stream);
                // Algorithm 3's second loop: dropped entries shared among strong neighbours
                const DevMat& a = c.A;
                launch_compact_copy(c.n, a.rp, a.ci, a.v, c.keep, c.Ahs.rp, c.Ahs.ci, c.Ahs.v, h->stream);
                launch_lump_threshold(c.n, a.rp, a.ci, a.v, h->sp.theta, c.lump_thr, h->stream);
                {
                    ProfScope pd(h, AMG_K_LUMP_DEN, l);
                    launch_lump_den(c.n, a.rp, a.ci, a.v, c.keep, c.lump_thr, c.lump_den, a.view().mean_row,
                                    h->lump_shapes, h->stream);
                }
                {
                    ProfScope pl(h, AMG_K_LUMP_SHARES, l);
                    launch_strong_lump(c.n, a.rp, a.ci, a.v, c.keep, c.lump_thr, c.lump_den, c.Ahs.rp, c.Ahs.ci,
                                       c.Ahs.v, a.view().mean_row, h->lump_shapes, h->stream);
                }
                launch_inverse_diagonal(c.Ahs.view(), c.dinv, h->fp32 ? c.dinv32 : nullptr, h->stream);
                if (h->fp32) launch_narrow(c.A.nnz, c.Ahs32, c.Ahs.v, h->stream);   // capacity; past nnz unused
            } else if (merge_level(c) && merged.count < kMaxMergedLevels) {
                // small levels: one launch for all of them, below
                in_merged[q] = 1;
                SparsifyLevel& v = merged.lv[merged.count++];
                v.a = c.A.view();
                v.in_m = c.in_m;
                v.m = c.rowmax;
                v.gamma = gamma;
                v.keep = c.keep;
                v.cnt = c.kcnt;
                v.bsum = c.kbsum;
                v.new_rp = c.Ahs.rp;
                v.new_ci = c.Ahs.ci;
                v.new_v = c.Ahs.v;
                v.dinv = c.dinv;
                v.new_v32 = h->fp32 ? c.Ahs32 : nullptr;
                v.dinv32 = h->fp32 ? c.dinv32 : nullptr;
                jobs.data[jobs.count] = c.kbsum;
                jobs.n[jobs.count] = keep_count_blocks(64, c.n);
                ++jobs.count;
            } else {
                launch_keep_count(c.A.width, c.A.view(), c.in_m, c.rowmax, gamma, c.keep, c.kcnt, c.kbsum,
                                  h->stream);
                jobs.data[jobs.count] = c.kbsum;
                jobs.n[jobs.count] = keep_count_blocks(c.A.width, c.n);
                ++jobs.count;
            }
            if (jobs.count == kMaxScanJobs) last = q + 1;   // the rest in the next round
            check_launch();
        }
        if (merged.count > 0) {
            ProfScope ps(h, AMG_K_SPARSIFY, todo[first].first);
            launch_keep_count_merged(merged, h->stream);
        }
        launch_scan_jobs(jobs, h->stream);
        if (merged.count > 0) {
            ProfScope ps(h, AMG_K_SPARSIFY, todo[first].first);
            launch_compact_lump_merged(merged, h->stream);
        }
        check_launch();
        for (size_t q = first; q < last; ++q) {
            const int l = todo[q].first;
            const double gamma = todo[q].second;
            if (gamma == 0.0) continue;
            DevLevel& c = h->lv[l];
            ProfScope ps(h, AMG_K_SPARSIFY, l);
            if (h->lumping != AMG_LUMP_STRONG && !in_merged[q])
                launch_compact_lump(c.A.width, c.A.view(), c.keep, c.kcnt, c.kbsum, c.Ahs.rp, c.Ahs.ci, c.Ahs.v,
                                    c.dinv, h->fp32 ? c.Ahs32 : nullptr, h->fp32 ? c.dinv32 : nullptr,
                                    h->stream);
            c.Ahs.nnz_known = false;
            c.Ah = c.Ahs;
            c.ah_alias = false;
            c.gamma = gamma;
            c.keep_valid = true;
            if (l == (int)h->lv.size() - 1) coarse_changed = true;
            check_launch();
        }
        next = last;
    }
    if (coarse_changed) refresh_coarse_inverse(h);
}

// ---------------------------------------------------------------------------
// V-cycle (Section 2, amg_solve): weighted Jacobi pre/post smoothing,
// restriction of the residual with R = P^T, coarsest dense solve,
// interpolation and correction.  Written once for both precisions: FP64
// (the method as stated) and FP32 (values, vectors and accumulation in single
// precision, used as a preconditioner of FP64 iterations; the coarsest solve
// keeps its FP64 inverse).
// ---------------------------------------------------------------------------

// the per-level arrays of one precision
template <class T>
struct LevelView {
    int n = 0;
    const DevMat* Ah = nullptr;
    const DevMat* P = nullptr;
    const DevMat* R = nullptr;
    const T *ahv = nullptr, *pv = nullptr, *rv = nullptr, *dinv = nullptr;
    T *b = nullptr, *x = nullptr, *xt = nullptr, *r = nullptr;
};

LevelView<double> level_view(amg_ctx* h, int l, double*) {
    DevLevel& v = h->lv[l];
    LevelView<double> o;
    o.n = v.n;
    o.Ah = &v.Ah; o.P = &v.P; o.R = &v.R;
    o.ahv = v.Ah.v; o.pv = v.P.v; o.rv = v.R.v; o.dinv = v.dinv;
    o.b = v.b; o.x = v.x; o.xt = v.xt; o.r = v.r;
    return o;
}

LevelView<float> level_view(amg_ctx* h, int l, float*) {
    DevLevel& v = h->lv[l];
    LevelView<float> o;
    o.n = v.n;
    o.Ah = &v.Ah; o.P = &v.P; o.R = &v.R;
    o.ahv = v.ah_alias ? v.A32 : v.Ahs32;
    o.pv = v.P32; o.rv = v.R32; o.dinv = v.dinv32;
    o.b = v.b32; o.x = v.x32; o.xt = v.xt32; o.r = v.r32;
    return o;
}

void row_op_t(amg_ctx* h, int kind, int l, RowOp op, const DevMat& m, const double*, const double* g,
              const double* u, const double* dinv, double* y, double* y2, int dot_slot) {
    row_op(h, kind, l, op, m, g, u, dinv, y, y2, dot_slot);
}

void row_op_t(amg_ctx* h, int kind, int l, RowOp op, const DevMat& m, const float* vals, const float* g,
              const float* u, const float* dinv, float* y, float* y2, int) {
    row_op(h, kind, l, op, m, vals, g, u, dinv, y, y2);
}

void fill_t(int64_t n, double* p, amg_ctx* h) { launch_fill_f64(n, p, 0.0, h->stream); }
void fill_t(int64_t n, float* p, amg_ctx* h) { launch_fill_f32(n, p, 0.0f, h->stream); }

template <class T>
void jacobi_sweeps(amg_ctx* h, int l, const LevelView<T>& v, const T* b, T*& cur, T*& alt, int sweeps,
                   int dot_slot_last) {
    for (int s = 0; s < sweeps; ++s) {
        const bool last = s == sweeps - 1;
        if (last && dot_slot_last >= 0)
            row_op_t(h, AMG_K_JACOBI, l, kJacobiDot, *v.Ah, v.ahv, cur, b, v.dinv, alt, nullptr, dot_slot_last);
        else
            row_op_t(h, AMG_K_JACOBI, l, kJacobi, *v.Ah, v.ahv, cur, b, v.dinv, alt, nullptr, -1);
        std::swap(cur, alt);
    }
}

enum class Guess { kNonzero, kZero, kPrescaled };

// First level handled by the single-workgroup coarse tail: the finest level
// >= 1 with at most kTailRows rows, if it is above the coarsest; 0 = no tail.
// The tail implements V(1,1) only.
#ifndef AMG_TAIL_ROWS
#define AMG_TAIL_ROWS 256
#endif
constexpr int kTailRows = AMG_TAIL_ROWS;
int tail_start(const amg_ctx* h) {
    const int L = (int)h->lv.size() - 1;
    if (h->sp.nu_pre != 1 || h->sp.nu_post != 1 || L < 2) return 0;
    for (int l = 1; l < L; ++l)
        if (h->lv[l].n <= kTailRows) return (L - l + 1 <= kTailMaxLevels) ? l : 0;
    return 0;
}

// Buffer that receives the zero-guess smoothing sweep omega D^-1 b of level
// l: on level 0 chosen so that after all later sweeps (each swaps buffers)
// the result lands in x0.
template <class T>
T* zero_start(amg_ctx* h, int l, T* x0) {
    LevelView<T> v = level_view(h, l, (T*)nullptr);
    if (l > 0) return v.x;
    const int swaps = std::max(h->sp.nu_pre - 1, 0) + h->sp.nu_post;
    return (swaps & 1) ? v.xt : x0;
}

// guess0: kNonzero -- x0 holds the iterate; kZero -- the iterate is zero;
// kPrescaled -- the iterate is zero and zero_start(h, 0, x0) already holds
// the first sweep omega D^-1 b0 (written by the CG update).  dot_slot >= 0
// (FP64 only): accumulate b0 . x0 (the CG inner product r.z) into that slot.
// The result is left in x0.
// l0_resid_ready: with guess0 = kPrescaled and one pre-sweep, the level-0
// residual of the prescaled sweep is already in level 0's r (formed together
// with the window's true residual), so the cycle does not form it again.
template <class T>
void vcycle(amg_ctx* h, const T* b0, T* x0, Guess guess0, int dot_slot, bool l0_resid_ready = false) {
    const int L = (int)h->lv.size() - 1;
    const int pre = h->sp.nu_pre, post = h->sp.nu_post;
    const T omega = (T)h->sp.omega;
    if (L == 0) {
        ProfScope ps(h, AMG_K_COARSE, 0);
        launch_dense_matvec(h->nL, h->coarse_inv, b0, x0, h->stream);
        check_launch();
        if constexpr (sizeof(T) == 8)
            if (dot_slot >= 0) launch_dot(h->lv[0].n, b0, x0, dot_to(h, dot_slot), h->stream);
        return;
    }
    std::vector<T*> cur(L + 1), alt(L + 1);
    const int tail = tail_start(h);
    const int down_end = tail > 0 ? tail : L;
    for (int l = 0; l < down_end; ++l) {
        LevelView<T> v = level_view(h, l, (T*)nullptr);
        const T* b = l == 0 ? b0 : v.b;
        const bool zero = l > 0 || guess0 != Guess::kNonzero;
        // on coarse levels the restriction has already written omega D^-1 b
        const bool prescaled = pre >= 1 && (l > 0 || guess0 == Guess::kPrescaled);
        cur[l] = zero ? zero_start<T>(h, l, x0) : x0;
        alt[l] = cur[l] == v.xt ? (l == 0 ? x0 : v.x) : v.xt;
        bool have_resid = false;
        if (zero) {
            if (pre == 0) {
                fill_t(v.n, cur[l], h);
                launch_copy(v.n, v.r, b, h->stream);
                have_resid = true;
            } else if (pre == 1 && !prescaled) {
                row_op_t(h, AMG_K_JACOBI_ZERO, l, kZeroJacobiResid, *v.Ah, v.ahv, nullptr, b, v.dinv, v.r,
                         cur[l], -1);
                have_resid = true;
            } else {
                if (!prescaled) launch_scaled_copy(v.n, cur[l], v.dinv, b, omega, h->stream);
                jacobi_sweeps<T>(h, l, v, b, cur[l], alt[l], pre - 1, -1);
            }
        } else {
            jacobi_sweeps<T>(h, l, v, b, cur[l], alt[l], pre, -1);
        }
        const bool ready0 = l == 0 && l0_resid_ready && zero && pre == 1 && prescaled;
        if (!have_resid && !ready0) {
            const int kind = (zero && pre == 1) ? AMG_K_JACOBI_ZERO : AMG_K_RESIDUAL;
            row_op_t(h, kind, l, kResid, *v.Ah, v.ahv, cur[l], b, nullptr, v.r, nullptr, -1);
        }
        LevelView<T> nx = level_view(h, l + 1, (T*)nullptr);
        if (pre >= 1 && l + 1 < L)
            row_op_t(h, AMG_K_RESTRICT, l, kSpmvScale, *v.R, v.rv, v.r, nullptr, nx.dinv, nx.b,
                     zero_start<T>(h, l + 1, nullptr), -1);
        else
            row_op_t(h, AMG_K_RESTRICT, l, kSpmv, *v.R, v.rv, v.r, nullptr, nullptr, nx.b, nullptr, -1);
    }
    if (tail > 0) {
        // levels tail..L in one workgroup; the level-tail result lands in its xt
        TailArgs<T> ta{};
        ta.count = L - tail + 1;
        ta.coarse_inv = h->coarse_inv;
        ta.omega = omega;
        for (int k = 0; k < ta.count; ++k) {
            LevelView<T> v = level_view(h, tail + k, (T*)nullptr);
            TailLevel<T>& t = ta.lv[k];
            // a sparsified operator's arrays hold the Galerkin operator's entry count
            t.A = TailCsr<T>{v.Ah->rp, v.Ah->ci, v.ahv, v.Ah->rows, (int)v.Ah->shape_nnz};
            if (tail + k < L) {
                t.R = TailCsr<T>{v.R->rp, v.R->ci, v.rv, v.R->rows, (int)v.R->nnz};
                t.P = TailCsr<T>{v.P->rp, v.P->ci, v.pv, v.P->rows, (int)v.P->nnz};
            }
            t.dinv = v.dinv;
            t.b = v.b;
            t.x = v.x;
            t.xt = v.xt;
            t.r = v.r;
        }
        ProfScope ps(h, AMG_K_COARSE, tail);
        launch_coarse_tail(ta, h->stream);
        check_launch();
        cur[tail] = level_view(h, tail, (T*)nullptr).xt;
    } else {
        LevelView<T> c = level_view(h, L, (T*)nullptr);
        ProfScope ps(h, AMG_K_COARSE, L);
        launch_dense_matvec(h->nL, h->coarse_inv, c.b, c.x, h->stream);
        check_launch();
        cur[L] = c.x;
    }
    for (int l = down_end - 1; l >= 0; --l) {
        LevelView<T> v = level_view(h, l, (T*)nullptr);
        const T* b = l == 0 ? b0 : v.b;
        row_op_t(h, AMG_K_INTERP, l, kSpmvAdd, *v.P, v.pv, cur[l + 1], cur[l], nullptr, cur[l], nullptr, -1);
        const int dslot = (l == 0) ? dot_slot : -1;
        jacobi_sweeps<T>(h, l, v, b, cur[l], alt[l], post, dslot);
        if (l == 0) {
            if (cur[0] != x0) launch_copy(v.n, x0, cur[0], h->stream);
            if constexpr (sizeof(T) == 8)
                if (post == 0 && dot_slot >= 0) launch_dot(v.n, b0, x0, dot_to(h, dot_slot), h->stream);
        }
    }
}

// V-cycle with hybrid Gauss-Seidel relaxation (FP64): forward sweeps before
// the coarse correction, backward sweeps after it, so the cycle is a
// symmetric preconditioner; guess0 kPrescaled is treated as kZero.  Every
// level runs level by level (the one-workgroup tail is for Jacobi).
void gs_sweeps(amg_ctx* h, int l, const double* b, double*& cur, double*& alt, bool forward, int sweeps) {
    const DevMat& a = h->lv[l].Ah;
    for (int s = 0; s < sweeps; ++s) {
        ProfScope ps(h, AMG_K_JACOBI, l);
        launch_hybrid_gs(forward, a.rows, a.rp, a.ci, a.v, b, cur, alt, h->gs_block, a.view().mean_row, h->stream);
        check_launch();
        std::swap(cur, alt);
    }
}

void vcycle_gs(amg_ctx* h, const double* b0, double* x0, Guess guess0, int dot_slot) {
    const int L = (int)h->lv.size() - 1;
    if (L == 0) {
        ProfScope ps(h, AMG_K_COARSE, 0);
        launch_dense_matvec(h->nL, h->coarse_inv, b0, x0, h->stream);
        check_launch();
        if (dot_slot >= 0) launch_dot(h->lv[0].n, b0, x0, dot_to(h, dot_slot), h->stream);
        return;
    }
    std::vector<double*> cur(L + 1), alt(L + 1);
    for (int l = 0; l < L; ++l) {
        DevLevel& d = h->lv[l];
        const double* b = l == 0 ? b0 : d.b;
        cur[l] = l == 0 ? x0 : d.x;
        alt[l] = d.xt;
        if (l > 0 || guess0 != Guess::kNonzero) launch_fill_f64(d.n, cur[l], 0.0, h->stream);
        gs_sweeps(h, l, b, cur[l], alt[l], true, h->sp.nu_pre);
        row_op(h, AMG_K_RESIDUAL, l, kResid, d.Ah, cur[l], b, nullptr, d.r, nullptr, -1);
        row_op(h, AMG_K_RESTRICT, l, kSpmv, d.R, d.r, nullptr, nullptr, h->lv[l + 1].b, nullptr, -1);
    }
    {
        DevLevel& c = h->lv[L];
        ProfScope ps(h, AMG_K_COARSE, L);
        launch_dense_matvec(h->nL, h->coarse_inv, c.b, c.x, h->stream);
        check_launch();
        cur[L] = c.x;
    }
    for (int l = L - 1; l >= 0; --l) {
        DevLevel& d = h->lv[l];
        const double* b = l == 0 ? b0 : d.b;
        row_op(h, AMG_K_INTERP, l, kSpmvAdd, d.P, cur[l + 1], cur[l], nullptr, cur[l], nullptr, -1);
        gs_sweeps(h, l, b, cur[l], alt[l], false, h->sp.nu_post);
    }
    if (cur[0] != x0) launch_copy(h->lv[0].n, x0, cur[0], h->stream);
    if (dot_slot >= 0) launch_dot(h->lv[0].n, b0, x0, dot_to(h, dot_slot), h->stream);
    check_launch();
}

bool gs_on(const amg_ctx* h) { return h->relax == AMG_RELAX_HYBRID_GS; }

void sell_fp32(amg_ctx* h, DevMat& m);

// FP32 copies of every operator's values, of dinv, and FP32 work vectors
void ensure_fp32(amg_ctx* h) {
    if (h->fp32) return;
    const int L = (int)h->lv.size() - 1;
    for (int l = 0; l <= L; ++l) {
        DevLevel& v = h->lv[l];
        v.A32 = dalloc_n<float>(h, v.A.nnz + kCsrPad);
        v.dinv32 = dalloc_n<float>(h, v.n);
        if (v.Ahs.rp) v.Ahs32 = dalloc_n<float>(h, v.A.nnz + kCsrPad);
        if (l < L) {
            v.P32 = dalloc_n<float>(h, v.P.nnz + kCsrPad);
            v.R32 = dalloc_n<float>(h, v.R.nnz + kCsrPad);
        }
        if (l > 0) {
            v.b32 = dalloc_n<float>(h, v.n);
            v.x32 = dalloc_n<float>(h, v.n);
        }
        v.xt32 = dalloc_n<float>(h, v.n);
        v.r32 = dalloc_n<float>(h, v.n);
    }
    h->cg_r32 = dalloc_n<float>(h, h->lv[0].n);
    h->cg_z32 = dalloc_n<float>(h, h->lv[0].n);
    for (int l = 0; l <= L; ++l) {
        DevLevel& v = h->lv[l];
        sell_fp32(h, v.A);
        if (l < L) sell_fp32(h, v.R);
        if (v.ah_alias) v.Ah = v.A;
        launch_narrow(v.A.nnz, v.A32, v.A.v, h->stream);
        launch_narrow(v.n, v.dinv32, v.dinv, h->stream);
        if (v.Ahs32) launch_narrow(v.A.nnz, v.Ahs32, v.Ahs.v, h->stream);   // capacity; entries past nnz unused
        if (l < L) {
            launch_narrow(v.P.nnz, v.P32, v.P.v, h->stream);
            launch_narrow(v.R.nnz, v.R32, v.R.v, h->stream);
        }
    }
    check_launch();
    h->fp32 = true;
}

// ---------------------------------------------------------------------------
// outer iterations
// ---------------------------------------------------------------------------
void ensure_solve_buffers(amg_ctx* h) {
    const int n = h->lv[0].n;
    if (!h->cg_r) h->cg_r = dalloc_n<double>(h, n);
    if (!h->cg_z) h->cg_z = dalloc_n<double>(h, n);
    if (!h->cg_p) h->cg_p = dalloc_n<double>(h, n);
    if (!h->cg_q) h->cg_q = dalloc_n<double>(h, n);
    if (!h->xw) h->xw = dalloc_n<double>(h, n);
    if (!h->rt) h->rt = dalloc_n<double>(h, n);
}

// Reads the scalar slots into host memory: a one-workgroup kernel writes
// them into the handle's host-coherent buffer and then a sequence number;
// the host polls for that number (a fault or a failed launch ends the wait
// through the stream's status) instead of waiting for a copy and a stream
// synchronization.  Only the slots are guaranteed on return: a caller that
// needs another download complete synchronizes the stream itself.
// The scalar slots as the device holds them once the stream reaches this
// point; with extra, slot S_COUNT of the result holds *extra.
const double* read_scalars(amg_ctx* h, const int* extra = nullptr) {
    const uint32_t seq = ++h->pub_seq;
    launch_publish_scalars(S_COUNT, h->scal, h->pinned_dev, h->flag_dev, seq, extra, h->stream);
    check_launch();
    const uint32_t* flag = h->flag_host;
    for (uint64_t k = 1; __atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq; ++k) {
        if ((k & 4095) != 0) continue;
        const hipError_t e = hipStreamQuery(h->stream);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) throw AmgFailure{AMG_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(e)};
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq)
            throw AmgFailure{AMG_ERR_DEVICE, "scalar readback: the stream finished without publishing"};
    }
    return h->pinned;
}

amg_status do_reintroduce(amg_ctx* h, int s, double gamma_min, int* first) {
    int ls = -1;
    for (int l = 1; l < (int)h->lv.size(); ++l)
        if (h->lv[l].gamma > 0.0) { ls = l; break; }
    if (first) *first = ls;
    if (ls < 0) return AMG_NOTHING_TO_REINTRODUCE;
    std::vector<std::pair<int, double>> todo;
    for (int l = ls; l < (int)h->lv.size(); ++l) {
        if (l < ls + s) {
            double g = h->lv[l].gamma / 10.0;
            if (!(g >= gamma_min)) g = 0.0;
            todo.emplace_back(l, g);
        } else if (h->method == AMG_HYBRID_GALERKIN && h->lv[l].gamma > 0.0) {
            // Hybrid Galerkin: this level's minimal pattern depends on the
            // finer operator just changed, so it is redone at its gamma
            todo.emplace_back(l, h->lv[l].gamma);
        }
    }
    sparsify_levels(h, todo);
    return AMG_OK;
}

// z = V(r, 0) for CG, with r.z accumulated into dot_slot.  Mixed: the cycle
// runs on r32 = (float) r (written by the CG update, or here when the guess is
// kZero) and z = (double) z32.
void precondition(amg_ctx* h, bool mixed, Guess guess, int dot_slot, bool l0_resid_ready = false) {
    const int n = h->lv[0].n;
    if (gs_on(h)) {
        vcycle_gs(h, h->cg_r, h->cg_z, Guess::kZero, dot_slot);
        return;
    }
    if (!mixed) {
        vcycle<double>(h, h->cg_r, h->cg_z, guess, dot_slot, l0_resid_ready);
        return;
    }
    if (guess == Guess::kZero) launch_narrow(n, h->cg_r32, h->cg_r, h->stream);
    vcycle<float>(h, h->cg_r32, h->cg_z32, guess, -1);
    ProfScope ps(h, AMG_K_VECTOR, 0);
    launch_widen_dot(n, h->cg_z, h->cg_z32, h->cg_r, dot_to(h, dot_slot), h->stream);
    check_launch();
}

amg_status solve(amg_ctx* h, const double* b, double* x, const amg_solve_params& p,
                 amg_solve_info* info_out, double* hist) {
    ensure_solve_buffers(h);
    DevLevel& f = h->lv[0];
    const int n = f.n;
    const DevMat& A = f.A;
    const bool pcg = p.method == AMG_PCG;
    // FP32 V-cycle as the preconditioner (PCG) or as the correction of
    // iterative refinement (stationary); everything else stays FP64
    const bool mixed = p.precision == 32;
    if (mixed) ensure_fp32(h);
    amg_solve_info info{0, 0, 0, 0, 0.0, 0.0};
    amg_status st = AMG_ERR_NOT_CONVERGED;
    double* r = h->cg_r;
    launch_fill_f64(S_COUNT, h->scal, 0.0, h->stream);
    if (p.zero_guess) {
        // x0 = 0: r0 = b - A 0 = b
        ProfScope ps(h, AMG_K_VECTOR, 0);
        launch_zero_guess_start(n, b, x, r, dot_to(h, S_NR2), h->stream);
        check_launch();
    } else {
        row_op(h, AMG_K_RESIDUAL, 0, kResidNorm, A, x, b, nullptr, r, nullptr, S_NR2);
    }
    // a pivot flag of the coarsest inversion not read yet comes back with the
    // initial residual norm
    const bool check = h->check_singular;
    const double* sc0 = read_scalars(h, check ? h->singular : nullptr);
    const double nr0 = std::sqrt(sc0[S_NR2]);
    if (check) {
        h->check_singular = false;
        if (sc0[S_COUNT] != 0.0) throw AmgFailure{AMG_ERR_BAD_MATRIX, "coarsest operator is singular"};
    }
    if (hist) hist[0] = nr0;
    double nws = nr0;
    int inwin = 0;
    int rz_slot = S_RZ0;
    double nrf_read = -1.0;   // the final true residual norm, when the loop has read it
    if (!std::isfinite(nr0)) {
        st = AMG_ERR_BREAKDOWN;
    } else if (nr0 == 0.0) {
        info.converged = 1;
        st = AMG_OK;
    } else {
        launch_copy(n, h->xw, x, h->stream);
        if (pcg) {
            precondition(h, mixed, Guess::kZero, rz_slot);
            launch_copy(n, h->cg_p, h->cg_z, h->stream);
        }
        while (info.iters < p.maxit) {
            if (pcg) {
                row_op(h, AMG_K_SPMV_DOT, 0, kSpmvDot, A, h->cg_p, nullptr, nullptr, h->cg_q, nullptr, S_PQ);
                {
                    ProfScope ps(h, AMG_K_VECTOR, 0);
                    // also forms the next preconditioner's zero-guess sweep omega D^-1 r
                    const bool pre1 = h->sp.nu_pre >= 1;
                    launch_cg_update_xr(n, x, r, h->cg_p, h->cg_q, h->scal, rz_slot, S_PQ, h->scal + S_FLAG,
                                        dot_to(h, S_NR2), f.dinv, h->sp.omega,
                                        (!mixed && pre1) ? zero_start<double>(h, 0, h->cg_z) : nullptr,
                                        mixed ? h->cg_r32 : nullptr, f.dinv32,
                                        (mixed && pre1) ? zero_start<float>(h, 0, h->cg_z32) : nullptr,
                                        h->stream);
                    check_launch();
                }
            } else if (mixed) {
                // iterative refinement: x += V32(r, 0) with r the current true residual
                launch_narrow(n, h->cg_r32, r, h->stream);
                vcycle<float>(h, h->cg_r32, h->cg_z32, Guess::kZero, -1);
                launch_add_widened(n, x, h->cg_z32, h->stream);
                row_op(h, AMG_K_RESIDUAL, 0, kResidNorm, A, x, b, nullptr, r, nullptr, S_NR2);
            } else {
                if (gs_on(h)) vcycle_gs(h, b, x, Guess::kNonzero, -1);
                else vcycle<double>(h, b, x, Guess::kNonzero, -1);
                row_op(h, AMG_K_RESIDUAL, 0, kResidNorm, A, x, b, nullptr, r, nullptr, S_NR2);
            }
            // the last iteration of an adaptive window needs the true
            // residual whatever its outcome (for the window test, or as the
            // final residual if it converges): computed before, read back
            // with the iteration's scalars
            const bool window_end = p.adaptive && inwin + 1 == p.k;
            // In the FP64 PCG with one pre-sweep, the next preconditioner's
            // first step is the level-0 residual r - A (omega D^-1 r): it is
            // formed in the same pass over A_0's SELL-64 copy as the true
            // residual (used unless CG restarts).
            bool l0_ready = false;
            if (window_end) {
                DevLevel& f0 = h->lv[0];
                const bool fuse = pcg && !mixed && !gs_on(h) && h->sp.nu_pre == 1 && h->lv.size() > 1 &&
                                  f0.ah_alias && A.sl_off != nullptr;
                if (fuse) {
                    const DotTarget dt = dot_to(h, S_NRT);
                    CsrView cv = A.view();
                    cv.rev = *A.next_rev;
                    *A.next_rev ^= 1;
                    int nparts = 0;
                    {
                        ProfScope ps(h, AMG_K_RESIDUAL, 0, true);
                        nparts = launch_sell_dual_resid(cv, zero_start<double>(h, 0, h->cg_z), r, f0.r, x, b,
                                                        h->rt, dt, h->stream);
                        check_launch();
                    }
                    if (nparts > 0) {
                        launch_dot_finish(dt, nparts, h->stream);
                        check_launch();
                        l0_ready = true;
                    }
                }
                if (!l0_ready) row_op(h, AMG_K_RESIDUAL, 0, kResidNorm, A, x, b, nullptr, h->rt, nullptr, S_NRT);
            }
            const double* sc = read_scalars(h);
            if (pcg && sc[S_FLAG] != 0.0) { st = AMG_ERR_BREAKDOWN; break; }
            const double nr = std::sqrt(sc[S_NR2]);
            info.iters++;
            inwin++;
            if (hist) hist[info.iters] = nr;
            if (!std::isfinite(nr)) { st = AMG_ERR_BREAKDOWN; break; }
            if (nr <= p.rtol * nr0) {
                info.converged = 1;
                st = AMG_OK;
                if (window_end) nrf_read = std::sqrt(sc[S_NRT]);
                break;
            }
            bool restart = false;
            if (window_end) {
                double nrt = std::sqrt(sc[S_NRT]);
                const double rho = std::pow(nrt / nws, 1.0 / (double)p.k);
                bool any = false;
                for (size_t l = 1; l < h->lv.size(); ++l) any = any || h->lv[l].gamma > 0.0;
                if (rho > p.rho_max && any) {
                    int first = -1;
                    amg_status rs = do_reintroduce(h, p.s, p.gamma_min, &first);
                    if (rs < 0) { st = rs; break; }
                    info.reintroductions++;
                    if (nrt > nws) {
                        launch_copy(n, x, h->xw, h->stream);
                        row_op(h, AMG_K_RESIDUAL, 0, kResidNorm, A, x, b, nullptr, r, nullptr, S_NRT);
                        nrt = std::sqrt(read_scalars(h)[S_NRT]);
                    } else {
                        launch_copy(n, r, h->rt, h->stream);
                    }
                    restart = true;
                }
                launch_copy(n, h->xw, x, h->stream);
                nws = nrt;
                inwin = 0;
            }
            if (pcg) {
                const int new_slot = rz_slot == S_RZ0 ? S_RZ1 : S_RZ0;
                // after a restart r was rebuilt, so the prescaled sweep is stale
                precondition(h, mixed, restart ? Guess::kZero : Guess::kPrescaled, new_slot, l0_ready && !restart);
                if (restart) {
                    info.restarts++;
                    launch_copy(n, h->cg_p, h->cg_z, h->stream);
                } else {
                    ProfScope ps(h, AMG_K_VECTOR, 0);
                    launch_cg_update_p(n, h->cg_p, h->cg_z, h->scal, new_slot, rz_slot, h->stream);
                    check_launch();
                }
                rz_slot = new_slot;
            } else if (restart) {
                info.restarts++;
            }
        }
    }
    double nrf = nrf_read;
    if (nrf < 0.0) {
        row_op(h, AMG_K_RESIDUAL, 0, kResidNorm, A, x, b, nullptr, r, nullptr, S_NRT);
        nrf = std::sqrt(read_scalars(h)[S_NRT]);
    }
    info.relres = nr0 > 0.0 ? nrf / nr0 : 0.0;
    info.rho_avg = (info.iters > 0 && info.relres > 0.0) ? std::pow(info.relres, 1.0 / info.iters) : 0.0;
    if (info_out) *info_out = info;
    prof_collect(h);
    return st;
}

// ---------------------------------------------------------------------------
// multiple right-hand sides: the V-cycle applied to an n x K block (K columns
// row-interleaved), iterative refinement with the residual in FP64
// ---------------------------------------------------------------------------
BlockBufs<double>& block_bufs(amg_ctx* h, double*) { return h->blk64; }
BlockBufs<float>& block_bufs(amg_ctx* h, float*) { return h->blk32; }

template <class T>
void free_block_bufs(amg_ctx* h, BlockBufs<T>& bb) {
    for (auto* v : {&bb.b, &bb.x, &bb.xt, &bb.r})
        for (T* p : *v) dfree(h, p);
    bb.b.clear(); bb.x.clear(); bb.xt.clear(); bb.r.clear();
    dfree(h, bb.rhs);
    bb.rhs = nullptr;
    bb.k = 0;
}

// per-level K-wide work blocks of precision T (reallocated for a wider K)
template <class T>
BlockBufs<T>& ensure_block(amg_ctx* h, int k) {
    BlockBufs<T>& bb = block_bufs(h, (T*)nullptr);
    if (!h->blk_partials) h->blk_partials = dalloc_n<double>(h, block_partials_needed());
    if (bb.k >= k) return bb;
    free_block_bufs(h, bb);
    const int L = (int)h->lv.size() - 1;
    bb.b.assign(L + 1, nullptr);
    bb.x.assign(L + 1, nullptr);
    bb.xt.assign(L + 1, nullptr);
    bb.r.assign(L + 1, nullptr);
    for (int l = 0; l <= L; ++l) {
        const int64_t cnt = (int64_t)h->lv[l].n * k;
        if (l > 0) bb.b[l] = dalloc_n<T>(h, cnt);
        bb.x[l] = dalloc_n<T>(h, cnt);
        bb.xt[l] = dalloc_n<T>(h, cnt);
        bb.r[l] = dalloc_n<T>(h, cnt);
        // columns outside the live prefix are never written: keep them finite
        for (T* q : {bb.b[l], bb.x[l], bb.xt[l], bb.r[l]})
            if (q) fill_t(cnt, q, h);
    }
    bb.rhs = dalloc_n<T>(h, (int64_t)h->lv[0].n * k);
    fill_t((int64_t)h->lv[0].n * k, bb.rhs, h);
    bb.k = k;
    return bb;
}

template <class T>
void block_op_t(amg_ctx* h, int kind, int l, BlockOp op, int k, const DevMat& m, const T* vals, const T* g,
                const T* u, const T* dinv, T* y, T* y2, double* acc) {
    ProfScope ps(h, kind, l);
    launch_block_op(op, k, CsrT<T>{m.rp, m.ci, vals, m.rows, 0.0}, g, u, dinv, (T)h->sp.omega, y, y2, acc,
                    h->stream, h->scal + S_LIVE);
    check_launch();
}

ColumnDots cols_to(amg_ctx* h, int slot) { return ColumnDots{h->blk_partials, h->scal + slot}; }

// Where the level-0 result of a block cycle goes: added to the FP64 block acc
// (refinement), or written to zt (cycle precision) with the column dots
// r64 . z (CG; CG widens z exactly where it uses it); neither: left in a
// buffer of the cycle's precision.
template <class T>
struct BlockSink {
    double* acc = nullptr;
    T* zt = nullptr;
    const double* r64 = nullptr;
    ColumnDots dot{};
};

// the preconditioned-residual block of precision T (inside the FP64 z block)
template <class T>
T* block_z(amg_ctx* h) {
    return reinterpret_cast<T*>(h->bcg_z);
}

// One V-cycle on K columns.  guess0: kNonzero -- bb.x[0] holds the iterate;
// kPrescaled -- the iterate is zero and bb.x[0] holds omega D^-1 b0.  The
// last level-0 sweep delivers the result to sink (then nullptr is returned);
// without a sink the buffer holding the result is returned.
template <class T>
T* vcycle_block(amg_ctx* h, int k, const T* b0, Guess guess0, const BlockSink<T>& sink) {
    const bool to_sink = sink.acc || sink.zt;
    BlockBufs<T>& bb = block_bufs(h, (T*)nullptr);
    const int L = (int)h->lv.size() - 1;
    const int pre = h->sp.nu_pre, post = h->sp.nu_post;
    // a level-0 result held in x (precision T) handed to the sink
    auto deliver = [&](const T* x) {
        ProfScope ps(h, AMG_K_VECTOR, 0);
        if (sink.acc) launch_block_accumulate((int64_t)h->lv[0].n * k, sink.acc, x, h->stream);
        else launch_block_copy_dot(h->lv[0].n, k, x, sink.zt, sink.r64, sink.dot, h->stream, h->scal + S_LIVE);
        check_launch();
    };
    if (L == 0) {
        {
            ProfScope ps(h, AMG_K_COARSE, 0);
            launch_block_dense_matvec(h->nL, k, h->coarse_inv, b0, bb.xt[0], h->stream, h->scal + S_LIVE);
            check_launch();
        }
        if (!to_sink) return bb.xt[0];
        deliver(bb.xt[0]);
        return nullptr;
    }
    std::vector<T*> cur(L + 1), alt(L + 1);
    auto sweep = [&](int l, const LevelView<T>& v, const T* b, bool last0) {
        if (last0 && sink.acc) {
            block_op_t<T>(h, AMG_K_JACOBI, l, kBJacobiAccum, k, *v.Ah, v.ahv, cur[l], b, v.dinv, nullptr,
                          nullptr, sink.acc);
        } else if (last0 && sink.zt) {
            ProfScope ps(h, AMG_K_JACOBI, l);
            launch_block_sweep_dot(k, CsrT<T>{v.Ah->rp, v.Ah->ci, v.ahv, v.Ah->rows, 0.0}, cur[l], b, v.dinv,
                                   (T)h->sp.omega, sink.zt, sink.r64, sink.dot, h->stream, h->scal + S_LIVE);
            check_launch();
        } else {
            block_op_t<T>(h, AMG_K_JACOBI, l, kBJacobi, k, *v.Ah, v.ahv, cur[l], b, v.dinv, alt[l], nullptr,
                          nullptr);
            std::swap(cur[l], alt[l]);
        }
    };
    for (int l = 0; l < L; ++l) {
        LevelView<T> v = level_view(h, l, (T*)nullptr);
        const int64_t cnt = (int64_t)v.n * k;
        const T* b = l == 0 ? b0 : bb.b[l];
        cur[l] = bb.x[l];
        alt[l] = bb.xt[l];
        const bool zero = l > 0 || guess0 != Guess::kNonzero;
        if (zero && pre == 0) {
            fill_t(cnt, cur[l], h);
            launch_copy((int)cnt, bb.r[l], b, h->stream);
            check_launch();
        } else {
            // a zero iterate arrives with its first sweep already formed
            for (int s = zero ? 1 : 0; s < pre; ++s) sweep(l, v, b, false);
            const int kind = (zero && pre == 1) ? AMG_K_JACOBI_ZERO : AMG_K_RESIDUAL;
            block_op_t<T>(h, kind, l, kBResid, k, *v.Ah, v.ahv, cur[l], b, nullptr, bb.r[l], nullptr, nullptr);
        }
        LevelView<T> nx = level_view(h, l + 1, (T*)nullptr);
        if (pre >= 1 && l + 1 < L)
            block_op_t<T>(h, AMG_K_RESTRICT, l, kBSpmvScale, k, *v.R, v.rv, bb.r[l], nullptr, nx.dinv, bb.b[l + 1],
                          bb.x[l + 1], nullptr);
        else
            block_op_t<T>(h, AMG_K_RESTRICT, l, kBSpmv, k, *v.R, v.rv, bb.r[l], nullptr, nullptr, bb.b[l + 1],
                          nullptr, nullptr);
    }
    {
        ProfScope ps(h, AMG_K_COARSE, L);
        launch_block_dense_matvec(h->nL, k, h->coarse_inv, bb.b[L], bb.x[L], h->stream, h->scal + S_LIVE);
        check_launch();
        cur[L] = bb.x[L];
    }
    for (int l = L - 1; l >= 0; --l) {
        LevelView<T> v = level_view(h, l, (T*)nullptr);
        const T* b = l == 0 ? b0 : bb.b[l];
        block_op_t<T>(h, AMG_K_INTERP, l, kBSpmvAdd, k, *v.P, v.pv, cur[l + 1], cur[l], nullptr, cur[l], nullptr,
                      nullptr);
        for (int s = 0; s < post; ++s) sweep(l, v, b, l == 0 && to_sink && s == post - 1);
    }
    if (!to_sink) return cur[0];
    if (post == 0) deliver(cur[0]);
    return nullptr;
}

// outer residual r = b - A_0 x (FP64) of all K columns into bb.rhs (precision
// T) with the next cycle's first sweep omega D^-1 r in bb.x[0] (and r itself
// into r64 when not null); squared column norms into the slots S_BLOCK..
template <class T>
void block_outer(amg_ctx* h, int k, const double* b, const double* x, double* r64 = nullptr) {
    BlockBufs<T>& bb = block_bufs(h, (T*)nullptr);
    DevLevel& f = h->lv[0];
    LevelView<T> v = level_view(h, 0, (T*)nullptr);
    ProfScope ps(h, AMG_K_RESIDUAL, 0);
    launch_block_outer_residual(k, f.A.view(), x, b, v.dinv, (T)h->sp.omega, bb.rhs, bb.x[0], r64,
                                cols_to(h, S_BLOCK), h->stream, h->scal + S_LIVE);
    check_launch();
}

// Iterative refinement x_c += V(b_c - A x_c, 0) on all K columns together;
// nrhs columns are real (the others are zero padding).
template <class T>
amg_status solve_block(amg_ctx* h, int k, int nrhs, const double* b, double* x, const amg_solve_params& p,
                       amg_solve_info* info_out, int32_t* col_iters, double* col_relres) {
    if constexpr (sizeof(T) == 4) ensure_fp32(h);
    BlockBufs<T>& bb = ensure_block<T>(h, k);
    amg_solve_info info{0, 0, 0, 0, 0.0, 0.0};
    amg_status st = AMG_ERR_NOT_CONVERGED;
    launch_fill_f64(S_COUNT, h->scal, 0.0, h->stream);
    launch_fill_f64(1, h->scal + S_LIVE, (double)nrhs, h->stream);
    block_outer<T>(h, k, b, x);
    const bool check = h->check_singular;
    const double* sc = read_scalars(h, check ? h->singular : nullptr);
    if (check) {
        h->check_singular = false;
        if (sc[S_COUNT] != 0.0) throw AmgFailure{AMG_ERR_BAD_MATRIX, "coarsest operator is singular"};
    }
    double nr0[kMaxBlockRhs], rel[kMaxBlockRhs];
    int first[kMaxBlockRhs];
    bool finite = true;
    for (int c = 0; c < nrhs; ++c) {
        nr0[c] = std::sqrt(sc[S_BLOCK + c]);
        finite = finite && std::isfinite(nr0[c]);
        rel[c] = 1.0;
        first[c] = nr0[c] == 0.0 ? 0 : -1;
        if (nr0[c] == 0.0) rel[c] = 0.0;
    }
    auto all_done = [&] {
        for (int c = 0; c < nrhs; ++c)
            if (first[c] < 0) return false;
        return true;
    };
    if (!finite) {
        st = AMG_ERR_BREAKDOWN;
    } else if (all_done()) {
        st = AMG_OK;
        info.converged = 1;
    } else {
        while (info.iters < p.maxit) {
            BlockSink<T> sink;
            sink.acc = x;
            vcycle_block<T>(h, k, bb.rhs, Guess::kPrescaled, sink);
            block_outer<T>(h, k, b, x);
            sc = read_scalars(h);
            info.iters++;
            bool bad = false;
            for (int c = 0; c < nrhs; ++c) {
                const double nr = std::sqrt(sc[S_BLOCK + c]);
                bad = bad || !std::isfinite(nr);
                if (nr0[c] > 0.0) rel[c] = nr / nr0[c];
                if (first[c] < 0 && nr <= p.rtol * nr0[c]) first[c] = info.iters;
            }
            if (bad) { st = AMG_ERR_BREAKDOWN; break; }
            if (all_done()) { st = AMG_OK; info.converged = 1; break; }
        }
    }
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        worst = std::max(worst, rel[c]);
        if (col_iters) col_iters[c] = first[c];
        if (col_relres) col_relres[c] = rel[c];
    }
    info.relres = worst;
    info.rho_avg = (info.iters > 0 && worst > 0.0) ? std::pow(worst, 1.0 / info.iters) : 0.0;
    if (info_out) *info_out = info;
    prof_collect(h);
    return st;
}

void ensure_block_cg(amg_ctx* h, int k) {
    if (h->bcg_k >= k) return;
    for (double** q : {&h->bcg_r, &h->bcg_p, &h->bcg_q, &h->bcg_z}) {
        dfree(h, *q);
        *q = nullptr;
    }
    const int64_t cnt = (int64_t)h->lv[0].n * k;
    h->bcg_r = dalloc_n<double>(h, cnt);
    h->bcg_p = dalloc_n<double>(h, cnt);
    h->bcg_q = dalloc_n<double>(h, cnt);
    h->bcg_z = dalloc_n<double>(h, cnt);
    for (double* q : {h->bcg_r, h->bcg_p, h->bcg_q, h->bcg_z}) launch_fill_f64(cnt, q, 0.0, h->stream);
    h->bcg_k = k;
}

// per-column active flags (1 = still iterating) to the device, staged in the
// pinned buffer (read_scalars later reads the same values back)
void upload_active(amg_ctx* h, const bool* active, int k) {
    for (int c = 0; c < k; ++c) h->pinned[S_BACT + c] = active[c] ? 1.0 : 0.0;
    HIP_CHECK(hipMemcpyAsync(h->scal + S_BACT, h->pinned + S_BACT, sizeof(double) * k, hipMemcpyHostToDevice,
                             h->stream));
}

// Preconditioned CG on every column at once (Section 5 PCG with the Section 2
// V-cycle as preconditioner): the FP64 iterates and column scalars stay on the
// device; one cycle of precision T and one FP64 product A p per iteration
// serve all columns.  A column stops changing once it meets the tolerance.
template <class T>
amg_status solve_block_pcg(amg_ctx* h, int k, int nrhs, const double* b, double* x, const amg_solve_params& p,
                           amg_solve_info* info_out, int32_t* col_iters, double* col_relres) {
    if constexpr (sizeof(T) == 4) ensure_fp32(h);
    BlockBufs<T>& bb = ensure_block<T>(h, k);
    ensure_block_cg(h, k);
    DevLevel& f = h->lv[0];
    const int n = f.n;
    LevelView<T> v0 = level_view(h, 0, (T*)nullptr);
    const T omega = (T)h->sp.omega;
    amg_solve_info info{0, 0, 0, 0, 0.0, 0.0};
    amg_status st = AMG_ERR_NOT_CONVERGED;
    launch_fill_f64(S_COUNT, h->scal, 0.0, h->stream);
    launch_fill_f64(1, h->scal + S_LIVE, (double)nrhs, h->stream);
    block_outer<T>(h, k, b, x, h->bcg_r);
    const bool check = h->check_singular;
    const double* sc = read_scalars(h, check ? h->singular : nullptr);
    if (check) {
        h->check_singular = false;
        if (sc[S_COUNT] != 0.0) throw AmgFailure{AMG_ERR_BAD_MATRIX, "coarsest operator is singular"};
    }
    double nr0[kMaxBlockRhs], rel[kMaxBlockRhs];
    int first[kMaxBlockRhs];
    bool active[kMaxBlockRhs] = {};
    bool finite = true;
    int nactive = 0;
    for (int c = 0; c < nrhs; ++c) {
        nr0[c] = std::sqrt(sc[S_BLOCK + c]);
        finite = finite && std::isfinite(nr0[c]);
        first[c] = nr0[c] == 0.0 ? 0 : -1;
        rel[c] = nr0[c] == 0.0 ? 0.0 : 1.0;
        active[c] = nr0[c] > 0.0;
        nactive += active[c];
    }
    auto precondition = [&](int slot) {
        BlockSink<T> sink;
        sink.zt = block_z<T>(h);
        sink.r64 = h->bcg_r;
        sink.dot = cols_to(h, slot);
        vcycle_block<T>(h, k, bb.rhs, Guess::kPrescaled, sink);
    };
    if (!finite) {
        st = AMG_ERR_BREAKDOWN;
    } else if (nactive == 0) {
        st = AMG_OK;
        info.converged = 1;
    } else {
        upload_active(h, active, k);
        int rz = S_BRZ0;
        precondition(rz);
        launch_block_cg_update_p(n, k, h->bcg_p, block_z<T>(h), h->scal, rz, rz, S_BACT, -1, true, h->stream,
                                 h->scal + S_LIVE);
        check_launch();
        while (info.iters < p.maxit) {
            {
                ProfScope ps(h, AMG_K_SPMV_DOT, 0);
                launch_block_spmv_dot(k, f.A.view(), h->bcg_p, h->bcg_q, cols_to(h, S_BPQ), h->stream,
                                      h->scal + S_LIVE);
                check_launch();
            }
            {
                ProfScope ps(h, AMG_K_VECTOR, 0);
                launch_block_cg_update_xr(n, k, x, h->bcg_r, h->bcg_p, h->bcg_q, h->scal, rz, S_BPQ, S_BACT,
                                          h->scal + S_BFLAG, v0.dinv, omega, bb.rhs, bb.x[0],
                                          cols_to(h, S_BLOCK), h->stream, h->scal + S_LIVE);
                check_launch();
            }
            sc = read_scalars(h);
            info.iters++;
            bool bad = false, changed = false;
            for (int c = 0; c < nrhs; ++c) bad = bad || sc[S_BFLAG + c] != 0.0;
            if (bad) { st = AMG_ERR_BREAKDOWN; break; }
            for (int c = 0; c < nrhs; ++c) {
                if (!active[c]) continue;
                const double nr = std::sqrt(sc[S_BLOCK + c]);
                bad = bad || !std::isfinite(nr);
                rel[c] = nr / nr0[c];
                if (nr <= p.rtol * nr0[c]) {
                    first[c] = info.iters;
                    active[c] = false;
                    changed = true;
                    --nactive;
                }
            }
            if (bad) { st = AMG_ERR_BREAKDOWN; break; }
            if (nactive == 0) { st = AMG_OK; info.converged = 1; break; }
            if (changed) upload_active(h, active, k);
            const int next = rz == S_BRZ0 ? S_BRZ1 : S_BRZ0;
            precondition(next);
            {
                ProfScope ps(h, AMG_K_VECTOR, 0);
                launch_block_cg_update_p(n, k, h->bcg_p, block_z<T>(h), h->scal, next, rz, S_BACT, -1, false,
                                         h->stream, h->scal + S_LIVE);
                check_launch();
            }
            rz = next;
        }
    }
    // final true residual of every column
    if (info.iters > 0) {
        block_outer<T>(h, k, b, x);
        sc = read_scalars(h);
        for (int c = 0; c < nrhs; ++c)
            if (nr0[c] > 0.0) rel[c] = std::sqrt(sc[S_BLOCK + c]) / nr0[c];
    }
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        worst = std::max(worst, rel[c]);
        if (col_iters) col_iters[c] = first[c];
        if (col_relres) col_relres[c] = rel[c];
    }
    info.relres = worst;
    info.rho_avg = (info.iters > 0 && worst > 0.0) ? std::pow(worst, 1.0 / info.iters) : 0.0;
    if (info_out) *info_out = info;
    prof_collect(h);
    return st;
}

// ---------------------------------------------------------------------------
// continuous batching: slots of a block PCG that start and finish on their
// own while the other slots keep iterating
// ---------------------------------------------------------------------------
enum SlotState : int { kSlotFree = 0, kSlotPending = 1, kSlotActive = 2, kSlotDone = 3 };

// device bytes of the FP32 copies ensure_fp32 allocates
int64_t fp32_mirror_bytes(const amg_ctx* h) {
    const int L = (int)h->lv.size() - 1;
    int64_t b = 0;
    for (int l = 0; l <= L; ++l) {
        const DevLevel& v = h->lv[l];
        b += 4 * (v.A.nnz + kCsrPad) + 4 * (int64_t)v.n;
        if (v.Ahs.rp) b += 4 * (v.A.nnz + kCsrPad);
        if (l < L) b += 4 * (v.P.nnz + kCsrPad) + 4 * (v.R.nnz + kCsrPad);
        b += 4 * (int64_t)v.n * (l > 0 ? 4 : 2);
    }
    return b + 8 * (int64_t)h->lv[0].n;
}

// device bytes a batch of k slots allocates beyond the hierarchy
int64_t batch_bytes(const amg_ctx* h, int k, int precision) {
    const int64_t vs = precision == 32 ? 4 : 8;
    const int64_t n0 = h->lv[0].n;
    int64_t b = 6 * 8 * n0 * k;                          // B, X and the CG vectors r, p, q, z
    for (size_t l = 0; l < h->lv.size(); ++l)
        b += vs * k * (int64_t)h->lv[l].n * (l > 0 ? 4 : 3);   // cycle blocks b, x, xt, r
    b += vs * k * n0 + 8 * (int64_t)block_partials_needed();
    if (precision == 32 && !h->fp32) b += fp32_mirror_bytes(h);
    return b;
}

}  // namespace

struct amg_batch_ctx {
    amg_ctx* h = nullptr;
    int k = 0, precision = 32, maxit = 0;
    double rtol = 0.0;
    bool graphs = false;          // replay captured iterations
    // one captured iteration per (r.z slot parity, with / without loads)
    hipGraph_t graph[2][2] = {};
    hipGraphExec_t exec[2][2] = {};
    double* B = nullptr;          // n x k right-hand sides of the slots
    double* X = nullptr;          // n x k iterates
    double* down = nullptr;       // pinned: the scalar slots after the last step
    double* up = nullptr;         // pinned: active flags [0, 16), load flags [16, 32), live columns [32]
    hipEvent_t done = nullptr;
    bool in_flight = false;
    int rz = S_BRZ0;
    int state[kMaxBlockRhs] = {};
    int iters[kMaxBlockRhs] = {};
    int status[kMaxBlockRhs] = {};
    bool loaded[kMaxBlockRhs] = {};   // started by the step in flight
    double nr0[kMaxBlockRhs] = {};
    double rel[kMaxBlockRhs] = {};
};

namespace {

// One PCG iteration of every active slot from r.z slot `rz` to `next`; with
// `load` the submitted slots start in it (x = 0, r = b, fresh direction).
template <class T>
void batch_iteration(amg_batch_ctx* e, bool load, int rz, int next) {
    amg_ctx* h = e->h;
    const int k = e->k;
    BlockBufs<T>& bb = block_bufs(h, (T*)nullptr);
    DevLevel& f = h->lv[0];
    const int n = f.n;
    LevelView<T> v0 = level_view(h, 0, (T*)nullptr);
    const T omega = (T)h->sp.omega;
    const int i_load = load ? S_BLOAD : -1;
    if (load) {
        ProfScope ps(h, AMG_K_VECTOR, 0);
        launch_block_load_columns(n, k, h->scal, S_BLOAD, e->B, e->X, h->bcg_r, v0.dinv, omega, bb.rhs, bb.x[0],
                                  cols_to(h, S_BNEW), h->stream);
        check_launch();
    }
    BlockSink<T> sink;
    sink.zt = block_z<T>(h);
    sink.r64 = h->bcg_r;
    sink.dot = cols_to(h, next);
    vcycle_block<T>(h, k, bb.rhs, Guess::kPrescaled, sink);
    {
        ProfScope ps(h, AMG_K_VECTOR, 0);
        launch_block_cg_update_p(n, k, h->bcg_p, block_z<T>(h), h->scal, next, rz, S_BACT, i_load, false,
                                 h->stream, h->scal + S_LIVE);
        check_launch();
    }
    {
        ProfScope ps(h, AMG_K_SPMV_DOT, 0);
        launch_block_spmv_dot(k, f.A.view(), h->bcg_p, h->bcg_q, cols_to(h, S_BPQ), h->stream, h->scal + S_LIVE);
        check_launch();
    }
    {
        ProfScope ps(h, AMG_K_VECTOR, 0);
        launch_block_cg_update_xr(n, k, e->X, h->bcg_r, h->bcg_p, h->bcg_q, h->scal, next, S_BPQ, S_BACT,
                                  h->scal + S_BFLAG, v0.dinv, omega, bb.rhs, bb.x[0], cols_to(h, S_BLOCK),
                                  h->stream, h->scal + S_LIVE);
        launch_block_converge(k, h->scal, S_BACT, S_BLOCK, S_BNR0, S_BFLAG, S_BITER, S_BSTAT, S_BREL, i_load,
                              S_BNEW, e->rtol, e->maxit, h->stream);
        check_launch();
    }
}

// the captured form of batch_iteration(load, rz, next), made on first use
template <class T>
hipGraphExec_t batch_graph(amg_batch_ctx* e, bool load, int rz, int next) {
    const int par = rz == S_BRZ0 ? 0 : 1;
    hipGraphExec_t& ex = e->exec[par][load ? 1 : 0];
    if (ex) return ex;
    hipGraph_t& g = e->graph[par][load ? 1 : 0];
    hipStream_t st = e->h->stream;
    HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
        batch_iteration<T>(e, load, rz, next);
    } catch (...) {
        hipGraph_t partial = nullptr;
        (void)hipStreamEndCapture(st, &partial);
        if (partial) (void)hipGraphDestroy(partial);
        throw;
    }
    HIP_CHECK(hipStreamEndCapture(st, &g));
    HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    return ex;
}

// Enqueues `iters` PCG iterations of every active slot, the slots submitted
// since the last step starting in the first one.  Each iteration ends with
// the device-side stop test, so a slot stops at exactly its own convergence
// iteration however many iterations a step holds.
template <class T>
void batch_step(amg_batch_ctx* e, int iters) {
    amg_ctx* h = e->h;
    const int k = e->k;
    bool any_load = false;
    int live = 0;
    for (int c = 0; c < kMaxBlockRhs; ++c) {
        e->loaded[c] = c < k && e->state[c] == kSlotPending;
        if (e->loaded[c]) {
            e->state[c] = kSlotActive;
            e->iters[c] = 0;
            any_load = true;
        }
        const bool act = c < k && e->state[c] == kSlotActive;
        if (act) live = c + 1;
        e->up[c] = act ? 1.0 : 0.0;
        e->up[kMaxBlockRhs + c] = e->loaded[c] ? 1.0 : 0.0;
    }
    // slots past the last iterating one are not computed
    e->up[2 * kMaxBlockRhs] = (double)live;
    static_assert(S_BLOAD == S_BACT + kMaxBlockRhs && S_LIVE == S_BLOAD + kMaxBlockRhs, "slot layout");
    HIP_CHECK(hipMemcpyAsync(h->scal + S_BACT, e->up, sizeof(double) * (2 * kMaxBlockRhs + 1), hipMemcpyHostToDevice,
                             h->stream));
    launch_fill_f64(k, h->scal + S_BFLAG, 0.0, h->stream);
    // graphs replay the same launches; event timing needs them issued one by one
    const bool graphs = e->graphs && !h->profiling;
    for (int it = 0; it < iters; ++it) {
        const bool load = it == 0 && any_load;
        const int next = e->rz == S_BRZ0 ? S_BRZ1 : S_BRZ0;
        if (graphs) HIP_CHECK(hipGraphLaunch(batch_graph<T>(e, load, e->rz, next), h->stream));
        else batch_iteration<T>(e, load, e->rz, next);
        e->rz = next;
    }
    HIP_CHECK(hipMemcpyAsync(e->down, h->scal, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, h->stream));
    HIP_CHECK(hipEventRecord(e->done, h->stream));
    e->in_flight = true;
}

// slot bookkeeping after a completed step, from the states the device wrote
void batch_finish_step(amg_batch_ctx* e, int32_t* finished) {
    const double* sc = e->down;
    for (int c = 0; c < e->k; ++c) {
        if (finished) finished[c] = 0;
        if (e->state[c] != kSlotActive) continue;
        e->iters[c] = (int)sc[S_BITER + c];
        e->rel[c] = sc[S_BREL + c];
        if (sc[S_BACT + c] != 0.0) continue;
        const int st = (int)sc[S_BSTAT + c];
        e->status[c] = st == 1 ? AMG_OK : st == 2 ? AMG_ERR_NOT_CONVERGED : AMG_ERR_BREAKDOWN;
        e->state[c] = kSlotDone;
        if (finished) finished[c] = 1;
    }
    e->in_flight = false;
}

void destroy_batch(amg_batch_ctx* e) {
    if (!e) return;
    amg_ctx* h = e->h;
    if (h) {
        (void)hipStreamSynchronize(h->stream);
        dfree(h, e->B);
        dfree(h, e->X);
        // the block work space goes with the batch, so that its bytes are free again
        free_block_bufs(h, h->blk64);
        free_block_bufs(h, h->blk32);
        for (double** q : {&h->bcg_r, &h->bcg_p, &h->bcg_q, &h->bcg_z}) {
            dfree(h, *q);
            *q = nullptr;
        }
        h->bcg_k = 0;
        dfree(h, h->blk_partials);
        h->blk_partials = nullptr;
        h->batch = nullptr;
    }
    for (int p = 0; p < 2; ++p)
        for (int l = 0; l < 2; ++l) {
            if (e->exec[p][l]) (void)hipGraphExecDestroy(e->exec[p][l]);
            if (e->graph[p][l]) (void)hipGraphDestroy(e->graph[p][l]);
        }
    if (e->down) (void)hipHostFree(e->down);
    if (e->up) (void)hipHostFree(e->up);
    if (e->done) (void)hipEventDestroy(e->done);
    delete e;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
void finish_setup(amg_ctx* h);

void setup(amg_ctx* h, int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
           const std::vector<double>& nongalerkin_gamma) {
    HostCsr a;
    a.rows = a.cols = (int)n;
    if (row_ptr[0] != 0 || row_ptr[n] < 0) throw AmgFailure{AMG_ERR_BAD_MATRIX, "row_ptr must start at 0"};
    for (int64_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) throw AmgFailure{AMG_ERR_BAD_MATRIX, "row_ptr is not non-decreasing"};
    const int64_t nnz = row_ptr[n];
    a.ptr.assign(row_ptr, row_ptr + n + 1);
    a.idx.assign(col, col + nnz);
    a.val.assign(val, val + nnz);
    std::string why;
    if (!check_input_matrix(a, why)) throw AmgFailure{AMG_ERR_BAD_MATRIX, why};
    SetupConfig cfg;
    cfg.theta = h->sp.theta;
    cfg.max_coarse = h->sp.max_coarse;
    cfg.max_levels = h->sp.max_levels;
    cfg.nongalerkin_gamma = nongalerkin_gamma;
    h->nongalerkin = !nongalerkin_gamma.empty();
    std::vector<HostLevel> hl;
    if (!build_galerkin_hierarchy(a, cfg, hl, why)) throw AmgFailure{AMG_ERR_BAD_MATRIX, why};
    if (hl.back().A.rows > kMaxDenseCoarse)
        throw AmgFailure{AMG_ERR_INVALID_ARG, "coarsest level has " + std::to_string(hl.back().A.rows) +
                                                  " rows; the dense coarse solve allows at most " +
                                                  std::to_string(kMaxDenseCoarse)};
    const int L = (int)hl.size() - 1;
    h->lv.resize(hl.size());
    for (int l = 0; l <= L; ++l) {
        DevLevel& d = h->lv[l];
        HostLevel& s = hl[l];
        d.n = s.A.rows;
        d.A = upload_mat(h, s.A);
        if (l < L) {
            d.P = upload_mat(h, s.P);
            d.R = upload_mat(h, s.R);
            d.nc = (int)s.c_points.size();
            d.c_points = dalloc_n<int32_t>(h, d.nc);
            upload(h, d.c_points, s.c_points.data(), d.nc);
            d.split = s.split;
        }
    }
    finish_setup(h);
}

// 16-bit column indices of a fixed matrix the LDS-staged kernels run on, if
// the columns of every row block of the launch span at most 65535 (a cut of
// 2 of the 12 bytes each entry moves)
void drop_indices(amg_ctx* h, DevMat& m) {
    dfree(h, m.ci16);
    dfree(h, m.cbase);
    m.ci16 = nullptr;
    m.cbase = nullptr;
    m.idx_rb = 0;
}

void compress_indices(amg_ctx* h, DevMat& m) {
    if (!h->compact_idx || m.ci16 || m.nnz <= 0) return;
    const int rb = stream_block_rows(m.view());
    if (rb == 0) return;
    const int nblk = (m.rows + rb - 1) / rb;
    m.ci16 = dalloc_n<uint16_t>(h, m.nnz + kCsrPad);
    m.cbase = dalloc_n<int32_t>(h, nblk);
    m.idx_rb = rb;
    int* wide = h->missing;
    launch_fill_u32(1, reinterpret_cast<unsigned*>(wide), 0u, h->stream);
    launch_compress_index(m.rows, rb, m.rp, m.ci, m.ci16, m.cbase, wide, h->stream);
    check_launch();
    int nwide = 0;
    download(h, &nwide, wide, 1);
    sync(h);
    if (nwide > 0) drop_indices(h, m);
}

// SELL-64 copy of a large operator with short rows, kept if its padding
// adds at most a tenth to the stored entries (structured stencils: a few
// percent; interpolation operators, whose C and F rows alternate, not)
constexpr double kSellMaxPadding = 0.10;

void build_sell(amg_ctx* h, DevMat& m) {
    if (m.sl_off || m.nnz <= 0 || !sell_candidate(m.view())) return;
    const int ns = sell_slices(m.rows);
    int32_t* off = dalloc_n<int32_t>(h, ns + 1);
    launch_sell_widths(m.rows, m.rp, h->cnt, h->stream);
    launch_exclusive_scan(ns, h->cnt, off, h->scan_scratch, h->stream);
    check_launch();
    int32_t total = 0;
    download(h, &total, off + ns, 1);
    sync(h);
    if ((double)total > (1.0 + kSellMaxPadding) * (double)m.nnz) {
        dfree(h, off);
        return;
    }
    std::vector<int32_t> offs(ns + 1);
    download(h, offs.data(), off, ns + 1);
    sync(h);
    int maxw = 0;
    for (int s = 0; s < ns; ++s) maxw = std::max(maxw, (offs[s + 1] - offs[s]) / 64);
    m.sl_off = off;
    m.sl_col = dalloc_n<int32_t>(h, total);
    m.sl_val = dalloc_n<double>(h, total);
    m.sl_maxw = maxw;
    m.sl_cap = total;
    launch_sell_fill(m.rows, m.rp, m.ci, m.v, off, m.sl_col, m.sl_val, h->stream);
    check_launch();
    if (!h->compact_idx) return;
    // square operators whose every slice has at most 64 distinct offsets
    // column - row (stencil-like operators): 8-bit positions in a table of
    // offsets per slice; then the 32-bit columns go
    if (m.rows == m.cols) {
        m.sl_idx8 = dalloc_n<uint8_t>(h, total);
        m.sl_tab = dalloc_n<int32_t>(h, (int64_t)ns * 64);
        launch_fill_u32(1, reinterpret_cast<unsigned*>(h->missing), 0u, h->stream);
        launch_sell_dictionary(m.rows, off, m.sl_col, m.sl_idx8, m.sl_tab, h->missing, h->stream);
        check_launch();
        int over = 0;
        download(h, &over, h->missing, 1);
        sync(h);
        if (over == 0) {
            dfree(h, m.sl_col);
            m.sl_col = nullptr;
            return;
        }
        dfree(h, m.sl_idx8);
        dfree(h, m.sl_tab);
        m.sl_idx8 = nullptr;
        m.sl_tab = nullptr;
    }
    // 16-bit offsets from a base per slice where every slice's columns span
    // at most 65535 (banded operators); then the 32-bit columns go
    m.sl_col16 = dalloc_n<uint16_t>(h, total);
    m.sl_base = dalloc_n<int32_t>(h, ns);
    launch_fill_u32(1, reinterpret_cast<unsigned*>(h->missing), 0u, h->stream);
    launch_sell_compress(m.rows, off, m.sl_col, m.sl_col16, m.sl_base, h->missing, h->stream);
    check_launch();
    int nwide = 0;
    download(h, &nwide, h->missing, 1);
    sync(h);
    if (nwide > 0) {
        dfree(h, m.sl_col16);
        dfree(h, m.sl_base);
        m.sl_col16 = nullptr;
        m.sl_base = nullptr;
    } else {
        dfree(h, m.sl_col);
        m.sl_col = nullptr;
    }
}

void drop_sell(amg_ctx* h, DevMat& m) {
    for (void* p : {(void*)m.sl_off, (void*)m.sl_col, (void*)m.sl_val, (void*)m.sl_col16, (void*)m.sl_base,
                    (void*)m.sl_idx8, (void*)m.sl_tab, (void*)m.sl_val32})
        dfree(h, p);
    m.sl_off = m.sl_col = m.sl_base = m.sl_tab = nullptr;
    m.sl_val = nullptr;
    m.sl_val32 = nullptr;
    m.sl_cap = 0;
    m.sl_col16 = nullptr;
    m.sl_idx8 = nullptr;
    m.sl_maxw = 0;
}

// FP32 values of a SELL-64 copy, for the FP32 cycle
void sell_fp32(amg_ctx* h, DevMat& m) {
    if (!m.sl_off || m.sl_val32) return;
    m.sl_val32 = dalloc_n<float>(h, m.sl_cap);
    launch_narrow(m.sl_cap, m.sl_val32, m.sl_val, h->stream);
    check_launch();
}

// builds or drops the 16-bit indices of every level's A, P and R (the
// sparsified operators keep 32-bit indices)
void set_compact_indices(amg_ctx* h, bool on) {
    h->compact_idx = on;
    for (auto& d : h->lv) {
        for (DevMat* m : {&d.A, &d.P, &d.R}) {
            if (!m->rp) continue;
            if (on) compress_indices(h, *m);
            else drop_indices(h, *m);
            if (m->sl_off && (m->sl_col == nullptr) != on) {
                // rebuilt in the other column width
                drop_sell(h, *m);
                build_sell(h, *m);
                if (h->fp32) sell_fp32(h, *m);
            }
        }
        if (d.ah_alias) d.Ah = d.A;
    }
}

// everything a hierarchy needs once its levels hold A, P, R, c_points and
// the split: 1/diag, work vectors, reduction and scan buffers, the coarsest
// inverse
void finish_setup(amg_ctx* h) {
    const int L = (int)h->lv.size() - 1;
    const int64_t n = h->lv[0].n;
    int partial_need = vector_launch_blocks(std::max(1, (int)n));
    h->missing = dalloc_n<int>(h, 1);
    h->singular = dalloc_n<int>(h, 1);
    int nmax = 0;
    for (auto& d : h->lv) nmax = std::max(nmax, d.n);
    h->cnt = dalloc_n<int32_t>(h, nmax + 1);
    h->scan_scratch = dalloc_n<int32_t>(h, scan_scratch_ints(nmax));
    {
        int64_t ncnt = 0, nbsum = 0;
        // block counts at 64 lanes a row (the most blocks any width gives), so
        // that a level fits whether it runs alone or merged with others
        for (auto& d : h->lv) {
            ncnt += d.n + 1;
            nbsum += keep_count_blocks(64, d.n) + 1;
        }
        h->sp_cnt = dalloc_n<int32_t>(h, ncnt);
        h->sp_bsum = dalloc_n<int32_t>(h, nbsum);
        ncnt = nbsum = 0;
        for (auto& d : h->lv) {
            d.kcnt = h->sp_cnt + ncnt;
            d.kbsum = h->sp_bsum + nbsum;
            ncnt += d.n + 1;
            nbsum += keep_count_blocks(64, d.n) + 1;
        }
    }
    for (int l = 0; l <= L; ++l) {
        DevLevel& d = h->lv[l];
        compress_indices(h, d.A);
        build_sell(h, d.A);
        if (l < L) {
            compress_indices(h, d.P);
            compress_indices(h, d.R);
            build_sell(h, d.R);
        }
        d.Ah = d.A;
        d.ah_alias = true;
        d.dinv = dalloc_n<double>(h, d.n);
        launch_inverse_diagonal(d.A.view(), d.dinv, nullptr, h->stream);
        partial_need = std::max(partial_need, row_launch_blocks(d.n, d.A.width));
        if (l < L) {
            partial_need = std::max(partial_need, row_launch_blocks(d.P.rows, d.P.width));
            partial_need = std::max(partial_need, row_launch_blocks(d.R.rows, d.R.width));
        }
        if (l > 0) d.b = dalloc_n<double>(h, d.n);
        if (l > 0) d.x = dalloc_n<double>(h, d.n);
        d.xt = dalloc_n<double>(h, d.n);
        d.r = dalloc_n<double>(h, d.n);
    }
    // sparsified-operator widths are chosen per build; partial buffers cover
    // every width for the largest level
    partial_need = std::max(partial_need, max_row_launch_blocks());
    h->partial_cap = partial_need;
    h->partials = dalloc_n<double>(h, partial_need);
    h->scal = dalloc_n<double>(h, S_COUNT);
    launch_fill_f64(S_COUNT, h->scal, 0.0, h->stream);
    check_launch();
    // the scalar slots, then the readback's sequence word, host-coherent so
    // that the device's writes reach the host without a copy
    HIP_CHECK(hipHostMalloc((void**)&h->pinned, sizeof(double) * (S_COUNT + 1) + 64,
                            hipHostMallocCoherent | hipHostMallocMapped));
    h->flag_host = reinterpret_cast<uint32_t*>(h->pinned + S_COUNT + 1);
    *h->flag_host = 0;
    HIP_CHECK(hipHostGetDevicePointer((void**)&h->pinned_dev, h->pinned, 0));
    h->flag_dev = reinterpret_cast<uint32_t*>(h->pinned_dev + S_COUNT + 1);
    sync(h);
    refresh_coarse_inverse(h);
    h->prof.assign((size_t)AMG_K_NUM * h->lv.size(), ProfAcc{});
}

// ---------------------------------------------------------------------------
// device setup (Section 2, amg_setup, with every step in device kernels)
// ---------------------------------------------------------------------------
// device temporaries of one setup; whatever is still held is freed on every
// exit path, and an array that becomes part of the hierarchy is claimed
struct SetupTemps {
    amg_ctx* h;
    std::vector<void*> held;
    explicit SetupTemps(amg_ctx* hh) : h(hh) {}
    ~SetupTemps() { rewind(0); }
    template <class T>
    T* get(int64_t n) {
        T* p = dalloc_n<T>(h, n);
        held.push_back(p);
        return p;
    }
    void claim(const void* p) {
        auto it = std::find(held.begin(), held.end(), p);
        if (it != held.end()) held.erase(it);
    }
    void release(void* p) {
        auto it = std::find(held.begin(), held.end(), p);
        if (it != held.end()) {
            held.erase(it);
            dfree(h, p);
        }
    }
    size_t mark() const { return held.size(); }
    void rewind(size_t m) {
        while (held.size() > m) {
            dfree(h, held.back());
            held.pop_back();
        }
    }
};

// process-wide totals of the setup timing (amg_setup_profile_*)
struct SetupProfile {
    std::mutex mu;
    bool on = false;
    int64_t count[AMG_SK_NUM] = {};
    double ms[AMG_SK_NUM] = {};
    double bytes[AMG_SK_NUM] = {};
};

SetupProfile& setup_profile() {
    static SetupProfile p;
    return p;
}

// event pairs of one setup, added to the totals once the setup is done
struct SetupTimer {
    struct Rec {
        int kind;
        double bytes;
        hipEvent_t start, stop;
    };
    hipStream_t st;
    bool on;
    std::vector<Rec> recs;
    explicit SetupTimer(hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> g(setup_profile().mu);
        on = setup_profile().on;
    }
    ~SetupTimer() {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
    }
    void begin(int kind, double bytes) {
        if (!on) return;
        Rec r{kind, bytes, nullptr, nullptr};
        HIP_CHECK(hipEventCreate(&r.start));
        HIP_CHECK(hipEventCreate(&r.stop));
        recs.push_back(r);
        HIP_CHECK(hipEventRecord(r.start, st));
    }
    void end() {
        if (on) HIP_CHECK(hipEventRecord(recs.back().stop, st));
    }
    void collect() {
        if (!on || recs.empty()) return;
        HIP_CHECK(hipStreamSynchronize(st));
        SetupProfile& p = setup_profile();
        std::lock_guard<std::mutex> g(p.mu);
        for (auto& r : recs) {
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, r.start, r.stop));
            p.count[r.kind] += 1;
            p.ms[r.kind] += ms;
            p.bytes[r.kind] += r.bytes;
        }
    }
};

// bits that hold every value in [0, count)
int bits_for(int64_t count) {
    int b = 1;
    while ((int64_t(1) << b) < count) ++b;
    return b;
}

template <class T>
T read_scalar(amg_ctx* h, const T* p) {
    T v{};
    download(h, &v, p, 1);
    sync(h);
    return v;
}

void check_setup_error(amg_ctx* h, int* err) {
    int e[2] = {0, 0};
    download(h, e, err, 2);
    sync(h);
    if (!e[0]) return;
    static const std::pair<int, const char*> why[] = {
        {kErrRowPtr, "row_ptr must start at 0, be non-decreasing and end at nnz"},
        {kErrColRange, "column index out of range"},
        {kErrColOrder, "columns not strictly ascending"},
        {kErrNonFinite, "non-finite value"},
        {kErrNoDiag, "missing diagonal"},
        {kErrDiagSign, "non-positive diagonal"},
        {kErrAsymmetric, "matrix is not bitwise symmetric"},
        {kErrPattern, "coarse operator pattern is not structurally symmetric"}};
    for (auto& w : why)
        if (e[0] & w.first) {
            std::string msg = w.second;
            if (w.first != kErrPattern) msg += " (first offending row " + std::to_string(e[1]) + ")";
            throw AmgFailure{AMG_ERR_BAD_MATRIX, msg};
        }
}

void scan_int64(amg_ctx* h, SetupTemps& t, const int64_t* in, int64_t* out, int64_t m) {
    size_t bytes = 0;
    HIP_CHECK(scan_counts(nullptr, bytes, in, out, m, h->stream));
    void* tmp = t.get<char>((int64_t)bytes);
    HIP_CHECK(scan_counts(tmp, bytes, in, out, m, h->stream));
    t.release(tmp);
}

// m terms (key = row << col_bits | col, value) in keys[0] / vals[0] (each
// with room for m + 1 entries) -> CSR of `rows` x `cols` with every entry the
// sum of its terms in list order; the sort is stable, so that order is the
// order the terms were listed in
DevMat combine_terms(amg_ctx* h, SetupTemps& t, SetupTimer& tm, uint64_t* keys[2], double* vals[2], int64_t m,
                     int rows, int cols, int col_bits, int key_bits) {
    hipStream_t st = h->stream;
    int res = 0;
    if (m > 0) {
        size_t bytes = 0;
        HIP_CHECK(sort_pairs(nullptr, bytes, keys, vals, m, key_bits, res, st));
        void* tmp = t.get<char>((int64_t)bytes);
        tm.begin(AMG_SK_SORT, 32.0 * m);
        HIP_CHECK(sort_pairs(tmp, bytes, keys, vals, m, key_bits, res, st));
        tm.end();
        t.release(tmp);
    }
    const uint64_t* sk = keys[res];
    const double* sv = vals[res];
    uint64_t* run_keys = keys[1 - res];
    int64_t* flags = reinterpret_cast<int64_t*>(vals[1 - res]);
    int64_t* head = t.get<int64_t>(m + 1);
    tm.begin(AMG_SK_COMBINE, 16.0 * m + 16.0 * m);
    launch_run_heads(m, sk, flags, st);
    scan_int64(h, t, flags, head, m);
    tm.end();
    const int64_t nnz = read_scalar(h, head + m);
    if (nnz > INT32_MAX) throw AmgFailure{AMG_ERR_INVALID_ARG, "coarse operator exceeds int32 nonzeros"};
    DevMat out;
    out.rows = rows;
    out.cols = cols;
    out.rp = t.get<int32_t>(rows + 1);
    out.ci = t.get<int32_t>(nnz + kCsrPad);
    out.v = t.get<double>(nnz + kCsrPad);
    set_shape(out, nnz);
    tm.begin(AMG_SK_COMBINE, 24.0 * m + 20.0 * nnz + 8.0 * nnz + 4.0 * (rows + 1));
    launch_run_sums(m, sk, sv, head, col_bits, out.ci, out.v, run_keys, st);
    launch_rowptr_from_keys(nnz, run_keys, col_bits, rows, out.rp, st);
    tm.end();
    check_launch();
    t.release(head);
    return out;
}

void claim_mat(SetupTemps& t, const DevMat& m) {
    t.claim(m.rp);
    t.claim(m.ci);
    t.claim(m.v);
}

void release_mat(SetupTemps& t, DevMat& m) {
    t.release(m.rp);
    t.release(m.ci);
    t.release(m.v);
    m = DevMat{};
}

// coarsening: AMG_COARSEN_RS (the first pass on the host, from the strength
// pattern built here) or AMG_COARSEN_PMIS (on the device, weights of level l
// from the SplitMix64 stream seed + l)
void setup_device(amg_ctx* h, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                  const double* val, int coarsening, uint64_t seed) {
    hipStream_t st = h->stream;
    SetupTemps t(h);
    SetupTimer tm(st);
    int* err = t.get<int>(2);
    const int err_init[2] = {0, INT32_MAX};
    upload(h, err, err_init, 2);
    launch_validate_csr((int)n, nnz, row_ptr, col, val, err, st);
    check_launch();
    check_setup_error(h, err);

    h->lv.clear();
    h->lv.emplace_back();
    {
        DevMat& A = h->lv[0].A;
        A.rows = A.cols = (int)n;
        A.rp = dalloc_n<int32_t>(h, n + 1);
        A.ci = dalloc_n<int32_t>(h, nnz + kCsrPad);
        A.v = dalloc_n<double>(h, nnz + kCsrPad);
        set_shape(A, nnz);
        HIP_CHECK(hipMemcpyAsync(A.rp, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, st));
        HIP_CHECK(hipMemcpyAsync(A.ci, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st));
        HIP_CHECK(hipMemcpyAsync(A.v, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, st));
        h->lv[0].n = (int)n;
    }
    int32_t* scan_tmp = t.get<int32_t>(scan_scratch_ints((int)n));
    while (h->lv.back().n > h->sp.max_coarse && (int)h->lv.size() < h->sp.max_levels) {
        const int l = (int)h->lv.size() - 1;
        const int nl = h->lv[l].n;
        const DevMat A = h->lv[l].A;
        const double anz = (double)A.nnz, np1 = (double)nl + 1;
        const size_t level_mark = t.mark();
        // strength pattern and lambda
        int32_t* cnt = t.get<int32_t>(nl + 1);
        int32_t* srp = t.get<int32_t>(nl + 1);
        tm.begin(AMG_SK_STRENGTH, 12 * anz + 4 * np1 + 4.0 * nl + 8 * np1);
        launch_strength_count(nl, A.rp, A.ci, A.v, h->sp.theta, cnt, st);
        launch_exclusive_scan(nl, cnt, srp, scan_tmp, st);
        tm.end();
        const int32_t snnz = read_scalar(h, srp + nl);
        int32_t* sci = t.get<int32_t>(snnz);
        int32_t* lam = t.get<int32_t>(nl);
        tm.begin(AMG_SK_STRENGTH, 12 * anz + 8 * np1 + 8.0 * snnz + 8.0 * nl);
        launch_fill_u32(nl, reinterpret_cast<unsigned*>(lam), 0u, st);
        launch_strength_fill(nl, A.rp, A.ci, A.v, h->sp.theta, srp, sci, lam, st);
        tm.end();
        // C/F split
        int32_t* state = t.get<int32_t>(nl);
        if (coarsening == AMG_COARSEN_PMIS) {
            double* w = t.get<double>(nl);
            int32_t* mark = t.get<int32_t>(nl);
            int32_t* left = t.get<int32_t>(1);
            tm.begin(AMG_SK_SPLIT, 4.0 * nl + 16.0 * nl);
            launch_pmis_init(nl, lam, seed + (uint64_t)l, w, state, mark, st);
            tm.end();
            // every round decides at least the undecided point of largest weight
            for (int round = 1;; ++round) {
                if (round > nl + 1) throw AmgFailure{AMG_ERR_DEVICE, "PMIS rounds did not finish"};
                tm.begin(AMG_SK_SPLIT, 2 * (4.0 * snnz + 4 * np1) + 36.0 * nl);
                launch_pmis_round(nl, srp, sci, w, state, mark, round, left, st);
                tm.end();
                check_launch();
                if (read_scalar(h, left) == 0) break;
            }
        } else {
            tm.begin(AMG_SK_SPLIT, 0.0);
            HostCsr s;
            s.rows = s.cols = nl;
            s.ptr.resize(nl + 1);
            s.idx.resize(snnz);
            download(h, s.ptr.data(), srp, nl + 1);
            download(h, s.idx.data(), sci, snnz);
            sync(h);
            const std::vector<int32_t> split = ruge_stueben_split(s);
            upload(h, state, split.data(), nl);
            tm.end();
            sync(h);   // the host copy goes out of scope
        }
        // coarse numbering
        int32_t* cidx = t.get<int32_t>(nl + 1);
        tm.begin(AMG_SK_INTERP, 8.0 * nl + 8 * np1);
        launch_c_flags(nl, state, cnt, st);
        launch_exclusive_scan(nl, cnt, cidx, scan_tmp, st);
        tm.end();
        const int32_t nc = read_scalar(h, cidx + nl);
        if (nc == 0 || nc == nl) {
            t.rewind(level_mark);
            break;
        }
        {
            std::vector<int32_t> cf(nl);
            download(h, cf.data(), state, nl);
            sync(h);
            for (auto& c : cf) c = c == kPtC;
            h->lv[l].split = std::move(cf);
        }
        h->lv[l].nc = nc;
        h->lv[l].c_points = dalloc_n<int32_t>(h, nc);
        // direct interpolation
        DevMat P;
        P.rows = nl;
        P.cols = nc;
        P.rp = t.get<int32_t>(nl + 1);
        tm.begin(AMG_SK_INTERP, 4.0 * snnz + 4 * np1 + 8.0 * nl + 4 * nc + 4 * np1);
        launch_c_points(nl, state, cidx, h->lv[l].c_points, st);
        launch_interp_count(nl, srp, sci, state, cnt, st);
        launch_exclusive_scan(nl, cnt, P.rp, scan_tmp, st);
        tm.end();
        const int32_t pnnz = read_scalar(h, P.rp + nl);
        P.ci = t.get<int32_t>(pnnz + kCsrPad);
        P.v = t.get<double>(pnnz + kCsrPad);
        set_shape(P, pnnz);
        tm.begin(AMG_SK_INTERP, 12 * anz + 4 * np1 + 4.0 * snnz + 4 * np1 + 8.0 * nl + 12.0 * pnnz);
        launch_interp_fill(nl, A.rp, A.ci, A.v, srp, sci, state, cidx, P.rp, P.ci, P.v, st);
        tm.end();
        check_launch();
        claim_mat(t, P);
        h->lv[l].P = P;
        const int rb = bits_for(nl), cb = bits_for(nc);
        // R = P^T: the entries of P sorted by (column, row)
        {
            uint64_t* keys[2] = {t.get<uint64_t>(pnnz + 1), t.get<uint64_t>(pnnz + 1)};
            double* vals[2] = {t.get<double>(pnnz + 1), t.get<double>(pnnz + 1)};
            tm.begin(AMG_SK_TRANSPOSE, 12.0 * pnnz + 4 * np1 + 16.0 * pnnz);
            launch_transpose_keys(nl, P.rp, P.ci, P.v, rb, keys[0], vals[0], st);
            tm.end();
            int res = 0;
            size_t bytes = 0;
            HIP_CHECK(sort_pairs(nullptr, bytes, keys, vals, pnnz, rb + cb, res, st));
            void* tmp = t.get<char>((int64_t)bytes);
            tm.begin(AMG_SK_SORT, 32.0 * pnnz);
            HIP_CHECK(sort_pairs(tmp, bytes, keys, vals, pnnz, rb + cb, res, st));
            tm.end();
            DevMat R;
            R.rows = nc;
            R.cols = nl;
            R.rp = dalloc_n<int32_t>(h, nc + 1);
            R.ci = dalloc_n<int32_t>(h, pnnz + kCsrPad);
            R.v = dalloc_n<double>(h, pnnz + kCsrPad);
            set_shape(R, pnnz);
            h->lv[l].R = R;
            tm.begin(AMG_SK_TRANSPOSE, 16.0 * pnnz + 12.0 * pnnz + 8.0 * pnnz + 4.0 * (nc + 1));
            launch_unpack_keys(pnnz, keys[res], vals[res], rb, R.ci, R.v, st);
            launch_rowptr_from_keys(pnnz, keys[res], rb, nc, R.rp, st);
            tm.end();
            check_launch();
            for (void* q : {(void*)tmp, (void*)keys[0], (void*)keys[1], (void*)vals[0], (void*)vals[1]})
                t.release(q);
        }
        // T = A P
        int64_t* cnt64 = t.get<int64_t>(nl + 1);
        int64_t* off = t.get<int64_t>(nl + 1);
        tm.begin(AMG_SK_EXPAND, 4 * np1 + 4 * anz + 4 * np1 + 8 * np1 + 16 * np1);
        launch_ap_count(nl, A.rp, A.ci, P.rp, cnt64, st);
        scan_int64(h, t, cnt64, off, nl);
        tm.end();
        int64_t m = read_scalar(h, off + nl);
        DevMat T;
        {
            uint64_t* keys[2] = {t.get<uint64_t>(m + 1), t.get<uint64_t>(m + 1)};
            double* vals[2] = {t.get<double>(m + 1), t.get<double>(m + 1)};
            tm.begin(AMG_SK_EXPAND, 12 * anz + 4 * np1 + 12.0 * pnnz + 4 * np1 + 8 * np1 + 16.0 * m);
            launch_ap_expand(nl, A.rp, A.ci, A.v, P.rp, P.ci, P.v, off, cb, keys[0], vals[0], st);
            tm.end();
            check_launch();
            T = combine_terms(h, t, tm, keys, vals, m, nl, nc, cb, rb + cb);
            for (void* q : {(void*)keys[0], (void*)keys[1], (void*)vals[0], (void*)vals[1]}) t.release(q);
        }
        // C = P^T T, terms of each (I, J) listed in ascending fine row
        tm.begin(AMG_SK_EXPAND, 8 * np1 + 8 * np1 + 16 * np1);
        launch_pt_count(nl, P.rp, T.rp, cnt64, st);
        scan_int64(h, t, cnt64, off, nl);
        tm.end();
        m = read_scalar(h, off + nl);
        DevMat C;
        {
            uint64_t* keys[2] = {t.get<uint64_t>(m + 1), t.get<uint64_t>(m + 1)};
            double* vals[2] = {t.get<double>(m + 1), t.get<double>(m + 1)};
            tm.begin(AMG_SK_EXPAND, 12.0 * pnnz + 4 * np1 + 12.0 * T.nnz + 4 * np1 + 8 * np1 + 16.0 * m);
            launch_pt_expand(nl, P.rp, P.ci, P.v, T.rp, T.ci, T.v, off, cb, keys[0], vals[0], st);
            tm.end();
            check_launch();
            release_mat(t, T);
            C = combine_terms(h, t, tm, keys, vals, m, nc, nc, cb, 2 * cb);
            for (void* q : {(void*)keys[0], (void*)keys[1], (void*)vals[0], (void*)vals[1]}) t.release(q);
        }
        // A_{l+1} = (C + C^T) / 2
        double* sym = t.get<double>(C.nnz + kCsrPad);
        tm.begin(AMG_SK_SYMMETRIZE, 12.0 * C.nnz + 4.0 * (nc + 1) + 8.0 * C.nnz);
        launch_symmetrize(nc, C.rp, C.ci, C.v, sym, err, st);
        tm.end();
        check_launch();
        check_setup_error(h, err);
        t.release(C.v);
        C.v = sym;
        claim_mat(t, C);
        t.rewind(level_mark);
        h->lv.emplace_back();
        h->lv.back().A = C;
        h->lv.back().n = nc;
    }
    t.rewind(0);
    tm.collect();
    if (h->lv.back().n > kMaxDenseCoarse)
        throw AmgFailure{AMG_ERR_INVALID_ARG, "coarsest level has " + std::to_string(h->lv.back().n) +
                                                  " rows; the dense coarse solve allows at most " +
                                                  std::to_string(kMaxDenseCoarse)};
    finish_setup(h);
}

void destroy(amg_ctx* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->batch) destroy_batch(h->batch);
    for (auto& d : h->lv) {
        free_mat(h, d.Ahs);
        free_mat(h, d.A);
        free_mat(h, d.P);
        free_mat(h, d.R);
        dfree(h, d.c_points);
        dfree(h, d.dinv);
        dfree(h, d.in_m);
        dfree(h, d.keep);
        dfree(h, d.rowmax);
        dfree(h, d.lump_thr);
        dfree(h, d.lump_den);
        dfree(h, d.b);
        dfree(h, d.x);
        dfree(h, d.xt);
        dfree(h, d.r);
        for (void* q : {(void*)d.A32, (void*)d.Ahs32, (void*)d.P32, (void*)d.R32, (void*)d.dinv32,
                        (void*)d.b32, (void*)d.x32, (void*)d.xt32, (void*)d.r32})
            dfree(h, q);
    }
    dfree(h, h->cg_r32);
    dfree(h, h->cg_z32);
    free_block_bufs(h, h->blk64);
    free_block_bufs(h, h->blk32);
    dfree(h, h->blk_partials);
    dfree(h, h->blk_b);
    dfree(h, h->blk_x);
    for (void* q : {(void*)h->bcg_r, (void*)h->bcg_p, (void*)h->bcg_q, (void*)h->bcg_z}) dfree(h, q);
    for (void* p : {(void*)h->coarse_inv, (void*)h->scal, (void*)h->partials,
                    (void*)h->scan_scratch, (void*)h->cnt, (void*)h->sp_cnt, (void*)h->sp_bsum, (void*)h->missing, (void*)h->singular, (void*)h->cg_r,
                    (void*)h->cg_z, (void*)h->cg_p, (void*)h->cg_q, (void*)h->xw, (void*)h->rt})
        dfree(h, p);
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (auto& pe : h->pending) {
        (void)hipEventDestroy(pe.start);
        (void)hipEventDestroy(pe.stop);
    }
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    delete h;
}

// ---------------------------------------------------------------------------
// work memory of the allocation-free solve: a file-scope device array that
// every GPU the library runs on holds until the process ends.  Layout, in
// doubles: the scalar slots, the per-workgroup dot partials, then the six
// n-vectors of the solve (r, z, p, q, the window-start x, the window's true
// residual), each starting on a 256-byte boundary.  Every call on a GPU uses
// that GPU's copy, so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxRows = 2097152;     // 2^21: 3D Poisson 128^3
constexpr int64_t kNoAllocScalars = 256;         // >= S_COUNT
constexpr int64_t kNoAllocPartials = 65536;      // >= every launch's workgroup count
constexpr int64_t kNoAllocVectors = 6;
constexpr int64_t kNoAllocDoubles = kNoAllocScalars + kNoAllocPartials + kNoAllocVectors * kNoAllocMaxRows + 32;
static_assert(S_COUNT <= kNoAllocScalars, "scalar slots do not fit the allocation-free work memory");

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kNoAllocMaxDevices = 64;

// device address of this GPU's scratch (the array's name in host code is a
// host-side stand-in, never passed to a kernel); looked up once per device
// with that device current
double* noalloc_scratch(int device) {
    static std::mutex mu;
    static double* addr[kNoAllocMaxDevices] = {};
    if (device < 0 || device >= kNoAllocMaxDevices)
        throw AmgFailure{AMG_ERR_DEVICE, "device index out of range for the allocation-free solve"};
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = 0;
        HIP_CHECK(hipGetDevice(&cur));
        if (cur != device) HIP_CHECK(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            throw AmgFailure{AMG_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e)};
        addr[device] = static_cast<double*>(ptr);
    }
    return addr[device];
}

// points the handle's solve work memory into the scratch array for the
// lifetime of the object and restores the handle's own buffers afterwards
struct NoAllocWork {
    amg_ctx* h;
    double *r, *z, *p, *q, *xw, *rt, *partials, *scal;
    NoAllocWork(amg_ctx* hh, double* base, int64_t n) : h(hh) {
        r = h->cg_r; z = h->cg_z; p = h->cg_p; q = h->cg_q; xw = h->xw; rt = h->rt;
        partials = h->partials; scal = h->scal;
        const int64_t stride = (n + 31) / 32 * 32;
        double* v = base + kNoAllocScalars + kNoAllocPartials;
        h->scal = base;
        h->partials = base + kNoAllocScalars;
        h->cg_r = v;
        h->cg_z = v + stride;
        h->cg_p = v + 2 * stride;
        h->cg_q = v + 3 * stride;
        h->xw = v + 4 * stride;
        h->rt = v + 5 * stride;
    }
    ~NoAllocWork() {
        h->cg_r = r; h->cg_z = z; h->cg_p = p; h->cg_q = q; h->xw = xw; h->rt = rt;
        h->partials = partials; h->scal = scal;
    }
};

template <class F>
amg_status guarded(amg_ctx* h, F&& f) {
    try {
        return f();
    } catch (const AmgFailure& e) {
        if (h) h->last_error = e.what;
        return e.status;
    } catch (const std::bad_alloc&) {
        if (h) h->last_error = "host allocation failed";
        return AMG_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        if (h) h->last_error = e.what();
        return AMG_ERR_DEVICE;
    } catch (...) {
        if (h) h->last_error = "unknown failure";
        return AMG_ERR_DEVICE;
    }
}

bool valid_gamma(double g) { return g >= 0.0 && g <= 1.0; }

// failure message of the last amg_setup_from_csr on this thread that failed
std::string& setup_error() {
    static thread_local std::string msg;
    return msg;
}

template <class T>
amg_status vcycle_block_abi(amg_handle h, int32_t nrhs, const T* b, T* x) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (gs_on(h)) {
        h->last_error = "hybrid Gauss-Seidel relaxation runs in the FP64 single-vector cycle only";
        return AMG_ERR_INVALID_ARG;
    }
    const int64_t n = h->lv[0].n;
    if (!b || !x || (nrhs != 4 && nrhs != 8 && nrhs != 16) || n * nrhs > INT32_MAX ||
        (((uintptr_t)b | (uintptr_t)x) & 15) != 0) {
        h->last_error = "nrhs must be 4, 8 or 16 and the blocks 16-byte aligned";
        return AMG_ERR_INVALID_ARG;
    }
    return guarded(h, [&] {
        if constexpr (sizeof(T) == 4) ensure_fp32(h);
        BlockBufs<T>& bb = ensure_block<T>(h, nrhs);
        launch_fill_f64(1, h->scal + S_LIVE, (double)nrhs, h->stream);
        launch_copy((int)(n * nrhs), bb.x[0], x, h->stream);
        T* res = vcycle_block<T>(h, nrhs, b, Guess::kNonzero, BlockSink<T>{});
        launch_copy((int)(n * nrhs), x, res, h->stream);
        check_launch();
        prof_collect(h);
        return AMG_OK;
    });
}

// a new handle built by `build` (which throws AmgFailure on failure); *out
// is cleared by the caller
template <class F>
amg_status setup_abi(const amg_setup_params* params, void* stream, amg_alloc_fn alloc, amg_free_fn free_fn,
                     void* user, amg_handle* out, F&& build) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return AMG_ERR_INVALID_ARG;
    amg_setup_params sp;
    amg_setup_params_default(&sp);
    if (params) sp = *params;
    if (!(sp.theta > 0.0 && sp.theta <= 1.0) || sp.max_coarse < 1 || sp.max_levels < 1 ||
        !(sp.omega > 0.0 && sp.omega < 2.0) || sp.nu_pre < 0 || sp.nu_post < 0)
        return AMG_ERR_INVALID_ARG;
    amg_ctx* h = new (std::nothrow) amg_ctx();
    if (!h) return AMG_ERR_OUT_OF_MEMORY;
    h->stream = (hipStream_t)stream;
    h->alloc_fn = alloc;
    h->free_fn = free_fn;
    h->user = user;
    h->sp = sp;
    amg_status st = guarded(h, [&] {
        HIP_CHECK(hipGetDevice(&h->device));
        build(h);
        return AMG_OK;
    });
    if (st != AMG_OK) {
        setup_error() = h->last_error;
        destroy(h);
        return st;
    }
    *out = h;
    return AMG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void amg_setup_params_default(amg_setup_params* p) {
    if (!p) return;
    p->theta = 0.25;
    p->max_coarse = 49;
    p->max_levels = 25;
    p->omega = 2.0 / 3.0;
    p->nu_pre = 1;
    p->nu_post = 1;
}

void amg_solve_params_default(amg_solve_params* p) {
    if (!p) return;
    p->method = AMG_PCG;
    p->rtol = 1e-8;
    p->maxit = 200;
    p->adaptive = 0;
    p->k = 3;
    p->s = 1;
    p->rho_max = 0.5;
    p->gamma_min = 0.01;
    p->precision = 64;
    p->zero_guess = 0;
}

amg_status amg_setup_from_csr(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                              const amg_setup_params* params, void* stream, amg_alloc_fn alloc,
                              amg_free_fn free_fn, void* user, amg_handle* out) {
    if (!out) return AMG_ERR_INVALID_ARG;
    *out = nullptr;
    if (n <= 0 || n > INT32_MAX - 1 || !row_ptr || !col || !val) return AMG_ERR_INVALID_ARG;
    return setup_abi(params, stream, alloc, free_fn, user, out,
                     [&](amg_ctx* h) { setup(h, n, row_ptr, col, val, {}); });
}

amg_status amg_setup_nongalerkin_from_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                                          const double* val, const amg_setup_params* params,
                                          const double* gamma, int32_t count, void* stream,
                                          amg_alloc_fn alloc, amg_free_fn free_fn, void* user,
                                          amg_handle* out) {
    if (!out) return AMG_ERR_INVALID_ARG;
    *out = nullptr;
    if (n <= 0 || n > INT32_MAX - 1 || !row_ptr || !col || !val) return AMG_ERR_INVALID_ARG;
    if (!gamma || count < 1) return AMG_ERR_INVALID_ARG;
    std::vector<double> ng(gamma, gamma + count);
    ng[0] = 0.0;    // A_0 is the given matrix
    for (double g : ng)
        if (!valid_gamma(g)) return AMG_ERR_INVALID_ARG;
    return setup_abi(params, stream, alloc, free_fn, user, out,
                     [&](amg_ctx* h) { setup(h, n, row_ptr, col, val, ng); });
}

amg_status amg_setup_device(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                            const double* val, const amg_setup_params* params, int32_t coarsening,
                            uint64_t seed, void* stream, amg_alloc_fn alloc, amg_free_fn free_fn, void* user,
                            amg_handle* out) {
    if (!out) return AMG_ERR_INVALID_ARG;
    *out = nullptr;
    if (n <= 0 || n > INT32_MAX - 1 || nnz < n || nnz > INT32_MAX - 8 || !row_ptr || !col || !val)
        return AMG_ERR_INVALID_ARG;
    if (coarsening != AMG_COARSEN_RS && coarsening != AMG_COARSEN_PMIS) return AMG_ERR_INVALID_ARG;
    return setup_abi(params, stream, alloc, free_fn, user, out,
                     [&](amg_ctx* h) { setup_device(h, n, nnz, row_ptr, col, val, coarsening, seed); });
}

amg_status amg_set_compact_indices(amg_handle h, int32_t enable) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    return guarded(h, [&] {
        set_compact_indices(h, enable != 0);
        return AMG_OK;
    });
}

amg_status amg_index_width(amg_handle h, int32_t l, int32_t which, int32_t* bytes) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 0 || l >= (int)h->lv.size() || !bytes || which < AMG_MAT_A || which > AMG_MAT_R)
        return AMG_ERR_INVALID_ARG;
    const DevLevel& d = h->lv[l];
    const DevMat& m = which == AMG_MAT_A ? d.A : which == AMG_MAT_AHAT ? d.Ah : which == AMG_MAT_P ? d.P : d.R;
    *bytes = m.sl_off ? (m.sl_idx8 ? 1 : m.sl_col16 ? 2 : 4) : m.ci16 ? 2 : 4;
    return AMG_OK;
}

amg_status amg_row_format(amg_handle h, int32_t l, int32_t which, int32_t* format) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 0 || l >= (int)h->lv.size() || !format || which < AMG_MAT_A || which > AMG_MAT_R)
        return AMG_ERR_INVALID_ARG;
    const DevLevel& d = h->lv[l];
    const DevMat& m = which == AMG_MAT_A ? d.A : which == AMG_MAT_AHAT ? d.Ah : which == AMG_MAT_P ? d.P : d.R;
    if (!m.rp) return AMG_ERR_INVALID_ARG;
    *format = m.sl_off ? AMG_FORMAT_SELL : stream_block_rows(m.view()) ? AMG_FORMAT_STREAM : AMG_FORMAT_ROW;
    return AMG_OK;
}

amg_status amg_setup_profile_enable(int32_t enable) {
    SetupProfile& p = setup_profile();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = enable != 0;
    if (p.on)
        for (int k = 0; k < AMG_SK_NUM; ++k) {
            p.count[k] = 0;
            p.ms[k] = 0.0;
            p.bytes[k] = 0.0;
        }
    return AMG_OK;
}

amg_status amg_setup_profile_read(int32_t kernel_class, int64_t* count, double* ms, double* bytes) {
    if (kernel_class < 0 || kernel_class >= AMG_SK_NUM) return AMG_ERR_INVALID_ARG;
    SetupProfile& p = setup_profile();
    std::lock_guard<std::mutex> g(p.mu);
    if (count) *count = p.count[kernel_class];
    if (ms) *ms = p.ms[kernel_class];
    if (bytes) *bytes = p.bytes[kernel_class];
    return AMG_OK;
}

amg_status amg_sparsify(amg_handle h, double gamma, int32_t first_level) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (!valid_gamma(gamma) || first_level < 1) {
        h->last_error = "gamma must lie in [0, 1] and first_level must be >= 1";
        return AMG_ERR_INVALID_ARG;
    }
    return guarded(h, [&] {
        std::vector<std::pair<int, double>> todo;
        for (int l = 1; l < (int)h->lv.size(); ++l) todo.emplace_back(l, l >= first_level ? gamma : 0.0);
        sparsify_levels(h, todo);
        prof_collect(h);
        return AMG_OK;
    });
}

amg_status amg_sparsify_levels(amg_handle h, const double* gamma, int32_t count) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (!gamma || count < 0) return AMG_ERR_INVALID_ARG;
    for (int l = 1; l < count; ++l)
        if (!valid_gamma(gamma[l])) {
            h->last_error = "gamma[" + std::to_string(l) + "] outside [0, 1]";
            return AMG_ERR_INVALID_ARG;
        }
    return guarded(h, [&] {
        std::vector<std::pair<int, double>> todo;
        for (int l = 1; l < (int)h->lv.size(); ++l) todo.emplace_back(l, l < count ? gamma[l] : 0.0);
        sparsify_levels(h, todo);
        prof_collect(h);
        return AMG_OK;
    });
}

amg_status amg_set_method(amg_handle h, int32_t method) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (method != AMG_SPARSE_GALERKIN && method != AMG_HYBRID_GALERKIN) return AMG_ERR_INVALID_ARG;
    h->method = method;
    return AMG_OK;
}

amg_status amg_reintroduce(amg_handle h, int32_t s, double gamma_min, int32_t* first_changed_level) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (s < 1 || !(gamma_min >= 0.0)) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        int first = -1;
        amg_status st = do_reintroduce(h, s, gamma_min, &first);
        if (first_changed_level) *first_changed_level = first;
        prof_collect(h);
        return st;
    });
}

amg_status amg_solve(amg_handle h, const double* b, double* x, const amg_solve_params* params,
                     amg_solve_info* info, double* hist) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (!b || !x) return AMG_ERR_INVALID_ARG;
    amg_solve_params p;
    amg_solve_params_default(&p);
    if (params) p = *params;
    if ((p.method != AMG_PCG && p.method != AMG_STATIONARY) || p.maxit < 0 || !(p.rtol >= 0.0) ||
        (p.adaptive && (p.k < 1 || p.s < 1)) || (p.precision != 64 && p.precision != 32) ||
        (p.zero_guess != 0 && p.zero_guess != 1)) {
        h->last_error = "invalid solve parameters";
        return AMG_ERR_INVALID_ARG;
    }
    if (gs_on(h) && p.precision != 64) {
        h->last_error = "hybrid Gauss-Seidel relaxation runs in the FP64 cycle only";
        return AMG_ERR_INVALID_ARG;
    }
    return guarded(h, [&] { return solve(h, b, x, p, info, hist); });
}

amg_status amg_solve_noalloc(amg_handle h, const double* b, double* x, const amg_solve_params* params,
                             amg_solve_info* info, double* hist) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (!b || !x) return AMG_ERR_INVALID_ARG;
    amg_solve_params p;
    amg_solve_params_default(&p);
    if (params) p = *params;
    if ((p.method != AMG_PCG && p.method != AMG_STATIONARY) || p.maxit < 0 || !(p.rtol >= 0.0) ||
        (p.adaptive && (p.k < 1 || p.s < 1)) || p.precision != 64 || (p.zero_guess != 0 && p.zero_guess != 1)) {
        h->last_error = "invalid solve parameters (the allocation-free solve runs the FP64 cycle only)";
        return AMG_ERR_INVALID_ARG;
    }
    const int64_t n = h->lv[0].n;
    if (n > kNoAllocMaxRows || h->partial_cap > kNoAllocPartials) {
        h->last_error = "the allocation-free solve takes at most " + std::to_string(kNoAllocMaxRows) +
                        " rows; this problem has " + std::to_string(n);
        return AMG_ERR_INVALID_ARG;
    }
    if (h->profiling) {
        h->last_error = "the allocation-free solve does not run with kernel profiling enabled";
        return AMG_ERR_STATE;
    }
    if (p.adaptive && h->lumping == AMG_LUMP_STRONG)
        for (size_t l = 1; l < h->lv.size(); ++l)
            if (h->lv[l].gamma > 0.0 && !h->lv[l].lump_thr) {
                h->last_error = "reintroduction under strong lumping would allocate: level " + std::to_string(l) +
                                " was sparsified with diagonal lumping";
                return AMG_ERR_STATE;
            }
    return guarded(h, [&] {
        double* base = noalloc_scratch(h->device);
        NoAllocWork work(h, base, n);
        return solve(h, b, x, p, info, hist);
    });
}

amg_status amg_vcycle(amg_handle h, const double* b, double* x) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (!b || !x) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        if (gs_on(h)) vcycle_gs(h, b, x, Guess::kNonzero, -1);
        else vcycle<double>(h, b, x, Guess::kNonzero, -1);
        prof_collect(h);
        return AMG_OK;
    });
}

amg_status amg_set_lumping(amg_handle h, int32_t lumping) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (lumping != AMG_LUMP_DIAGONAL && lumping != AMG_LUMP_STRONG) return AMG_ERR_INVALID_ARG;
    h->lumping = lumping;
    return AMG_OK;
}

amg_status amg_set_lump_shapes(amg_handle h, double wide_mean_row, double den_wave_mean_row, int32_t small_rows) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (std::isnan(wide_mean_row) || std::isnan(den_wave_mean_row) || small_rows < 0) return AMG_ERR_INVALID_ARG;
    h->lump_shapes.wide_mean_row = wide_mean_row;
    h->lump_shapes.den_wave_mean_row = den_wave_mean_row;
    h->lump_shapes.small_rows = small_rows;
    return AMG_OK;
}

amg_status amg_set_relaxation(amg_handle h, int32_t relaxation, int32_t block_rows) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if ((relaxation != AMG_RELAX_JACOBI && relaxation != AMG_RELAX_HYBRID_GS) || block_rows < 1)
        return AMG_ERR_INVALID_ARG;
    h->relax = relaxation;
    h->gs_block = block_rows;
    return AMG_OK;
}

amg_status amg_vcycle32(amg_handle h, const float* b, float* x) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (!b || !x) return AMG_ERR_INVALID_ARG;
    if (gs_on(h)) {
        h->last_error = "hybrid Gauss-Seidel relaxation runs in the FP64 single-vector cycle only";
        return AMG_ERR_INVALID_ARG;
    }
    return guarded(h, [&] {
        ensure_fp32(h);
        vcycle<float>(h, b, x, Guess::kNonzero, -1);
        prof_collect(h);
        return AMG_OK;
    });
}

amg_status amg_solve_block(amg_handle h, int32_t nrhs, const double* b, double* x, const amg_solve_params* params,
                           amg_solve_info* info, int32_t* col_iters, double* col_relres) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (gs_on(h)) {
        h->last_error = "hybrid Gauss-Seidel relaxation runs in the FP64 single-vector cycle only";
        return AMG_ERR_INVALID_ARG;
    }
    amg_solve_params p;
    amg_solve_params_default(&p);
    if (params) p = *params;
    const int64_t n = h->lv[0].n;
    if (!b || !x || nrhs < 1 || nrhs > kMaxBlockRhs || n * block_width(nrhs) > INT32_MAX ||
        (p.method != AMG_STATIONARY && p.method != AMG_PCG) || p.adaptive || p.maxit < 0 || !(p.rtol >= 0.0) ||
        (p.precision != 64 && p.precision != 32) || p.zero_guess != 0) {
        h->last_error = "invalid block solve arguments (1 <= nrhs <= 16, not adaptive, zero_guess 0)";
        return AMG_ERR_INVALID_ARG;
    }
    const int k = block_width(nrhs);
    if (k == nrhs && (((uintptr_t)b | (uintptr_t)x) & 15) != 0) {
        h->last_error = "block vectors must be 16-byte aligned";
        return AMG_ERR_INVALID_ARG;
    }
    return guarded(h, [&] {
        const double* bk = b;
        double* xk = x;
        if (k != nrhs) {
            // K-wide copies with zero columns nrhs..K-1
            if (h->blk_pack_k < k) {
                dfree(h, h->blk_b);
                dfree(h, h->blk_x);
                h->blk_b = h->blk_x = nullptr;
                h->blk_b = dalloc_n<double>(h, n * k);
                h->blk_x = dalloc_n<double>(h, n * k);
                h->blk_pack_k = k;
            }
            launch_block_pack((int)n, nrhs, k, b, h->blk_b, h->stream);
            launch_block_pack((int)n, nrhs, k, x, h->blk_x, h->stream);
            check_launch();
            bk = h->blk_b;
            xk = h->blk_x;
        }
        amg_status st;
        if (p.method == AMG_PCG)
            st = p.precision == 32 ? solve_block_pcg<float>(h, k, nrhs, bk, xk, p, info, col_iters, col_relres)
                                   : solve_block_pcg<double>(h, k, nrhs, bk, xk, p, info, col_iters, col_relres);
        else
            st = p.precision == 32 ? solve_block<float>(h, k, nrhs, bk, xk, p, info, col_iters, col_relres)
                                   : solve_block<double>(h, k, nrhs, bk, xk, p, info, col_iters, col_relres);
        if (k != nrhs) {
            launch_block_unpack((int)n, nrhs, k, xk, x, h->stream);
            check_launch();
        }
        return st;
    });
}

amg_status amg_vcycle_block(amg_handle h, int32_t nrhs, const double* b, double* x) {
    return vcycle_block_abi<double>(h, nrhs, b, x);
}

amg_status amg_vcycle_block32(amg_handle h, int32_t nrhs, const float* b, float* x) {
    return vcycle_block_abi<float>(h, nrhs, b, x);
}

amg_status amg_level_op(amg_handle h, int32_t level, int32_t op, const double* in, const double* x,
                        double* out) {
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    const int L = (int)h->lv.size() - 1;
    if (op == AMG_OP_COARSE_SOLVE) level = L;
    if (level < 0 || level > L || !out) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        DevLevel& v = h->lv[level];
        switch (op) {
            case AMG_OP_RESIDUAL:
                if (!in || !x) return AMG_ERR_INVALID_ARG;
                row_op(h, AMG_K_RESIDUAL, level, kResid, v.Ah, x, in, nullptr, out, nullptr, -1);
                break;
            case AMG_OP_JACOBI:
                if (!in || !x || x == out) return AMG_ERR_INVALID_ARG;
                row_op(h, AMG_K_JACOBI, level, kJacobi, v.Ah, x, in, v.dinv, out, nullptr, -1);
                break;
            case AMG_OP_RESTRICT:
                if (level == L || !in) return AMG_ERR_INVALID_ARG;
                row_op(h, AMG_K_RESTRICT, level, kSpmv, v.R, in, nullptr, nullptr, out, nullptr, -1);
                break;
            case AMG_OP_INTERPOLATE:
                if (level == L || !in || !x) return AMG_ERR_INVALID_ARG;
                row_op(h, AMG_K_INTERP, level, kSpmvAdd, v.P, in, x, nullptr, out, nullptr, -1);
                break;
            case AMG_OP_COARSE_SOLVE: {
                if (!in) return AMG_ERR_INVALID_ARG;
                ProfScope ps(h, AMG_K_COARSE, L);
                launch_dense_matvec(h->nL, h->coarse_inv, in, out, h->stream);
                check_launch();
                break;
            }
            case AMG_OP_SPMV_A:
                if (!x) return AMG_ERR_INVALID_ARG;
                row_op(h, AMG_K_RESIDUAL, level, kSpmv, v.A, x, nullptr, nullptr, out, nullptr, -1);
                break;
            case AMG_OP_SPMV_AHAT:
                if (!x) return AMG_ERR_INVALID_ARG;
                row_op(h, AMG_K_RESIDUAL, level, kSpmv, v.Ah, x, nullptr, nullptr, out, nullptr, -1);
                break;
            case AMG_OP_GS_FORWARD:
            case AMG_OP_GS_BACKWARD: {
                if (!in || !x || x == out) return AMG_ERR_INVALID_ARG;
                ProfScope ps(h, AMG_K_JACOBI, level);
                launch_hybrid_gs(op == AMG_OP_GS_FORWARD, v.n, v.Ah.rp, v.Ah.ci, v.Ah.v, in, x, out, h->gs_block,
                                 v.Ah.view().mean_row, h->stream);
                check_launch();
                break;
            }
            default:
                return AMG_ERR_INVALID_ARG;
        }
        return AMG_OK;
    });
}

amg_status amg_num_levels(amg_handle h, int32_t* nlev) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (!nlev) return AMG_ERR_INVALID_ARG;
    *nlev = (int32_t)h->lv.size();
    return AMG_OK;
}

static int64_t level_bytes(amg_ctx* h, int l) {
    // algorithmic bytes of one zero-guess V-cycle's work on level l: FP64
    // values, int32 indices, every vector entry counted once per kernel
    DevLevel& v = h->lv[l];
    const int L = (int)h->lv.size() - 1;
    const int64_t n = v.n;
    if (l == L) return 8 * n * n + 16 * n;
    const int64_t nnz = operator_nnz(h, v.Ah), nc = v.nc;
    int64_t b = 0;
    b += 12 * nnz + 4 * (n + 1) + 32 * n;                 // zero-guess sweep fused with residual
    b += 12 * v.R.nnz + 4 * (nc + 1) + 8 * n + 8 * nc;    // restriction
    b += 12 * v.P.nnz + 4 * (n + 1) + 8 * nc + 16 * n;    // interpolation and correction
    b += 12 * nnz + 4 * (n + 1) + 32 * n;                 // post-smoothing sweep
    return b;
}

amg_status amg_get_level(amg_handle h, int32_t l, int64_t* n, int64_t* nnz_galerkin, int64_t* nnz_sparse,
                         int64_t* nnz_p, int64_t* n_coarse, double* gamma, int64_t* bytes) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 0 || l >= (int)h->lv.size()) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        DevLevel& v = h->lv[l];
        if (n) *n = v.n;
        if (nnz_galerkin) *nnz_galerkin = v.A.nnz;
        if (nnz_sparse) *nnz_sparse = operator_nnz(h, v.Ah);
        if (nnz_p) *nnz_p = v.P.nnz;
        if (n_coarse) *n_coarse = v.nc;
        if (gamma) *gamma = v.gamma;
        if (bytes) *bytes = level_bytes(h, l);
        return AMG_OK;
    });
}

amg_status amg_export_level(amg_handle h, int32_t l, int32_t which, int32_t* row_ptr, int32_t* col,
                            double* val) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 0 || l >= (int)h->lv.size()) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        DevLevel& v = h->lv[l];
        DevMat* m = which == AMG_MAT_A ? &v.A : which == AMG_MAT_AHAT ? &v.Ah
                  : which == AMG_MAT_P ? &v.P : which == AMG_MAT_R ? &v.R : nullptr;
        if (!m || !m->rp) return AMG_ERR_INVALID_ARG;
        operator_nnz(h, *m);
        if (row_ptr) download(h, row_ptr, m->rp, m->rows + 1);
        if (col) download(h, col, m->ci, m->nnz);
        if (val) download(h, val, m->v, m->nnz);
        sync(h);
        return AMG_OK;
    });
}

amg_status amg_export_mask(amg_handle h, int32_t l, int32_t which, uint8_t* out) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 1 || l >= (int)h->lv.size() || !out) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        DevLevel& v = h->lv[l];
        if (which == AMG_MASK_M) {
            mark_minimal_pattern(h, l, h->method == AMG_HYBRID_GALERKIN);
            download(h, out, v.in_m, v.A.nnz);
        } else if (which == AMG_MASK_KEEP) {
            if (v.keep_valid) download(h, out, v.keep, v.A.nnz);
            else std::memset(out, 1, (size_t)v.A.nnz);
        } else {
            return AMG_ERR_INVALID_ARG;
        }
        sync(h);
        return AMG_OK;
    });
}

amg_status amg_export_vector(amg_handle h, int32_t l, int32_t which, double* out) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 0 || l >= (int)h->lv.size() || !out) return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        DevLevel& v = h->lv[l];
        if (which == AMG_VEC_ROWMAX) {
            if (l < 1) return AMG_ERR_INVALID_ARG;
            ensure_minimal_pattern(h, l);
            download(h, out, v.rowmax, v.n);
        } else if (which == AMG_VEC_DINV) {
            download(h, out, v.dinv, v.n);
        } else {
            return AMG_ERR_INVALID_ARG;
        }
        sync(h);
        return AMG_OK;
    });
}

amg_status amg_export_split(amg_handle h, int32_t l, int32_t* cf) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (l < 0 || l >= (int)h->lv.size() - 1 || !cf) return AMG_ERR_INVALID_ARG;
    std::memcpy(cf, h->lv[l].split.data(), sizeof(int32_t) * h->lv[l].split.size());
    return AMG_OK;
}

amg_status amg_profile_enable(amg_handle h, int32_t enable, int32_t kernel_class, int32_t level) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (kernel_class < -1 || kernel_class >= AMG_K_NUM || level < -1 || level >= (int)h->lv.size())
        return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        prof_collect(h);
        h->profiling = enable != 0;
        h->prof_kind = kernel_class;
        h->prof_level = level;
        for (auto& p : h->prof) p = ProfAcc{};
        return AMG_OK;
    });
}

amg_status amg_profile_read(amg_handle h, int32_t kernel_class, int32_t level, int64_t* count,
                            double* total_ms) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (kernel_class < 0 || kernel_class >= AMG_K_NUM || level < 0 || level >= (int)h->lv.size())
        return AMG_ERR_INVALID_ARG;
    return guarded(h, [&] {
        prof_collect(h);
        const ProfAcc& a = h->prof[(size_t)kernel_class * h->lv.size() + level];
        if (count) *count = a.count;
        if (total_ms) *total_ms = a.ms;
        return AMG_OK;
    });
}

amg_status amg_batch_bytes(amg_handle h, int32_t slots, int32_t precision, int64_t* bytes) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (!bytes || (slots != 4 && slots != 8 && slots != 16) || (precision != 32 && precision != 64))
        return AMG_ERR_INVALID_ARG;
    *bytes = batch_bytes(h, slots, precision);
    return AMG_OK;
}

amg_status amg_batch_create(amg_handle h, int32_t slots, int32_t precision, double rtol, int32_t maxit,
                            int32_t flags, amg_batch* out) {
    if (!out) return AMG_ERR_INVALID_ARG;
    *out = nullptr;
    if (!h || h->lv.empty() || h->batch) return AMG_ERR_STATE;
    if (gs_on(h)) {
        h->last_error = "hybrid Gauss-Seidel relaxation runs in the FP64 single-vector cycle only";
        return AMG_ERR_INVALID_ARG;
    }
    if ((slots != 4 && slots != 8 && slots != 16) || (precision != 32 && precision != 64) || !(rtol >= 0.0) ||
        maxit < 1 || (int64_t)h->lv[0].n * slots > INT32_MAX) {
        h->last_error = "invalid batch parameters (slots 4, 8 or 16; precision 32 or 64; maxit >= 1)";
        return AMG_ERR_INVALID_ARG;
    }
    amg_batch_ctx* e = new (std::nothrow) amg_batch_ctx();
    if (!e) return AMG_ERR_OUT_OF_MEMORY;
    e->h = h;
    e->k = slots;
    e->precision = precision;
    e->rtol = rtol;
    e->maxit = maxit;
    // stream capture needs a stream other than the null stream
    e->graphs = (flags & AMG_BATCH_GRAPHS) != 0 && h->stream != nullptr;
    amg_status st = guarded(h, [&] {
        const int64_t cnt = (int64_t)h->lv[0].n * slots;
        if (precision == 32) {
            ensure_fp32(h);
            ensure_block<float>(h, slots);
        } else {
            ensure_block<double>(h, slots);
        }
        ensure_block_cg(h, slots);
        e->B = dalloc_n<double>(h, cnt);
        e->X = dalloc_n<double>(h, cnt);
        // p must be finite in every column before its first use
        launch_fill_f64(cnt, h->bcg_p, 0.0, h->stream);
        launch_fill_f64(cnt, e->X, 0.0, h->stream);
        check_launch();
        HIP_CHECK(hipHostMalloc((void**)&e->down, sizeof(double) * S_COUNT, hipHostMallocDefault));
        HIP_CHECK(hipHostMalloc((void**)&e->up, sizeof(double) * (2 * kMaxBlockRhs + 1), hipHostMallocDefault));
        HIP_CHECK(hipEventCreateWithFlags(&e->done, hipEventDisableTiming));
        h->batch = e;
        return AMG_OK;
    });
    if (st != AMG_OK) {
        h->batch = e;
        destroy_batch(e);
        return st;
    }
    *out = e;
    return AMG_OK;
}

amg_status amg_batch_submit(amg_batch b, const double* rhs, int32_t* slot) {
    if (!b) return AMG_ERR_STATE;
    if (!rhs) return AMG_ERR_INVALID_ARG;
    amg_ctx* h = b->h;
    int c = 0;
    while (c < b->k && b->state[c] != kSlotFree) ++c;
    if (c == b->k) {
        h->last_error = "no free slot";
        return AMG_ERR_STATE;
    }
    return guarded(h, [&] {
        launch_block_column_in(h->lv[0].n, b->k, c, rhs, b->B, h->stream);
        check_launch();
        b->state[c] = kSlotPending;
        b->iters[c] = 0;
        b->rel[c] = 1.0;
        if (slot) *slot = c;
        return AMG_OK;
    });
}

amg_status amg_batch_step(amg_batch b, int32_t iters, int32_t* launched) {
    if (!b) return AMG_ERR_STATE;
    if (launched) *launched = 0;
    if (iters < 1) return AMG_ERR_INVALID_ARG;
    if (b->in_flight) {
        b->h->last_error = "the previous step has not been completed by amg_batch_poll";
        return AMG_ERR_STATE;
    }
    bool work = false;
    for (int c = 0; c < b->k; ++c) work = work || b->state[c] == kSlotPending || b->state[c] == kSlotActive;
    if (!work) return AMG_OK;
    return guarded(b->h, [&] {
        if (b->precision == 32) batch_step<float>(b, iters);
        else batch_step<double>(b, iters);
        if (launched) *launched = 1;
        return AMG_OK;
    });
}

amg_status amg_batch_poll(amg_batch b, int32_t wait, int32_t* finished) {
    if (!b) return AMG_ERR_STATE;
    if (!b->in_flight) {
        if (finished) std::fill(finished, finished + b->k, 0);
        return AMG_OK;
    }
    return guarded(b->h, [&] {
        if (wait) {
            HIP_CHECK(hipEventSynchronize(b->done));
        } else {
            const hipError_t q = hipEventQuery(b->done);
            if (q == hipErrorNotReady) return AMG_NOT_READY;
            HIP_CHECK(q);
        }
        batch_finish_step(b, finished);
        return AMG_OK;
    });
}

amg_status amg_batch_collect(amg_batch b, int32_t slot, double* x, int32_t* iters, double* relres,
                             int32_t* status) {
    if (!b) return AMG_ERR_STATE;
    if (slot < 0 || slot >= b->k || !x) return AMG_ERR_INVALID_ARG;
    if (b->state[slot] != kSlotDone) {
        b->h->last_error = "slot has not finished";
        return AMG_ERR_STATE;
    }
    return guarded(b->h, [&] {
        launch_block_column_out(b->h->lv[0].n, b->k, slot, b->X, x, b->h->stream);
        check_launch();
        if (iters) *iters = b->iters[slot];
        if (relres) *relres = b->rel[slot];
        if (status) *status = b->status[slot];
        b->state[slot] = kSlotFree;
        return AMG_OK;
    });
}

amg_status amg_batch_slots(amg_batch b, int32_t* state) {
    if (!b) return AMG_ERR_STATE;
    if (!state) return AMG_ERR_INVALID_ARG;
    for (int c = 0; c < b->k; ++c) state[c] = b->state[c];
    return AMG_OK;
}

void amg_batch_destroy(amg_batch b) { destroy_batch(b); }

amg_status amg_device_bytes(amg_handle h, int64_t* bytes) {
    if (!h || h->lv.empty()) return AMG_ERR_STATE;
    if (!bytes) return AMG_ERR_INVALID_ARG;
    int64_t t = 0;
    for (const auto& kv : h->blocks) t += (int64_t)kv.second;
    *bytes = t;
    return AMG_OK;
}

void amg_destroy(amg_handle h) { destroy(h); }

const char* amg_status_string(amg_status s) {
    switch (s) {
        case AMG_OK: return "ok";
        case AMG_NOTHING_TO_REINTRODUCE: return "nothing to reintroduce: every coarse gamma is 0";
        case AMG_NOT_READY: return "not ready: the batch step is still running";
        case AMG_ERR_INVALID_ARG: return "invalid argument";
        case AMG_ERR_BAD_MATRIX: return "matrix violates the input contract";
        case AMG_ERR_OUT_OF_MEMORY: return "out of device memory";
        case AMG_ERR_DEVICE: return "HIP error";
        case AMG_ERR_NOT_CONVERGED: return "not converged within maxit";
        case AMG_ERR_BREAKDOWN: return "breakdown (non-finite residual or p'Ap <= 0)";
        case AMG_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* amg_last_error(amg_handle h) { return h ? h->last_error.c_str() : setup_error().c_str(); }

}  // extern "C"
