// Host-side Galerkin setup: strength, Ruge-Stueben first-pass split, direct
// interpolation and the Galerkin product, in a fixed order so that the
// coarse operators are reproducible bit for bit.
//
// Section 2 (amg_setup) names the three steps (strength, interpolation,
// P^T A P) and defers their formulas to the classical Ruge-Stueben method;
// the choices fixed here are:
//   strength:  S_ij = 1 iff j != i and -a_ij >= fl(theta * max_{k!=i}(-a_ik)),
//              only when that maximum is positive;
//   split:     repeatedly take the undecided point of largest measure
//              lambda (ties: smallest index), where lambda_k counts the points
//              that depend strongly on k, undecided ones once and F points
//              twice; a point whose measure is 0 and that already depends on a
//              C point becomes F, otherwise it becomes C and every undecided
//              point depending on it becomes F;
//   direct interpolation: w_ij = -(alpha a_ij) / d for strong C neighbours
//              j, alpha = (sum of negative off-diagonals) / (sum of a_ij over
//              strong C neighbours), d = a_ii + sum of positive off-diagonals,
//              every sum taken in ascending column order;
//   Galerkin:  T = A P, T[k,J] summed over ascending l; C = P^T T, C[I,J]
//              summed over ascending k; first term assigned; no fused
//              multiply-add; A_c = (C + C^T) / 2 entrywise.
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

namespace amg355 {

namespace {

template <class F>
void parallel_rows(int n, F&& body) {
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
    if (n < 4096 || nt <= 1) {
        body(0, n, 0);
        return;
    }
    std::vector<std::thread> pool;
    int chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        int lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        pool.emplace_back([&, lo, hi, t] { body(lo, hi, t); });
    }
    for (auto& th : pool) th.join();
}

int64_t lower_bound_col(const HostCsr& m, int row, int col) {
    auto b = m.idx.begin() + m.ptr[row], e = m.idx.begin() + m.ptr[row + 1];
    auto it = std::lower_bound(b, e, col);
    return (it != e && *it == col) ? (int64_t)(it - m.idx.begin()) : -1;
}

// Strength pattern: per row, the columns of strong negative couplings.
HostCsr strength_pattern(const HostCsr& a, double theta) {
    HostCsr s;
    s.rows = s.cols = a.rows;
    s.ptr.assign(a.rows + 1, 0);
    std::vector<double> thr(a.rows, 0.0);
    std::vector<char> has(a.rows, 0);
    for (int i = 0; i < a.rows; ++i) {
        double big = 0.0;
        for (int p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
            if (a.idx[p] != i) big = std::max(big, -a.val[p]);
        if (big > 0.0) {
            has[i] = 1;
            thr[i] = theta * big;
            int c = 0;
            for (int p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
                if (a.idx[p] != i && -a.val[p] >= thr[i]) ++c;
            s.ptr[i + 1] = c;
        }
    }
    for (int i = 0; i < a.rows; ++i) s.ptr[i + 1] += s.ptr[i];
    s.idx.resize(s.ptr.back());
    for (int i = 0; i < a.rows; ++i) {
        if (!has[i]) continue;
        int w = s.ptr[i];
        for (int p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
            if (a.idx[p] != i && -a.val[p] >= thr[i]) s.idx[w++] = a.idx[p];
    }
    return s;
}

// Tournament tree over point indices returning the undecided point with the
// largest measure, ties resolved to the smallest index.  Decided points carry
// key -1.
class MeasureTree {
public:
    explicit MeasureTree(const std::vector<int>& key) : n_((int)key.size()) {
        size_ = 1;
        while (size_ < n_) size_ <<= 1;
        key_.assign(2 * size_, -1);
        who_.assign(2 * size_, -1);
        for (int i = 0; i < n_; ++i) { key_[size_ + i] = key[i]; who_[size_ + i] = i; }
        for (int v = size_ - 1; v >= 1; --v) pull(v);
    }
    void set(int i, int k) {
        int v = size_ + i;
        key_[v] = k;
        // an ancestor depends only on its children's winners: stop where the
        // winner of a subtree is unchanged
        for (v >>= 1; v >= 1; v >>= 1) {
            const int old_key = key_[v], old_who = who_[v];
            pull(v);
            if (key_[v] == old_key && who_[v] == old_who) break;
        }
    }
    int top_key() const { return key_[1]; }
    int top() const { return who_[1]; }

private:
    void pull(int v) {
        int l = 2 * v, r = l + 1;
        // left subtree holds smaller indices: it wins ties
        int w = (key_[l] >= key_[r]) ? l : r;
        key_[v] = key_[w];
        who_[v] = who_[w];
    }
    int n_, size_;
    std::vector<int> key_, who_;
};

std::vector<int32_t> rs_first_pass(const HostCsr& s) {
    const int n = s.rows;
    HostCsr st = transpose_csr(s);     // row i of st: points depending strongly on i
    enum : int8_t { UND = 0, CPT = 1, FPT = 2 };
    std::vector<int8_t> state(n, UND);
    std::vector<int> measure(n);
    for (int i = 0; i < n; ++i) {
        measure[i] = st.ptr[i + 1] - st.ptr[i];
        if (s.ptr[i + 1] == s.ptr[i] && measure[i] == 0) state[i] = FPT;
    }
    std::vector<int> key(n);
    for (int i = 0; i < n; ++i) key[i] = state[i] == UND ? measure[i] : -1;
    MeasureTree tree(key);
    std::vector<int> fresh_f;
    while (tree.top_key() >= 0) {
        int i = tree.top();
        fresh_f.clear();
        bool to_f = false;
        if (measure[i] == 0) {
            for (int p = s.ptr[i]; p < s.ptr[i + 1] && !to_f; ++p) to_f = state[s.idx[p]] == CPT;
        }
        if (to_f) {
            state[i] = FPT;
            fresh_f.push_back(i);
        } else {
            state[i] = CPT;
            for (int p = st.ptr[i]; p < st.ptr[i + 1]; ++p) {
                int j = st.idx[p];
                if (state[j] == UND) { state[j] = FPT; fresh_f.push_back(j); tree.set(j, -1); }
            }
        }
        tree.set(i, -1);
        for (int j : fresh_f)
            for (int p = s.ptr[j]; p < s.ptr[j + 1]; ++p) {
                int k = s.idx[p];
                if (state[k] == UND) tree.set(k, ++measure[k]);
            }
        if (state[i] == CPT)
            for (int p = s.ptr[i]; p < s.ptr[i + 1]; ++p) {
                int k = s.idx[p];
                if (state[k] == UND) tree.set(k, --measure[k]);
            }
    }
    std::vector<int32_t> split(n);
    for (int i = 0; i < n; ++i) split[i] = state[i] == CPT ? 1 : 0;
    return split;
}

HostCsr direct_interpolation(const HostCsr& a, const HostCsr& s, const std::vector<int32_t>& split,
                             const std::vector<int32_t>& coarse_of, int nc) {
    const int n = a.rows;
    HostCsr P;
    P.rows = n;
    P.cols = nc;
    P.ptr.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        if (split[i]) { P.ptr[i + 1] = 1; continue; }
        int c = 0;
        for (int p = s.ptr[i]; p < s.ptr[i + 1]; ++p) c += split[s.idx[p]];
        P.ptr[i + 1] = c;
    }
    for (int i = 0; i < n; ++i) P.ptr[i + 1] += P.ptr[i];
    P.idx.resize(P.ptr.back());
    P.val.resize(P.ptr.back());
    parallel_rows(n, [&](int lo, int hi, int) {
        for (int i = lo; i < hi; ++i) {
            int w = P.ptr[i];
            if (split[i]) { P.idx[w] = coarse_of[i]; P.val[w] = 1.0; continue; }
            if (P.ptr[i + 1] == w) continue;
            double neg = 0.0, dsum = 0.0, strong_c = 0.0;
            int64_t dpos = lower_bound_col(a, i, i);
            dsum = a.val[dpos];
            for (int p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
                if (a.idx[p] == i) continue;
                double v = a.val[p];
                if (v < 0.0) neg = neg + v;
                else if (v > 0.0) dsum = dsum + v;
            }
            // strong C neighbours: merge the sorted S row with the A row
            int q = a.ptr[i];
            for (int p = s.ptr[i]; p < s.ptr[i + 1]; ++p) {
                int j = s.idx[p];
                while (a.idx[q] < j) ++q;
                if (split[j]) strong_c = strong_c + a.val[q];
            }
            double alpha = neg / strong_c;
            q = a.ptr[i];
            for (int p = s.ptr[i]; p < s.ptr[i + 1]; ++p) {
                int j = s.idx[p];
                while (a.idx[q] < j) ++q;
                if (!split[j]) continue;
                double t = alpha * a.val[q];
                P.idx[w] = coarse_of[j];
                P.val[w] = -t / dsum;
                ++w;
            }
        }
    });
    return P;
}

// Z = X * Y with every Z[i,J] summed over X's row i in ascending order of
// its columns, the first product assigned.  Two passes: symbolic row sizes,
// then values; rows are independent and split across threads.
HostCsr ordered_product(const HostCsr& X, const HostCsr& Y) {
    const int nr = X.rows, nc = Y.cols;
    HostCsr Z;
    Z.rows = nr;
    Z.cols = nc;
    Z.ptr.assign(nr + 1, 0);
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
    std::vector<std::vector<int>> stamp(nt, std::vector<int>());
    parallel_rows(nr, [&](int lo, int hi, int t) {
        auto& seen = stamp[t];
        seen.assign(nc, -1);
        for (int i = lo; i < hi; ++i) {
            int c = 0;
            for (int p = X.ptr[i]; p < X.ptr[i + 1]; ++p) {
                int l = X.idx[p];
                for (int q = Y.ptr[l]; q < Y.ptr[l + 1]; ++q)
                    if (seen[Y.idx[q]] != i) { seen[Y.idx[q]] = i; ++c; }
            }
            Z.ptr[i + 1] = c;
        }
    });
    for (int i = 0; i < nr; ++i) Z.ptr[i + 1] += Z.ptr[i];
    Z.idx.resize(Z.ptr.back());
    Z.val.resize(Z.ptr.back());
    parallel_rows(nr, [&](int lo, int hi, int t) {
        auto& seen = stamp[t];
        std::fill(seen.begin(), seen.end(), -1);
        std::vector<double> acc(nc);
        std::vector<int> cols;
        for (int i = lo; i < hi; ++i) {
            cols.clear();
            for (int p = X.ptr[i]; p < X.ptr[i + 1]; ++p) {
                int l = X.idx[p];
                double xv = X.val[p];
                for (int q = Y.ptr[l]; q < Y.ptr[l + 1]; ++q) {
                    int J = Y.idx[q];
                    double prod = xv * Y.val[q];
                    if (seen[J] != i) { seen[J] = i; acc[J] = prod; cols.push_back(J); }
                    else acc[J] = acc[J] + prod;
                }
            }
            std::sort(cols.begin(), cols.end());
            int w = Z.ptr[i];
            for (int J : cols) { Z.idx[w] = J; Z.val[w] = acc[J]; ++w; }
        }
    });
    return Z;
}

// A_c = (C + C^T)/2 on the structurally symmetric pattern of C, using the
// position of each entry's mirror from a counting transpose.
bool symmetrize(HostCsr& c, std::string& why) {
    const int n = c.rows;
    std::vector<int64_t> mirror(c.nnz());
    std::vector<int64_t> fill(c.ptr.begin(), c.ptr.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int p = c.ptr[i]; p < c.ptr[i + 1]; ++p) {
            int j = c.idx[p];
            int64_t q = fill[j]++;
            if (q >= c.ptr[j + 1] || c.idx[q] != i) {
                why = "coarse operator pattern is not structurally symmetric";
                return false;
            }
            mirror[q] = p;      // entry q = (j,i) mirrors p = (i,j)
        }
    std::vector<double> out(c.nnz());
    for (int64_t p = 0; p < c.nnz(); ++p) out[p] = 0.5 * (c.val[p] + c.val[mirror[p]]);
    c.val.swap(out);
    return true;
}

}  // namespace

std::vector<int32_t> ruge_stueben_split(const HostCsr& s) { return rs_first_pass(s); }

HostCsr transpose_csr(const HostCsr& p) {
    HostCsr t;
    t.rows = p.cols;
    t.cols = p.rows;
    t.ptr.assign(p.cols + 1, 0);
    for (int64_t q = 0; q < p.nnz(); ++q) t.ptr[p.idx[q] + 1]++;
    for (int i = 0; i < p.cols; ++i) t.ptr[i + 1] += t.ptr[i];
    t.idx.resize(p.nnz());
    t.val.resize(p.val.empty() ? 0 : p.nnz());
    std::vector<int32_t> fill(t.ptr.begin(), t.ptr.end() - 1);
    for (int i = 0; i < p.rows; ++i)
        for (int q = p.ptr[i]; q < p.ptr[i + 1]; ++q) {
            int w = fill[p.idx[q]]++;
            t.idx[w] = i;
            if (!p.val.empty()) t.val[w] = p.val[q];
        }
    return t;
}

bool check_input_matrix(const HostCsr& a, std::string& why) {
    const int n = a.rows;
    if (n <= 0 || a.cols != n || (int)a.ptr.size() != n + 1 || a.ptr[0] != 0) {
        why = "matrix must be square with n > 0 and row_ptr[0] == 0";
        return false;
    }
    for (int i = 0; i < n; ++i) {
        if (a.ptr[i + 1] < a.ptr[i]) { why = "row_ptr is not non-decreasing"; return false; }
        bool diag = false;
        for (int p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
            int j = a.idx[p];
            if (j < 0 || j >= n) { why = "column index out of range in row " + std::to_string(i); return false; }
            if (p > a.ptr[i] && j <= a.idx[p - 1]) { why = "columns not strictly ascending in row " + std::to_string(i); return false; }
            if (!std::isfinite(a.val[p])) { why = "non-finite value in row " + std::to_string(i); return false; }
            if (j == i) {
                diag = true;
                if (!(a.val[p] > 0.0)) { why = "non-positive diagonal in row " + std::to_string(i); return false; }
            }
        }
        if (!diag) { why = "missing diagonal in row " + std::to_string(i); return false; }
    }
    HostCsr t = transpose_csr(a);
    if (t.ptr != a.ptr || t.idx != a.idx ||
        std::memcmp(t.val.data(), a.val.data(), sizeof(double) * a.val.size()) != 0) {
        why = "matrix is not bitwise symmetric";
        return false;
    }
    return true;
}

// Sparsifies the coarse product C of the fine operator A and interpolation P
// (coarse point I is fine point cpts[I]) with tolerance gamma: minimal pattern
// M = edges(Phat^T A P + P^T A Phat) (structural), keep (i,j) iff i == j, in
// M, |c_ij| >= gamma m_i or |c_ij| >= gamma m_j with m_i = max_{k!=i} |c_ik|
// (Algorithm 3's symmetric keep set), dropped entries added to the diagonal
// in ascending column order (Algorithm 3b).
static bool sparsify_coarse(HostCsr& C, const HostCsr& A, const HostCsr& P, const std::vector<int32_t>& cpts,
                            double gamma, std::string& why) {
    const int nc = C.rows;
    std::vector<uint8_t> in_m(C.nnz(), 0);
    auto pos = [&](int i, int j) -> int64_t {
        const int32_t* b = C.idx.data() + C.ptr[i];
        const int32_t* e = C.idx.data() + C.ptr[i + 1];
        const int32_t* it = std::lower_bound(b, e, j);
        return (it != e && *it == j) ? (int64_t)(it - C.idx.data()) : -1;
    };
    for (int I = 0; I < nc; ++I) {
        const int f = cpts[I];
        for (int32_t p = A.ptr[f]; p < A.ptr[f + 1]; ++p) {
            const int l = A.idx[p];
            for (int32_t q = P.ptr[l]; q < P.ptr[l + 1]; ++q) {
                const int J = P.idx[q];
                const int64_t a = pos(I, J), b = pos(J, I);
                if (a < 0 || b < 0) {
                    why = "minimal pattern outside the coarse product";
                    return false;
                }
                in_m[a] = in_m[b] = 1;
            }
        }
    }
    std::vector<double> m(nc, 0.0);
    for (int i = 0; i < nc; ++i)
        for (int32_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p)
            if (C.idx[p] != i) m[i] = std::max(m[i], std::fabs(C.val[p]));
    HostCsr out;
    out.rows = out.cols = nc;
    out.ptr.assign(nc + 1, 0);
    out.idx.reserve(C.idx.size());
    out.val.reserve(C.val.size());
    for (int i = 0; i < nc; ++i) {
        double d = 0.0;
        int64_t dpos = -1;
        for (int32_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p)
            if (C.idx[p] == i) d = C.val[p];
        for (int32_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p) {
            const int j = C.idx[p];
            const double av = std::fabs(C.val[p]);
            const bool keep = j == i || in_m[p] || av >= gamma * m[i] || av >= gamma * m[j];
            if (!keep) {
                d += C.val[p];
                continue;
            }
            if (j == i) dpos = (int64_t)out.idx.size();
            out.idx.push_back(j);
            out.val.push_back(C.val[p]);
        }
        if (dpos >= 0) out.val[dpos] = d;
        out.ptr[i + 1] = (int32_t)out.idx.size();
    }
    C = std::move(out);
    return true;
}

bool build_galerkin_hierarchy(const HostCsr& a, const SetupConfig& cfg,
                              std::vector<HostLevel>& levels, std::string& why) {
    levels.clear();
    levels.emplace_back();
    levels[0].A = a;
    while (levels.back().A.rows > cfg.max_coarse && (int)levels.size() < cfg.max_levels) {
        HostLevel& cur = levels.back();
        const int n = cur.A.rows;
        HostCsr s = strength_pattern(cur.A, cfg.theta);
        std::vector<int32_t> split = rs_first_pass(s);
        std::vector<int32_t> coarse_of(n, -1);
        std::vector<int32_t> cpts;
        for (int i = 0; i < n; ++i)
            if (split[i]) { coarse_of[i] = (int32_t)cpts.size(); cpts.push_back(i); }
        const int nc = (int)cpts.size();
        if (nc == 0 || nc == n) break;
        cur.split = std::move(split);
        cur.c_points = std::move(cpts);
        cur.P = direct_interpolation(cur.A, s, cur.split, coarse_of, nc);
        cur.R = transpose_csr(cur.P);
        HostCsr T = ordered_product(cur.A, cur.P);
        HostCsr C = ordered_product(cur.R, T);
        if ((int64_t)C.nnz() > INT32_MAX) { why = "coarse operator exceeds int32 nonzeros"; return false; }
        if (!symmetrize(C, why)) return false;
        const size_t lc = levels.size();   // index of the level C forms
        if (lc < cfg.nongalerkin_gamma.size() && cfg.nongalerkin_gamma[lc] > 0.0 &&
            !sparsify_coarse(C, cur.A, cur.P, cur.c_points, cfg.nongalerkin_gamma[lc], why))
            return false;
        HostLevel next;
        next.A = std::move(C);
        levels.push_back(std::move(next));
    }
    return true;
}

}  // namespace amg355
