// Exercise of the library's threaded host setup (Galerkin hierarchy) for the
// host sanitizer run (AddressSanitizer + UndefinedBehaviorSanitizer): input
// checks on good and malformed matrices, the Galerkin hierarchy and the
// non-Galerkin variant on 2D/3D Poisson and an irregular graph, with
// structural checks of every level.  Test infrastructure: built and run by
// tests/test_sanitizers_cpu.py; exits non-zero on a failed check.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_1512_04629_amd/csrc/host_setup.hpp"

using amg355::HostCsr;

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);   \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

static HostCsr poisson(int nx, int ny, int nz) {
    HostCsr a;
    a.rows = a.cols = nx * ny * nz;
    a.ptr.push_back(0);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int r = (k * ny + j) * nx + i;
                const int nb[7] = {r - nx * ny, r - nx, r - 1, r, r + 1, r + nx, r + nx * ny};
                const bool ok[7] = {k > 0, j > 0, i > 0, true, i < nx - 1, j < ny - 1, k < nz - 1};
                for (int t = 0; t < 7; ++t) {
                    if (!ok[t]) continue;
                    a.idx.push_back(nb[t]);
                    a.val.push_back(nb[t] == r ? (nz > 1 ? 6.0 : 4.0) : -1.0);
                }
                a.ptr.push_back((int32_t)a.idx.size());
            }
    return a;
}

// graph Laplacian of a ring with pseudo-random chords, diagonal shifted by one
static HostCsr graph(int n) {
    std::vector<std::vector<int>> nb(n);
    uint64_t z = 99;
    auto link = [&](int i, int j) {
        if (i == j) return;
        for (int q : nb[i]) if (q == j) return;
        nb[i].push_back(j);
        nb[j].push_back(i);
    };
    for (int i = 0; i < n; ++i) {
        link(i, (i + 1) % n);
        z = z * 6364136223846793005ull + 1442695040888963407ull;
        link(i, (int)((z >> 33) % (uint64_t)n));
    }
    HostCsr a;
    a.rows = a.cols = n;
    a.ptr.push_back(0);
    for (int i = 0; i < n; ++i) {
        std::vector<int> cols = nb[i];
        cols.push_back(i);
        std::sort(cols.begin(), cols.end());
        for (int c : cols) {
            a.idx.push_back(c);
            a.val.push_back(c == i ? (double)nb[i].size() + 1.0 : -1.0);
        }
        a.ptr.push_back((int32_t)a.idx.size());
    }
    return a;
}

static double at(const HostCsr& m, int i, int j) {
    for (int p = m.ptr[i]; p < m.ptr[i + 1]; ++p)
        if (m.idx[p] == j) return m.val[p];
    return 0.0;
}

static void check_structure(const HostCsr& m, int rows, int cols) {
    CHECK(m.rows == rows && m.cols == cols && (int)m.ptr.size() == rows + 1 && m.ptr[0] == 0);
    for (int i = 0; i < rows; ++i) {
        CHECK(m.ptr[i] <= m.ptr[i + 1]);
        for (int p = m.ptr[i]; p < m.ptr[i + 1]; ++p) {
            CHECK(m.idx[p] >= 0 && m.idx[p] < cols);
            if (p > m.ptr[i]) CHECK(m.idx[p] > m.idx[p - 1]);
        }
    }
}

static void hierarchy(const HostCsr& a, const std::vector<double>& ng) {
    std::string why;
    CHECK(amg355::check_input_matrix(a, why));
    amg355::SetupConfig cfg;
    cfg.max_coarse = 20;
    cfg.nongalerkin_gamma = ng;
    std::vector<amg355::HostLevel> lv;
    CHECK(amg355::build_galerkin_hierarchy(a, cfg, lv, why));
    CHECK(lv.size() >= 2);
    for (size_t l = 0; l < lv.size(); ++l) {
        const HostCsr& A = lv[l].A;
        check_structure(A, A.rows, A.rows);
        for (int i = 0; i < A.rows; ++i)
            for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const double u = A.val[p], w = at(A, A.idx[p], i);
                CHECK(std::memcmp(&u, &w, sizeof(double)) == 0);   // bitwise symmetric
            }
        if (l + 1 < lv.size()) {
            const int nc = lv[l + 1].A.rows;
            check_structure(lv[l].P, A.rows, nc);
            check_structure(lv[l].R, nc, A.rows);
            HostCsr t = amg355::transpose_csr(lv[l].P);
            CHECK(t.ptr == lv[l].R.ptr && t.idx == lv[l].R.idx);
            CHECK((int)lv[l].c_points.size() == nc && (int)lv[l].split.size() == A.rows);
            for (int c = 0; c < nc; ++c) {
                CHECK(lv[l].split[lv[l].c_points[c]] == 1);
                if (c) CHECK(lv[l].c_points[c] > lv[l].c_points[c - 1]);
                CHECK(at(lv[l].P, lv[l].c_points[c], c) == 1.0);
            }
        }
    }
}

int main() {
    const std::vector<double> galerkin, nongalerkin = {0.0, 0.0, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1};
    for (const HostCsr& a : {poisson(24, 20, 1), poisson(10, 9, 8), graph(900)}) {
        hierarchy(a, galerkin);
        hierarchy(a, nongalerkin);
    }
    // malformed inputs are refused with a reason
    std::string why;
    HostCsr bad = poisson(8, 8, 1);
    bad.val[1] = -0.5;
    CHECK(!amg355::check_input_matrix(bad, why) && !why.empty());
    bad = poisson(8, 8, 1);
    std::swap(bad.idx[0], bad.idx[1]);
    CHECK(!amg355::check_input_matrix(bad, why));
    bad = poisson(8, 8, 1);
    bad.val[0] = -4.0;
    CHECK(!amg355::check_input_matrix(bad, why));
    bad = poisson(8, 8, 1);
    bad.idx[2] = 1000;
    CHECK(!amg355::check_input_matrix(bad, why));
    std::printf("host setup sanitizer exercise: ok\n");
    return 0;
}
