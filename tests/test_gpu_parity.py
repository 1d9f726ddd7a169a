"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars:
  * setup, C/F split, P, R, A_l, minimal pattern M, row maxima, keep flags,
    sparsified pattern and kept off-diagonal values: bit-exact;
  * lumped diagonal: |d_gpu - d_or| <= 1e-13 (|a_ii| + sum_dropped |a_ij|);
  * single kernels: |y_gpu - y_or|_i <= 1e-13 (|M| |v| + |u|)_i;
  * V-cycle: normwise 1e-12;
  * solves: equal iteration counts, ||x_gpu - x_or|| <= 1e-10 ||x_or||,
    |relres_gpu - relres_or| <= 1e-10, both converged.
"""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    amg.load_library()
    return amg


def _sp(m):
    import scipy.sparse as sp
    return sp.csr_matrix((m.val, m.col, m.row_ptr), shape=(m.nrows, m.ncols))


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


PROBLEMS = {
    "poisson2d_64": lambda: I.poisson2d(64),
    "poisson3d_20": lambda: I.poisson3d(20),
    "aniso2d_48": lambda: I.aniso2d(48),
    "fv3d_12": lambda: I.fv3d_lognormal(12),
    "graph_3000": lambda: I.random_graph_laplacian(3000),
}


def both(A, **kw):
    from paper_1512_04629_amd import amg
    from oracle import oracle as O
    return amg.Hierarchy(A, **kw), O.OracleAMG(A, **kw)


def same_csr(g, o):
    nr, nc, rp, ci, v = g
    return (np.array_equal(rp, o.row_ptr) and np.array_equal(ci, o.col)
            and v.tobytes() == o.val.tobytes())


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_setup_bitwise(lib, name):
    A = PROBLEMS[name]()
    g, o = both(A)
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        assert same_csr(g.export(l, "A"), o.export(l, "A")), l
        if l < o.nlev - 1:
            assert same_csr(g.export(l, "P"), o.export(l, "P")), l
            assert same_csr(g.export(l, "R"), o.export(l, "R")), l
            assert np.array_equal(g.split(l), o.cf(l)), l


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.01, 0.1, 1.0])
def test_sparsify_parity(lib, name, gamma):
    A = PROBLEMS[name]()
    g, o = both(A)
    gam = [0.0] + [gamma] * (o.nlev - 1)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    for l in range(1, o.nlev):
        assert np.array_equal(g.mask(l, "M"), o.mask(l, "M")), ("M", l)
        assert g.vector(l, "ROWMAX").tobytes() == o.rowmax(l).tobytes(), ("rowmax", l)
        assert np.array_equal(g.mask(l, "KEEP"), o.mask(l, "KEEP")), ("keep", l)
        nr, nc, rp, ci, v = g.export(l, "AHAT")
        ref = o.export(l, "AHAT")
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col), ("pattern", l)
        rows = np.repeat(np.arange(nr), np.diff(rp))
        off = rows != ci
        assert v[off].tobytes() == ref.val[off].tobytes(), ("offdiag", l)
        # lumped diagonal within the rounding of the dropped sum
        Ad = o.export(l, "A")
        arow = np.repeat(np.arange(Ad.nrows), np.diff(Ad.row_ptr))
        keep = o.mask(l, "KEEP").astype(bool)
        dropped_abs = np.bincount(arow[~keep], weights=np.abs(Ad.val[~keep]), minlength=nr)
        aii = Ad.val[arow == Ad.col]
        d_g, d_o = v[~off], ref.val[~off]
        assert np.all(np.abs(d_g - d_o) <= 1e-13 * (np.abs(aii) + dropped_abs)), ("diag", l)
        # dinv is the reciprocal of the device's own lumped diagonal (that
        # diagonal is checked against the oracle just above)
        dinv = g.vector(l, "DINV")
        assert np.all(np.abs(dinv - 1.0 / d_g) <= 2.3e-16 * np.abs(1.0 / d_g))
        assert g.gamma(l) == o.gamma(l)


def test_sparsify_gamma_zero_is_galerkin_and_run_twice_is_deterministic(lib):
    A = I.aniso2d(64)
    from paper_1512_04629_amd import amg
    g = amg.Hierarchy(A)
    g.sparsify(0.1, 2)
    first = [g.export(l, "AHAT") for l in range(g.nlev)]
    g.sparsify(0.1, 2)
    for l in range(g.nlev):
        a, b = first[l], g.export(l, "AHAT")
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and a[4].tobytes() == b[4].tobytes()
    g.sparsify(0.0, 1)
    for l in range(g.nlev):
        a, b = g.export(l, "A"), g.export(l, "AHAT")
        assert np.array_equal(a[2], b[2]) and a[4].tobytes() == b[4].tobytes()


def test_reintroduce_ladder_and_parity(lib):
    A = I.poisson2d(160)     # seven levels: the hierarchy of the Section 6 Example
    g, o = both(A)
    assert g.nlev == 7
    start = [0.0, 0.0, 0.01, 0.1, 1.0, 1.0, 1.0]
    g.sparsify_levels(start)
    o.sparsify(start)
    for step in range(12):
        rg = g.reintroduce(s=2)
        ro = o.reintroduce(s=2)
        assert rg == ro
        for l in range(1, 7):
            assert g.gamma(l) == o.gamma(l)
            nr, nc, rp, ci, v = g.export(l, "AHAT")
            ref = o.export(l, "AHAT")
            assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col)
        if rg[0] == 1:
            break
    assert rg == (1, -1)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_level_kernels(lib, name):
    A = PROBLEMS[name]()
    g, o = both(A)
    gam = [0.0, 0.0] + [0.1] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    rng = np.random.default_rng(0)
    for l in range(o.nlev):
        n = o.sizes(l)["n"]
        b = rng.uniform(-1, 1, n)
        x = rng.uniform(-1, 1, n)
        Ah = _sp(o.export(l, "AHAT"))
        absAx = abs(Ah) @ np.abs(x)
        # residual
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        g.level_op(l, "RESIDUAL", dev(b), dev(x), out)
        ref = o.level_op(l, 0, b, x, n)
        assert np.all(np.abs(host(out) - ref) <= 1e-13 * (absAx + np.abs(b)))
        # Jacobi sweep
        g.level_op(l, "JACOBI", dev(b), dev(x), out)
        ref = o.level_op(l, 1, b, x, n)
        d = np.abs(Ah.diagonal())
        assert np.all(np.abs(host(out) - ref) <= 1e-13 * ((absAx + np.abs(b)) / d + np.abs(x)))
        if l < o.nlev - 1:
            nc = o.sizes(l)["n_coarse"]
            P = _sp(o.export(l, "P"))
            out_c = torch.empty(nc, dtype=torch.float64, device="cuda")
            g.level_op(l, "RESTRICT", dev(x), None, out_c)
            ref = o.level_op(l, 2, x, None, nc)
            assert np.all(np.abs(host(out_c) - ref) <= 1e-13 * (abs(P.T) @ np.abs(x)))
            xc = rng.uniform(-1, 1, nc)
            g.level_op(l, "INTERPOLATE", dev(xc), dev(x), out)
            ref = o.level_op(l, 3, xc, x, n)
            assert np.all(np.abs(host(out) - ref) <= 1e-13 * (abs(P) @ np.abs(xc) + np.abs(x)))
    L = o.nlev - 1
    nL = o.sizes(L)["n"]
    bL = rng.uniform(-1, 1, nL)
    out = torch.empty(nL, dtype=torch.float64, device="cuda")
    g.level_op(L, "COARSE_SOLVE", dev(bL), None, out)
    ref = o.level_op(L, 4, bL, None, nL)
    assert np.linalg.norm(host(out) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_vcycle_parity(lib, name):
    A = PROBLEMS[name]()
    g, o = both(A)
    gam = [0.0, 0.0] + [0.1] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    b = I.rhs(A.n, 7)
    x0 = I.rhs(A.n, 8)
    for xin in (np.zeros(A.n), x0):
        xd = dev(xin)
        g.vcycle(dev(b), xd)
        ref = o.vcycle(b, xin)
        assert np.linalg.norm(host(xd) - ref) <= 1e-12 * np.linalg.norm(ref)


def _solve_pair(A, gam, b, **kw):
    g, o = both(A)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(dev(b), xd, **kw)
    xo, ro = o.solve(b, **kw)
    return host(xd), rg, xo, ro, g, o


def crossing_margin(res, tol):
    """Smallest |log(rho_k / tol)| over the stop tests a solve took, rho_k the
    relative residual after iteration k: how far the iteration count is from
    flipping under a rounding-level change of the residuals."""
    rel = np.asarray(res.hist[1:], float) / res.hist[0]
    rel = rel[np.isfinite(rel) & (rel > 0)]
    return float(np.min(np.abs(np.log(rel / tol)))) if rel.size else float("inf")


def _assert_solve_parity(xg, rg, xo, ro, tol=None):
    if tol is not None:
        m = crossing_margin(ro, tol)
        print(f"crossing margin |log(rho/tol)| = {m:.3e} over {ro.iters} iterations", flush=True)
        if m < 1e-9:
            pytest.skip(f"ill-conditioned for count parity: crossing margin {m:.2e} < 1e-9")
    assert rg.status == ro.status
    assert rg.iters == ro.iters, (rg.iters, ro.iters, rg.hist, ro.hist)
    assert rg.reintroductions == ro.reintroductions and rg.restarts == ro.restarts
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    assert abs(rg.relres - ro.relres) <= 1e-10
    assert np.all(np.abs(rg.hist - ro.hist) <= 1e-9 * ro.hist[0])


def test_config1_stationary_poisson2d_64(lib):
    # 2D Poisson 64x64, gamma 0.01 on levels >= 2, stationary V(1,1) to 1e-8
    A = I.poisson2d(64)
    b = I.rhs(A.n, 1)
    for gamma in (0.0, 0.01):
        gam = [0.0, 0.0] + [gamma] * 10
        xg, rg, xo, ro, g, o = _solve_pair(A, gam, b, method=0, tol=1e-8, maxit=100)
        assert ro.converged and rg.converged
        _assert_solve_parity(xg, rg, xo, ro, 1e-8)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("method", [0, 1])
def test_solve_parity(lib, name, method):
    A = PROBLEMS[name]()
    b = I.rhs(A.n, 2)
    from oracle import oracle as O
    nlev = O.OracleAMG(A).nlev
    gam = [0.0, 0.0] + [0.1] * (nlev - 2)
    xg, rg, xo, ro, g, o = _solve_pair(A, gam, b, method=method, tol=1e-8, maxit=300)
    if ro.status == -5:
        pytest.skip("oracle did not converge in 300 iterations for this case")
    _assert_solve_parity(xg, rg, xo, ro, 1e-8)


def test_adaptive_forced_reintroduction(lib):
    A = I.poisson3d(16)
    b = I.rhs(A.n, 2)
    from oracle import oracle as O
    nlev = O.OracleAMG(A).nlev
    gam = [0.0, 0.0] + [1.0] * (nlev - 2)
    xg, rg, xo, ro, g, o = _solve_pair(A, gam, b, method=1, tol=1e-12, maxit=200, adaptive=True,
                                       k=2, s=1, rho_max=0.0)
    assert ro.reintroductions >= 3
    _assert_solve_parity(xg, rg, xo, ro, 1e-12)
    for l in range(nlev):
        assert g.gamma(l) == o.gamma(l)


def test_adaptive_diverged_window_reverts(lib):
    A = I.random_graph_laplacian(5000)
    b = I.rhs(A.n, 1)
    from oracle import oracle as O
    nlev = O.OracleAMG(A).nlev
    gam = [0.0] + [1.0] * (nlev - 1)
    xg, rg, xo, ro, g, o = _solve_pair(A, gam, b, method=0, tol=1e-14, maxit=5, adaptive=True, k=3, s=1)
    assert ro.reintroductions == 1 and ro.status == -5
    _assert_solve_parity(xg, rg, xo, ro, 1e-14)


def test_single_level_hierarchy(lib):
    A = I.poisson2d(6)     # n = 36 <= 49: the coarsest level is the fine level
    b = I.rhs(A.n, 3)
    xg, rg, xo, ro, g, o = _solve_pair(A, [0.0], b, method=1, tol=1e-10, maxit=10)
    assert g.nlev == 1
    assert rg.iters == ro.iters == 1
    assert np.linalg.norm(xg - xo) <= 1e-12 * np.linalg.norm(xo)


def test_error_statuses(lib):
    from paper_1512_04629_amd import amg
    A = I.poisson2d(16)
    bad = I.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.val[1] = -0.5
    with pytest.raises(amg.AmgError) as e:
        amg.Hierarchy(bad)
    assert e.value.status == -2 and "symmetric" in str(e.value)
    g = amg.Hierarchy(A)
    with pytest.raises(amg.AmgError) as e:
        g.sparsify(1.5, 2)
    assert e.value.status == -1
    b = I.rhs(A.n, 1)
    r = g.solve(dev(b), torch.zeros(A.n, dtype=torch.float64, device="cuda"), tol=1e-14, maxit=1)
    assert r.status == -5 and r.iters == 1
    bb = b.copy(); bb[3] = np.nan
    r = g.solve(dev(bb), torch.zeros(A.n, dtype=torch.float64, device="cuda"))
    assert r.status == -6
    r = g.solve(dev(np.zeros(A.n)), torch.zeros(A.n, dtype=torch.float64, device="cuda"))
    assert r.status == 0 and r.iters == 0
    assert g.reintroduce(1) == (1, -1)


def test_allocator_failure_is_reported(lib):
    """An allocator that returns NULL makes setup fail with OUT_OF_MEMORY and
    leaves no handle (forced from the host; no kernel misbehaves)."""
    import ctypes as C
    from paper_1512_04629_amd import amg
    A = I.poisson2d(16)
    lib_ = amg.load_library()
    null_alloc = amg.ALLOC_FN(lambda n, s, u: None)
    nop_free = amg.FREE_FN(lambda p, n, s, u: None)
    out = C.c_void_p()
    st = lib_.amg_setup_from_csr(A.n, A.row_ptr.ctypes.data, A.col.ctypes.data, A.val.ctypes.data,
                                 None, None, null_alloc, nop_free, None, C.byref(out))
    assert st == -3 and out.value is None
    assert b"allocation" in lib_.amg_last_error(None)


LARGE = {
    # large enough that the fine operators take the LDS-staged kernel
    "poisson3d_64": lambda: I.poisson3d(64),
    "aniso2d_512": lambda: I.aniso2d(512),
}


@pytest.mark.parametrize("name", sorted(LARGE))
def test_level_kernels_large(lib, name):
    A = LARGE[name]()
    g, o = both(A)
    gam = [0.0, 0.0] + [0.1] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    rng = np.random.default_rng(1)
    for l in range(min(3, o.nlev - 1)):
        n, nc = o.sizes(l)["n"], o.sizes(l)["n_coarse"]
        b, x, xc = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, nc)
        Ah = _sp(o.export(l, "AHAT"))
        P = _sp(o.export(l, "P"))
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        out_c = torch.empty(nc, dtype=torch.float64, device="cuda")
        g.level_op(l, "RESIDUAL", dev(b), dev(x), out)
        assert np.all(np.abs(host(out) - o.level_op(l, 0, b, x, n)) <= 1e-13 * (abs(Ah) @ np.abs(x) + np.abs(b)))
        g.level_op(l, "JACOBI", dev(b), dev(x), out)
        bound = 1e-13 * ((abs(Ah) @ np.abs(x) + np.abs(b)) / np.abs(Ah.diagonal()) + np.abs(x))
        assert np.all(np.abs(host(out) - o.level_op(l, 1, b, x, n)) <= bound)
        g.level_op(l, "RESTRICT", dev(x), None, out_c)
        assert np.all(np.abs(host(out_c) - o.level_op(l, 2, x, None, nc)) <= 1e-13 * (abs(P.T) @ np.abs(x)))
        g.level_op(l, "INTERPOLATE", dev(xc), dev(x), out)
        assert np.all(np.abs(host(out) - o.level_op(l, 3, xc, x, n)) <= 1e-13 * (abs(P) @ np.abs(xc) + np.abs(x)))
        g.level_op(l, "SPMV_A", None, dev(x), out)
        A_l = _sp(o.export(l, "A"))
        assert np.all(np.abs(host(out) - A_l @ x) <= 1e-13 * (abs(A_l) @ np.abs(x)))
    for xin in (np.zeros(A.n), rng.uniform(-1, 1, A.n)):
        b = I.rhs(A.n, 7)
        xd = dev(xin)
        g.vcycle(dev(b), xd)
        ref = o.vcycle(b, xin)
        assert np.linalg.norm(host(xd) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", sorted(LARGE))
def test_solve_parity_large(lib, name):
    A = LARGE[name]()
    b = I.rhs(A.n, 2)
    from oracle import oracle as O
    nlev = O.OracleAMG(A).nlev
    gam = [0.0, 0.0] + [0.1] * (nlev - 2)
    xg, rg, xo, ro, g, o = _solve_pair(A, gam, b, method=1, tol=1e-8, maxit=200, adaptive=True, k=3, s=1)
    assert ro.converged
    _assert_solve_parity(xg, rg, xo, ro, 1e-8)


def test_full_size_poisson3d_128(lib):
    """The benchmark workload at full size (n = 2,097,152): hierarchy, minimal
    patterns, keep flags and sparsified patterns bit-exact; the adaptive
    AMG-PCG solve (k = 3, s = 1, rho_max = 0.5) takes the oracle's iteration
    count and agrees to 1e-10 at every gamma of the comparison (0.1, 0.01 and
    0, the Galerkin hierarchy), and with gamma = 1 and every window forced to
    reintroduce (rho_max = 0), which walks the gamma ladder at full size."""
    from oracle import oracle as O
    A = I.poisson3d(128)
    b = I.rhs(A.n, 2)
    g, o = both(A)
    assert g.nlev == o.nlev == 8
    for l in range(o.nlev):
        ga, oa = g.export(l, "A"), o.export(l, "A")
        assert same_csr(ga, oa), l
    kw = dict(method=1, tol=1e-8, maxit=200, adaptive=True, k=3, s=1)
    runs = [(0.1, 0.5), (0.01, 0.5), (0.0, 0.5), (1.0, 0.0)]
    for gamma, rho_max in runs:
        print(f"128^3 gamma {gamma} rho_max {rho_max}", flush=True)
        g.sparsify(gamma, 2)
        o.sparsify_from(gamma, 2)
        for l in range(1, o.nlev):
            if gamma == 0.1:
                assert np.array_equal(g.mask(l, "M"), o.mask(l, "M")), l
            assert np.array_equal(g.mask(l, "KEEP"), o.mask(l, "KEEP")), (gamma, l)
            gh, oh = g.export(l, "AHAT"), o.export(l, "AHAT")
            assert np.array_equal(gh[2], oh.row_ptr) and np.array_equal(gh[3], oh.col), (gamma, l)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        rg = g.solve(dev(b), x, rho_max=rho_max, **kw)
        xo, ro = o.solve(b, rho_max=rho_max, **kw)
        print(f"  iterations {rg.iters}/{ro.iters}, reintroductions {rg.reintroductions}/{ro.reintroductions}",
              flush=True)
        _assert_solve_parity(host(x), rg, xo, ro, kw["tol"])
        assert rg.converged and rg.relres <= 1e-8
        if rho_max == 0.0:
            assert ro.reintroductions >= 3
            for l in range(o.nlev):
                assert g.gamma(l) == o.gamma(l), l
            for l in range(1, o.nlev):
                gh, oh = g.export(l, "AHAT"), o.export(l, "AHAT")
                assert np.array_equal(gh[2], oh.row_ptr) and np.array_equal(gh[3], oh.col), l


def test_full_size_aniso2d_1024_adaptive_reintroduction(lib):
    """Rotated anisotropic Q1 1024^2 (n = 1,048,576), gamma = 0.1 on levels
    >= 2, adaptive AMG-PCG (k = 3, s = 1, rho_max = 0.5) to 1e-8: the windowed
    convergence factor exceeds 0.5 and the solve reintroduces dropped entries
    many times; the device takes the oracle's iterations, reintroductions and
    restarts, agrees to 1e-10 and ends on the oracle's gamma ladder and
    sparsified patterns."""
    from oracle import oracle as O
    A = I.aniso2d(1024)
    b = I.rhs(A.n, 3)
    g, o = both(A)
    g.sparsify(0.1, 2)
    o.sparsify_from(0.1, 2)
    kw = dict(method=1, tol=1e-8, maxit=300, adaptive=True, k=3, s=1, rho_max=0.5)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    print("aniso 1024^2 adaptive: device solve", flush=True)
    rg = g.solve(dev(b), x, **kw)
    print("aniso 1024^2 adaptive: oracle solve", flush=True)
    xo, ro = o.solve(b, **kw)
    print(f"  iterations {rg.iters}/{ro.iters}, reintroductions {rg.reintroductions}/{ro.reintroductions}",
          flush=True)
    assert ro.converged and ro.reintroductions >= 5
    _assert_solve_parity(host(x), rg, xo, ro, kw["tol"])
    for l in range(o.nlev):
        assert g.gamma(l) == o.gamma(l), l
    for l in range(1, o.nlev):
        gh, oh = g.export(l, "AHAT"), o.export(l, "AHAT")
        assert np.array_equal(gh[2], oh.row_ptr) and np.array_equal(gh[3], oh.col), l


def _shifted_poisson2d(N, sigma):
    from tests.test_oracle_coarse_lu import shifted_poisson2d
    return shifted_poisson2d(N, sigma)


def test_indefinite_coarsest_operator(lib):
    """Coarsest operators that are not positive definite, where the oracle
    leaves Cholesky for partial pivoting: a dense symmetric indefinite 40 x 40
    matrix (one level) and 2D Poisson 16^2 shifted by -0.1 (three levels, the
    coarsest Galerkin operator indefinite).  The coarsest solve (device:
    Gauss-Jordan inverse with partial pivoting; oracle: LU with partial
    pivoting) agrees normwise to 64 n eps cond, the forward-error bound of
    either; the V-cycle to 1e-12; stationary AMG takes the oracle's
    iterations, and CG breaks down where the oracle's does."""
    eps = np.finfo(np.float64).eps
    from tests.test_oracle_coarse_lu import dense_indefinite
    D = dense_indefinite(40, 13)
    g, o = both(D)
    assert g.nlev == o.nlev == 1
    kappa = np.linalg.cond(D.to_dense())
    for rs in (1, 2):
        bb = I.rhs(40, rs)
        out = torch.empty(40, dtype=torch.float64, device="cuda")
        g.level_op(0, "COARSE_SOLVE", dev(bb), None, out)
        ref = o.level_op(0, 4, bb, None, 40)
        assert np.linalg.norm(host(out) - ref) <= 64 * 40 * eps * kappa * np.linalg.norm(ref)
    A = _shifted_poisson2d(16, 0.1)
    g, o = both(A)
    assert g.nlev == o.nlev == 3
    L = o.nlev - 1
    DL = o.export(L, "AHAT").to_dense()
    assert np.linalg.eigvalsh(DL).min() < 0
    nL = DL.shape[0]
    bL = I.rhs(nL, 5)
    out = torch.empty(nL, dtype=torch.float64, device="cuda")
    g.level_op(L, "COARSE_SOLVE", dev(bL), None, out)
    ref = o.level_op(L, 4, bL, None, nL)
    assert np.linalg.norm(host(out) - ref) <= 64 * nL * eps * np.linalg.cond(DL) * np.linalg.norm(ref)
    b = I.rhs(A.n, 1)
    for xin in (np.zeros(A.n), I.rhs(A.n, 8)):
        xd = dev(xin)
        g.vcycle(dev(b), xd)
        ref = o.vcycle(b, xin)
        assert np.linalg.norm(host(xd) - ref) <= 1e-12 * np.linalg.norm(ref)
    xg, rg, xo, ro, g2, o2 = _solve_pair(A, [0.0], b, method=0, tol=1e-10, maxit=100)
    assert ro.converged
    _assert_solve_parity(xg, rg, xo, ro, 1e-10)
    xg, rg, xo, ro, g2, o2 = _solve_pair(A, [0.0], b, method=1, tol=1e-10, maxit=100)
    assert ro.status == rg.status == -6 and rg.iters == ro.iters


def test_row_formats_and_sell_ops(lib):
    """3D Poisson 64^3: the fine operators A_0, A_1, R_0 run on their SELL-64
    copies (slices pad them by a few percent), the interpolation P_0 (C and F
    rows alternate: about 70% padding) on the LDS-staged CSR kernel, the
    small coarse levels on the subgroup kernel; every level operation on the
    SELL operators agrees with the oracle row by row, in both slice orders."""
    A = I.poisson3d(64)
    g, o = both(A)
    assert g.row_format(0, "A") == g.row_format(1, "A") == g.row_format(0, "R") == "sell"
    assert g.row_format(0, "P") == "stream"
    assert g.row_format(o.nlev - 1, "A") == "row"
    rng = np.random.default_rng(3)
    for l in (0, 1):
        n = o.sizes(l)["n"]
        b, x = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        Ah = _sp(o.export(l, "AHAT"))
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        for _ in range(2):          # consecutive passes visit the slices in opposite orders
            g.level_op(l, "RESIDUAL", dev(b), dev(x), out)
            assert np.all(np.abs(host(out) - o.level_op(l, 0, b, x, n)) <= 1e-13 * (abs(Ah) @ np.abs(x) + np.abs(b)))
            g.level_op(l, "JACOBI", dev(b), dev(x), out)
            bound = 1e-13 * ((abs(Ah) @ np.abs(x) + np.abs(b)) / np.abs(Ah.diagonal()) + np.abs(x))
            assert np.all(np.abs(host(out) - o.level_op(l, 1, b, x, n)) <= bound)
