"""Degenerate inputs through the C ABI, against the oracle.

* a 1 x 1 system and a diagonal matrix of 500 rows: no strong couplings, so
  the split is empty and the fine level is the coarsest (solved by the dense
  inverse); one PCG iteration gives x = D^-1 b;
* a zero right-hand side: converged at iteration 0 with x = 0 exactly, for
  PCG and the stationary iteration, with the FP64 and the FP32 cycle;
* rows without couplings inside a coupled problem (isolated points, which the
  split makes F points with empty interpolation rows): hierarchy, keep flags
  and sparsified operators bit-exact under diagonal and strong-neighbour
  lumping, and the solve at the parity bars;
* a hierarchy with more sparsified levels than one launch of the count scans
  takes: every operator as sparsified alone, row sums kept;
* the zero initial guess (zero_guess): the iterates of the solve from a
  zeroed x, whatever x held; rejected by the block solve and for values
  other than 0 and 1;
* the adaptive windows' fused residual pass: without a reintroduction the
  iterates of the plain PCG, bit for bit.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_gpu_parity import _assert_solve_parity, _solve_pair, both, dev, host, same_csr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    amg.load_library()
    return amg


def _diagonal(d):
    n = len(d)
    return I.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, np.float64))


def _isolate(A, rows):
    """A with every off-diagonal coupling of the given rows (and their mirror
    entries) removed: still bitwise symmetric."""
    iso = np.zeros(A.n, bool)
    iso[list(rows)] = True
    r = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    keep = (r == A.col) | ~(iso[r] | iso[A.col])
    rp = np.concatenate([[0], np.cumsum(np.bincount(r[keep], minlength=A.n))]).astype(np.int32)
    return I.CSR(A.n, rp, A.col[keep].astype(np.int32), A.val[keep].copy())


@pytest.mark.parametrize("d", [[4.0], list(2.0 + np.arange(500) % 7)], ids=["1x1", "diag500"])
def test_no_couplings_single_level(lib, d):
    A = _diagonal(d)
    b = I.rhs(A.n, 5)
    xg, rg, xo, ro, g, o = _solve_pair(A, [0.0], b, method=1, tol=1e-10, maxit=10)
    assert g.nlev == o.nlev == 1
    assert rg.converged and rg.iters == ro.iters == 1
    np.testing.assert_allclose(xg, b / np.asarray(d), rtol=1e-14, atol=0)
    assert np.linalg.norm(xg - xo) <= 1e-14 * np.linalg.norm(xo)
    g.sparsify(0.1, 2)            # nothing to sparsify on a single level
    g.set_lumping("strong")
    g.sparsify(1.0, 1)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    assert g.solve(dev(b), x, method=1, tol=1e-10, maxit=10).iters == 1


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [64, 32])
def test_zero_right_hand_side(lib, method, precision):
    A = I.poisson2d(16)
    g, o = both(A)
    g.sparsify(0.1, 2)
    o.sparsify_from(0.1, 2)
    xo, ro = o.solve(np.zeros(A.n), method=method, tol=1e-10, maxit=10)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(torch.zeros(A.n, dtype=torch.float64, device="cuda"), x, method=method, tol=1e-10, maxit=10,
                 precision=precision)
    assert rg.converged and rg.iters == ro.iters == 0 and rg.status == ro.status == 0
    assert torch.count_nonzero(x).item() == 0 and not np.any(xo)


@pytest.mark.parametrize("noalloc", [False, True])
def test_zero_guess_start(lib, noalloc):
    """zero_guess: the solve starts from x0 = 0 whatever x holds (x zeroed,
    r0 = b with no product by the zero vector): the iterations, the
    reintroductions and the iterates are those of the solve from an explicitly
    zeroed x, and the result meets the oracle's parity bars."""
    A = I.poisson3d(20)
    b = I.rhs(A.n, 3)
    g, o = both(A)
    kw = dict(method=1, tol=1e-8, maxit=100, adaptive=True, k=3, s=1, rho_max=0.5)
    g.sparsify(0.1, 2)
    x0 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r0 = g.solve(dev(b), x0, noalloc=noalloc, **kw)
    g.sparsify(0.1, 2)
    gen = torch.Generator(device="cuda").manual_seed(11)
    x1 = 10.0 * torch.randn(A.n, dtype=torch.float64, device="cuda", generator=gen)
    r1 = g.solve(dev(b), x1, noalloc=noalloc, zero_guess=True, **kw)
    assert r1.converged and (r1.iters, r1.reintroductions) == (r0.iters, r0.reintroductions)
    assert torch.equal(x1, x0)
    nb = float(np.linalg.norm(b))
    assert abs(r1.hist[0] - nb) <= 1e-13 * nb
    assert abs(r1.relres - r0.relres) <= 1e-12 * r0.relres
    o.sparsify_from(0.1, 2)
    xo, ro = o.solve(b, **kw)
    _assert_solve_parity(host(x1), r1, xo, ro, kw["tol"])


def test_adaptive_windows_keep_the_pcg_iterates(lib):
    """The adaptive solve forms the true residual every k iterations, in one
    pass over A_0's SELL-64 copy together with the next preconditioner's
    level-0 residual.  Without a reintroduction (rho_max out of reach) the
    iterates and the residual history are those of the plain PCG bit for
    bit."""
    A = I.poisson3d(72)
    b = I.rhs(A.n, 4)
    g = lib.Hierarchy(A)
    assert g.row_format(0, "A") == "sell"
    kw = dict(method=1, tol=1e-10, maxit=100)
    g.sparsify(0.1, 2)
    x1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r1 = g.solve(dev(b), x1, **kw)
    g.sparsify(0.1, 2)
    x2 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r2 = g.solve(dev(b), x2, adaptive=True, k=3, s=1, rho_max=1e9, **kw)
    assert r1.converged and r2.converged and r2.reintroductions == 0
    assert r1.iters == r2.iters and r1.iters >= 6
    assert np.array_equal(r1.hist, r2.hist)
    assert torch.equal(x1, x2)
    g.close()


def test_zero_guess_rejected_by_block_solve(lib):
    A = I.poisson2d(16)
    g = lib.Hierarchy(A)
    p = lib.SolveParams(0, 1e-10, 10, 0, 3, 1, 0.5, 0.01, 64, 1)
    b = torch.zeros((A.n, 4), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    assert g._lib.amg_solve_block(g._h, 4, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(p),
                                  None, None, None) == -1
    p.zero_guess = 2
    assert g._lib.amg_solve(g._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(p), None,
                            None) == -1
    g.close()


@pytest.mark.parametrize("lumping", ["diagonal", "strong"])
def test_isolated_rows_inside_a_coupled_problem(lib, lumping):
    A = _isolate(I.poisson3d(12), [0, 17, 100, 863, 1727])
    b = I.rhs(A.n, 6)
    g, o = both(A)
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        assert same_csr(g.export(l, "A"), o.export(l, "A")), l
        if l < o.nlev - 1:
            assert same_csr(g.export(l, "P"), o.export(l, "P")), l
    g.set_lumping(lumping)
    o.set_lumping(lumping)
    gam = [0.0, 0.0] + [1.0] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    for l in range(1, o.nlev):
        assert np.array_equal(g.mask(l, "KEEP"), o.mask(l, "KEEP")), l
        gh, oh = g.export(l, "AHAT"), o.export(l, "AHAT")
        assert np.array_equal(gh[2], oh.row_ptr) and np.array_equal(gh[3], oh.col), l
        if lumping == "strong":
            assert gh[4].tobytes() == oh.val.tobytes(), l
        else:
            assert np.allclose(gh[4], oh.val, rtol=1e-13, atol=0), l
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(dev(b), x, method=1, tol=1e-10, maxit=100)
    xo, ro = o.solve(b, method=1, tol=1e-10, maxit=100)
    _assert_solve_parity(host(x), rg, xo, ro, 1e-10)
    # an isolated row's residual is b_i - a_ii x_i, at most the stopping residual
    xh, nb = host(x), np.linalg.norm(b)
    for i in (0, 17, 100, 863, 1727):
        d = A.val[A.row_ptr[i]]
        assert abs(xh[i] - b[i] / d) <= 1.01e-10 * nb / d, i


def test_singular_coarsest_reported_after_index_toggle(lib):
    """[[1, -1], [-1, 1]] passes validation (symmetric, positive diagonal) but
    is singular; the device inversion of the coarsest operator meets a zero
    pivot.  The pending flag survives rebuilding and dropping the 16-bit
    column indices (which use a device word of their own) and the next solve
    reports the matrix as bad."""
    A = I.CSR(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32),
              np.array([1.0, -1.0, -1.0, 1.0]))
    g = lib.Hierarchy(A)
    g.set_compact_indices(False)
    g.set_compact_indices(True)
    x = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.AmgError) as e:
        g.solve(dev(np.array([1.0, 2.0])), x, method=1, tol=1e-10, maxit=5)
    assert e.value.status == -2 and "singular" in str(e.value)


def test_sparsify_more_levels_than_one_scan_launch(lib):
    """1D Poisson on 2^23 points: 19 levels, 17 of them sparsified (levels >=
    2), more than one launch of the per-level count scans takes (16), so the
    levels go in two rounds.  Every sparsified operator must be bitwise the
    one a call sparsifying that level alone produces, and its lumped rows must
    keep the Galerkin row sums (Section 3.1)."""
    n = 1 << 23
    A = I._structured((n,), [(0,), (-1,), (1,)], [2.0, -1.0, -1.0])
    g = lib.Hierarchy(A)
    L = g.nlev
    assert L - 2 > 16, L
    gam = [0.0, 0.0] + [0.1] * (L - 2)
    g.sparsify_levels(gam)
    together = {l: g.export(l, "AHAT") for l in range(2, L)}
    for l in range(2, L):
        one = [0.0] * L
        one[l] = 0.1
        g.sparsify_levels(one)
        alone = g.export(l, "AHAT")
        for a, b in zip(together[l], alone):
            assert np.asarray(a).tobytes() == np.asarray(b).tobytes(), l
        nr, nc, rp, ci, v = alone
        Al = g.export(l, "A")
        rows = np.repeat(np.arange(nr), np.diff(rp))
        arows = np.repeat(np.arange(Al[0]), np.diff(Al[2]))
        rs_hat = np.bincount(rows, weights=v, minlength=nr)
        rs = np.bincount(arows, weights=Al[4], minlength=nr)
        scale = np.bincount(arows, weights=np.abs(Al[4]), minlength=nr)
        assert np.all(np.abs(rs_hat - rs) <= 1e-13 * scale), l
    g.close()
