"""Hybrid Galerkin (Section 3, sparse_hybrid_setup, hybrid branch: the minimal
pattern of level l from the sparsified \\hat A_{l-1}) on the device against the
oracle in the same mode.  Bars as for Sparse Galerkin: minimal pattern, keep
flags, sparsified pattern and kept off-diagonal values bit-exact; lumped
diagonal within 1e-13 of the dropped magnitudes; solves with equal iteration
counts, reintroductions and the solution within 1e-10."""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_gpu_parity import PROBLEMS, _assert_solve_parity, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    amg.load_library()
    return amg


def hybrid_pair(A):
    from oracle import oracle as O
    from paper_1512_04629_amd import amg
    g, o = amg.Hierarchy(A), O.OracleAMG(A)
    g.set_method(True)
    o.set_method(True)
    return g, o


def compare_levels(g, o):
    for l in range(1, o.nlev):
        assert g.gamma(l) == o.gamma(l)
        assert np.array_equal(g.mask(l, "M"), o.mask(l, "M")), ("M", l)
        assert np.array_equal(g.mask(l, "KEEP"), o.mask(l, "KEEP")), ("keep", l)
        nr, nc, rp, ci, v = g.export(l, "AHAT")
        ref = o.export(l, "AHAT")
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col), ("pattern", l)
        rows = np.repeat(np.arange(nr), np.diff(rp))
        off = rows != ci
        assert v[off].tobytes() == ref.val[off].tobytes(), ("offdiag", l)
        Ad = o.export(l, "A")
        arow = np.repeat(np.arange(Ad.nrows), np.diff(Ad.row_ptr))
        keep = o.mask(l, "KEEP").astype(bool)
        dropped_abs = np.bincount(arow[~keep], weights=np.abs(Ad.val[~keep]), minlength=nr)
        aii = Ad.val[arow == Ad.col]
        assert np.all(np.abs(v[~off] - ref.val[~off]) <= 1e-13 * (np.abs(aii) + dropped_abs)), ("diag", l)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.1, 1.0])
def test_hybrid_sparsify_parity(lib, name, gamma):
    A = PROBLEMS[name]()
    g, o = hybrid_pair(A)
    gam = [0.0] + [gamma] * (o.nlev - 1)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    compare_levels(g, o)
    # sparsifying again (the finer operators unchanged) is a fixed point
    g.sparsify_levels(gam)
    compare_levels(g, o)


def test_hybrid_reintroduce_ladder_parity(lib):
    A = I.poisson2d(160)
    g, o = hybrid_pair(A)
    start = [0.0, 0.0, 0.01, 0.1, 1.0, 1.0, 1.0]
    g.sparsify_levels(start)
    o.sparsify(start)
    for _ in range(8):
        assert g.reintroduce(s=1) == o.reintroduce(s=1)
        compare_levels(g, o)


def test_hybrid_adaptive_solve_parity(lib):
    A = I.poisson3d(16)
    b = I.rhs(A.n, 2)
    g, o = hybrid_pair(A)
    gam = [0.0, 0.0] + [1.0] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    kw = dict(method=1, tol=1e-12, maxit=200, adaptive=True, k=2, s=1, rho_max=0.0)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(dev(b), xd, **kw)
    xo, ro = o.solve(b, **kw)
    assert ro.reintroductions >= 3
    _assert_solve_parity(host(xd), rg, xo, ro, kw["tol"])
    compare_levels(g, o)


def test_switching_back_to_sparse_galerkin(lib):
    from oracle import oracle as O
    from paper_1512_04629_amd import amg
    A = I.aniso2d(64)
    g = amg.Hierarchy(A)
    g.set_method(True)
    gam = [0.0] + [0.1] * (g.nlev - 1)
    g.sparsify_levels(gam)
    g.set_method(False)
    g.sparsify_levels(gam)
    o = O.OracleAMG(A)
    o.sparsify(gam)
    compare_levels(g, o)
    with pytest.raises(amg.AmgError):
        g._check(g._lib.amg_set_method(g._h, 2))
