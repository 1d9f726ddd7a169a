"""The method of non-Galerkin coarse grids (Section 2.1: each coarse product
sparsified during setup and used to build the next level) through the C ABI,
against the oracle in the same mode.  Bars as for the Galerkin hierarchy: the
hierarchy (operators, interpolation, restriction, C/F splits) bit for bit;
solves with equal iteration counts and the solution within 1e-10; a Sparse
Galerkin post-pass on top with the sparsify bars."""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_gpu_hybrid import compare_levels
from .test_gpu_parity import PROBLEMS, _assert_solve_parity, dev, host, same_csr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    amg.load_library()
    return amg


def pair(A, ng):
    from oracle import oracle as O
    from paper_1512_04629_amd import amg
    return amg.Hierarchy(A, nongalerkin_gamma=ng), O.OracleAMG(A, nongalerkin_gamma=ng)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.1, 0.5])
def test_nongalerkin_setup_bitwise(lib, name, gamma):
    A = PROBLEMS[name]()
    ng = [0.0, 0.0] + [gamma] * 20
    g, o = pair(A, ng)
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        assert same_csr(g.export(l, "A"), o.export(l, "A")), l
        if l < o.nlev - 1:
            assert same_csr(g.export(l, "P"), o.export(l, "P")), l
            assert same_csr(g.export(l, "R"), o.export(l, "R")), l
            assert np.array_equal(g.split(l), o.cf(l)), l


@pytest.mark.parametrize("method", [0, 1])
def test_nongalerkin_solve_parity(lib, method):
    A = I.poisson3d(24)
    b = I.rhs(A.n, 5)
    g, o = pair(A, [0.0, 0.0] + [0.1] * 20)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    kw = dict(method=method, tol=1e-10, maxit=300)
    rg = g.solve(dev(b), xd, **kw)
    xo, ro = o.solve(b, **kw)
    assert ro.converged
    _assert_solve_parity(host(xd), rg, xo, ro, kw["tol"])


def test_sparse_galerkin_post_pass_on_a_nongalerkin_hierarchy(lib):
    A = I.aniso2d(96)
    g, o = pair(A, [0.0, 0.0, 0.05, 0.05])
    gam = [0.0] + [0.1] * (o.nlev - 1)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    compare_levels(g, o)


def test_invalid_nongalerkin_gamma_rejected(lib):
    from paper_1512_04629_amd import amg
    A = I.poisson2d(20)
    with pytest.raises(amg.AmgError):
        amg.Hierarchy(A, nongalerkin_gamma=[0.0, 0.0, 1.5])
    with pytest.raises(amg.AmgError):
        amg.Hierarchy(A, nongalerkin_gamma=[])
