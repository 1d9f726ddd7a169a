"""FP32 V-cycle (values, vectors and accumulation in single precision) used
inside FP64 iterations, checked against the FP64 oracle.

Bars:
  * one FP32 V-cycle vs the oracle's FP64 V-cycle: normwise 2e-5 relative.
    Each level's row sums are FP32 sums of at most ~100 terms (relative error
    up to ~100 u_32 = 6e-6 per row in the worst case, typically far less);
    errors of the ~10 levels are damped by the cycle rather than compounded.
  * solves to rtol 1e-10: the true FP64 residual of the device solution is
    <= 1e-10 ||b|| (up to a 1% margin for the final residual evaluation), and
    the solution differs from the oracle's FP64 solution by at most what two
    1e-10-accurate solutions can differ by: ||A (x - x_or)|| <= 2.02e-10 ||b||.
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


PROBLEMS = {
    "poisson2d_64": lambda: I.poisson2d(64),
    "aniso2d_128": lambda: I.aniso2d(128),
    "fv3d_16": lambda: I.fv3d_lognormal(16),
    "graph_3000": lambda: I.random_graph_laplacian(3000),
    "poisson3d_64": lambda: I.poisson3d(64),      # fine operators on the LDS-staged kernel
    "aniso2d_512": lambda: I.aniso2d(512),
}


def both(A):
    from oracle import oracle as O
    from paper_1512_04629_amd import amg
    return amg.Hierarchy(A), O.OracleAMG(A)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_vcycle32_matches_fp64_oracle(lib, name):
    A = PROBLEMS[name]()
    g, o = both(A)
    gam = [0.0, 0.0] + [0.1] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    b = I.rhs(A.n, 7)
    for x0 in (np.zeros(A.n), I.rhs(A.n, 8)):
        x32 = torch.as_tensor(x0.astype(np.float32)).cuda()
        g.vcycle32(torch.as_tensor(b.astype(np.float32)).cuda(), x32)
        torch.cuda.synchronize()
        ref = o.vcycle(b.astype(np.float32).astype(np.float64), x0.astype(np.float32).astype(np.float64))
        err = np.linalg.norm(x32.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)
        assert err <= 2e-5, err


def _check_solution(A, b, xg, xo, rg):
    import scipy.sparse as sp
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    nb = np.linalg.norm(b)
    assert np.linalg.norm(b - S @ xg) <= 1.01e-10 * nb
    assert abs(rg.relres - np.linalg.norm(b - S @ xg) / nb) <= 1e-12
    assert np.linalg.norm(S @ (xg - xo)) <= 2.02e-10 * nb


@pytest.mark.parametrize("name", ["aniso2d_128", "fv3d_16", "poisson3d_64", "aniso2d_512"])
@pytest.mark.parametrize("method", [0, 1])
def test_mixed_solve_reaches_fp64_accuracy(lib, name, method):
    A = PROBLEMS[name]()
    b = I.rhs(A.n, 3)
    g, o = both(A)
    gam = [0.0, 0.0] + [0.1] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(torch.as_tensor(b).cuda(), x, method=method, tol=1e-10, maxit=400, precision=32)
    xo, ro = o.solve(b, method=method, tol=1e-10, maxit=400)
    assert rg.converged and ro.converged, (rg, ro)
    torch.cuda.synchronize()
    _check_solution(A, b, x.cpu().numpy(), xo, rg)
    # the FP32 preconditioner costs at most a few extra iterations here
    assert rg.iters <= ro.iters + 3, (rg.iters, ro.iters)


def test_fp32_copies_follow_resparsification(lib):
    """The FP32 operators rebuilt by a later sparsify equal those a fresh
    hierarchy builds: same iterates, bit for bit."""
    from paper_1512_04629_amd import amg
    A = I.poisson3d(24)
    b = torch.as_tensor(I.rhs(A.n, 2)).cuda()
    g1 = amg.Hierarchy(A)
    g1.sparsify(0.1, 2)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    g1.solve(b, x, tol=1e-10, maxit=100, precision=32)
    g1.sparsify(0.01, 2)
    x1 = torch.zeros_like(x)
    r1 = g1.solve(b, x1, tol=1e-10, maxit=100, precision=32, adaptive=True)
    g2 = amg.Hierarchy(A)
    g2.sparsify(0.01, 2)
    x2 = torch.zeros_like(x)
    r2 = g2.solve(b, x2, tol=1e-10, maxit=100, precision=32, adaptive=True)
    assert r1.iters == r2.iters
    assert torch.equal(x1, x2)


def test_mixed_adaptive_reintroduction(lib):
    A = I.poisson3d(16)
    b = I.rhs(A.n, 2)
    g, o = both(A)
    gam = [0.0, 0.0] + [1.0] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(torch.as_tensor(b).cuda(), x, method=1, tol=1e-10, maxit=200, adaptive=True, k=2, s=1,
                 rho_max=0.0, precision=32)
    xo, ro = o.solve(b, method=1, tol=1e-10, maxit=200, adaptive=True, k=2, s=1, rho_max=0.0)
    assert rg.converged and rg.reintroductions >= 3
    torch.cuda.synchronize()
    _check_solution(A, b, x.cpu().numpy(), xo, rg)
