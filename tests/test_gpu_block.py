"""Several right-hand sides per cycle (n x K row-interleaved blocks) against the
FP64 oracle, column by column, through the C ABI.

Bars:
  * FP64 block V-cycle vs the oracle's V-cycle of each column: normwise 1e-12
    (the single-vector bar: only the order of the row sums differs);
  * FP32 block V-cycle: normwise 2e-5 per column (FP32 row sums of at most
    ~100 terms on ~10 levels, damped by the cycle);
  * block iterative refinement to rtol 1e-10.  A stationary V-cycle iteration
    x <- V(b, x) and refinement x <- x + V(b - A x, 0) are the same iteration
    (the cycle is affine in b and x), so the oracle's stationary solve of each
    column is the reference: FP64 -- the first iteration at which a column
    meets the tolerance equals the oracle's count; FP32 -- within 2 of it; both
    -- the column's true FP64 residual <= 1.01e-10 ||r0_c|| and
    ||A (x_c - x_or,c)|| <= 2.02e-10 ||r0_c||;
  * a column solved inside a block equals, bit for bit, the same column solved
    alone for the same number of iterations (every kernel applies the same
    operations in the same order to each column, whatever the block width);
  * block PCG (one CG recurrence per column, all columns per launch) against
    the oracle's PCG of each column: FP64 -- equal iteration counts; FP32
    cycle -- at most 3 more; both -- the residual and solution bars above;
    a column's result is bitwise the same alone (other columns zero) and in
    a full block of the same width.
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
    "poisson2d_63": lambda: I.poisson2d(63),        # ragged last row tile
    "aniso2d_128": lambda: I.aniso2d(128),
    "fv3d_16": lambda: I.fv3d_lognormal(16),
    "graph_3000": lambda: I.random_graph_laplacian(3000),
    "poisson3d_32": lambda: I.poisson3d(32),
}


def hier(A, gamma=0.1):
    from oracle import oracle as O
    from paper_1512_04629_amd import amg
    g, o = amg.Hierarchy(A), O.OracleAMG(A)
    gam = [0.0, 0.0] + [gamma] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    return g, o


def block_rhs(n, k, seed0):
    return np.stack([I.rhs(n, seed0 + c) for c in range(k)], axis=1)


def sp(A):
    import scipy.sparse as S
    return S.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("k", [4, 8, 16])
def test_vcycle_block_fp64_matches_oracle(lib, name, k):
    A = PROBLEMS[name]()
    g, o = hier(A)
    B = block_rhs(A.n, k, 100)
    X0 = block_rhs(A.n, k, 200) if k == 8 else np.zeros((A.n, k))
    X = dev(X0)
    g.vcycle_block(dev(B), X)
    Xg = host(X)
    for c in range(k):
        ref = o.vcycle(B[:, c], X0[:, c])
        assert np.linalg.norm(Xg[:, c] - ref) <= 1e-12 * np.linalg.norm(ref), (c, name)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("k", [4, 16])
def test_vcycle_block_fp32_matches_oracle(lib, name, k):
    A = PROBLEMS[name]()
    g, o = hier(A)
    B = block_rhs(A.n, k, 300).astype(np.float32)
    X0 = block_rhs(A.n, k, 400).astype(np.float32) if k == 4 else np.zeros((A.n, k), np.float32)
    X = dev(X0, torch.float32)
    g.vcycle_block(dev(B, torch.float32), X)
    Xg = host(X)
    for c in range(k):
        ref = o.vcycle(B[:, c].astype(np.float64), X0[:, c].astype(np.float64))
        assert np.linalg.norm(Xg[:, c] - ref) <= 2e-5 * np.linalg.norm(ref), (c, name)


def _check_columns(A, B, X0, Xg, res, o, precision, tol=1e-10, method=0):
    S = sp(A)
    for c in range(B.shape[1]):
        xo, ro = o.solve(B[:, c], x0=X0[:, c], method=method, tol=tol, maxit=400)
        assert ro.converged
        r0 = np.linalg.norm(B[:, c] - S @ X0[:, c])
        assert np.linalg.norm(B[:, c] - S @ Xg[:, c]) <= 1.01 * tol * r0, c
        assert np.linalg.norm(S @ (Xg[:, c] - xo)) <= 2.02 * tol * r0, c
        if precision == 64:
            assert res.col_iters[c] == ro.iters, (c, res.col_iters[c], ro.iters)
        elif method == 0:
            assert abs(int(res.col_iters[c]) - ro.iters) <= 2, (c, res.col_iters[c], ro.iters)
        else:
            assert ro.iters <= res.col_iters[c] <= ro.iters + 3, (c, res.col_iters[c], ro.iters)
        assert res.col_relres[c] <= 1.01 * tol
    assert res.iters == max(res.col_iters)


@pytest.mark.parametrize("name", ["aniso2d_128", "fv3d_16", "graph_3000", "poisson2d_63"])
@pytest.mark.parametrize("precision", [64, 32])
def test_solve_block_matches_oracle(lib, name, precision):
    A = PROBLEMS[name]()
    g, o = hier(A, 0.01)
    B = block_rhs(A.n, 16, 41)
    X0 = np.zeros_like(B)
    X = dev(X0)
    res = g.solve_block(dev(B), X, method=0, tol=1e-10, maxit=400, precision=precision)
    assert res.status == 0 and res.converged
    _check_columns(A, B, X0, host(X), res, o, precision)


@pytest.mark.parametrize("nrhs", [1, 3, 5, 13])
@pytest.mark.parametrize("precision", [64, 32])
def test_solve_block_padded_widths_and_initial_guess(lib, nrhs, precision):
    A = I.fv3d_lognormal(16)
    g, o = hier(A, 0.01)
    B = block_rhs(A.n, nrhs, 500)
    X0 = 0.5 * block_rhs(A.n, nrhs, 600)
    X = dev(X0)
    res = g.solve_block(dev(B), X, method=0, tol=1e-10, maxit=400, precision=precision)
    assert res.status == 0 and res.converged and len(res.col_iters) == nrhs
    _check_columns(A, B, X0, host(X), res, o, precision)


@pytest.mark.parametrize("precision", [64, 32])
def test_block_columns_equal_single_column_solves_bitwise(lib, precision):
    A = I.aniso2d(96)
    g, _ = hier(A)
    B = block_rhs(A.n, 16, 700)
    X = torch.zeros(A.n, 16, dtype=torch.float64, device="cuda")
    res = g.solve_block(dev(B), X, method=0, tol=0.0, maxit=6, precision=precision)
    assert res.status == -5 and res.iters == 6 and all(res.col_iters == -1)
    Xb = X.cpu().numpy()
    for c in (0, 5, 15):
        xc = torch.zeros(A.n, 1, dtype=torch.float64, device="cuda")
        rc = g.solve_block(dev(B[:, c:c + 1]), xc, method=0, tol=0.0, maxit=6, precision=precision)
        assert rc.iters == 6
        assert xc.cpu().numpy()[:, 0].tobytes() == Xb[:, c].tobytes(), c
        # the norms are reduced over a different row partition: rounding only
        assert abs(rc.col_relres[0] - res.col_relres[c]) <= 1e-12 * res.col_relres[c]


def test_block_edge_cases(lib):
    from paper_1512_04629_amd import amg
    A = I.poisson2d(40)
    g, _ = hier(A)
    n = A.n
    B = block_rhs(n, 4, 800)
    B[:, 2] = 0.0                                  # zero column: converged at once, stays zero
    X = torch.zeros(n, 4, dtype=torch.float64, device="cuda")
    res = g.solve_block(dev(B), X, method=0, tol=1e-10, maxit=100)
    assert res.converged and res.col_iters[2] == 0 and res.col_relres[2] == 0.0
    assert torch.count_nonzero(X[:, 2]).item() == 0
    # not converged within maxit: status and per-column -1
    X.zero_()
    res = g.solve_block(dev(B), X, method=0, tol=1e-14, maxit=2)
    assert res.status == -5 and not res.converged and res.col_iters[0] == -1 and res.iters == 2
    # all columns zero: nothing to do
    X.zero_()
    res = g.solve_block(torch.zeros(n, 4, dtype=torch.float64, device="cuda"), X)
    assert res.status == 0 and res.iters == 0 and res.converged
    # argument errors
    lib_ = amg.load_library()
    Bd, Xd = dev(B), torch.zeros(n, 4, dtype=torch.float64, device="cuda")
    p = amg.SolveParams(0, 1e-10, 10, 0, 3, 1, 0.5, 0.01, 32)
    vp = lambda t: amg.C.c_void_p(t.data_ptr())
    for nrhs in (0, 17):
        assert lib_.amg_solve_block(g._h, nrhs, vp(Bd), vp(Xd), amg.C.byref(p), None, None, None) == -1
    for bad in (amg.SolveParams(2, 1e-10, 10, 0, 3, 1, 0.5, 0.01, 32),      # no such method
                amg.SolveParams(0, 1e-10, 10, 1, 3, 1, 0.5, 0.01, 32),      # adaptive
                amg.SolveParams(0, 1e-10, 10, 0, 3, 1, 0.5, 0.01, 16)):     # precision
        assert lib_.amg_solve_block(g._h, 4, vp(Bd), vp(Xd), amg.C.byref(bad), None, None, None) == -1
    flat = torch.zeros(n * 4 + 1, dtype=torch.float64, device="cuda")
    mis = amg.C.c_void_p(flat.data_ptr() + 8)                              # 8-byte aligned only
    assert lib_.amg_solve_block(g._h, 4, vp(Bd), mis, amg.C.byref(p), None, None, None) == -1
    assert lib_.amg_vcycle_block(g._h, 3, vp(Bd), vp(Xd)) == -1
    assert lib_.amg_solve_block(None, 4, vp(Bd), vp(Xd), amg.C.byref(p), None, None, None) == -7


@pytest.mark.parametrize("precision", [64, 32])
def test_block_after_resparsification(lib, precision):
    """The block cycle uses the operators of the latest sparsification."""
    A = I.poisson3d(20)
    g, o = hier(A, 1.0)
    g.sparsify(0.01, 2)
    o.sparsify([0.0, 0.0] + [0.01] * (o.nlev - 2))
    B = block_rhs(A.n, 8, 900)
    X = torch.zeros(A.n, 8, dtype=torch.float64, device="cuda")
    res = g.solve_block(dev(B), X, method=0, tol=1e-10, maxit=200, precision=precision)
    assert res.converged
    _check_columns(A, B, np.zeros_like(B), host(X), res, o, precision)


def test_block_large_multi_tile(lib):
    """373,248 rows: more row tiles than workgroups (grid-stride loops)."""
    A = I.poisson3d(72)
    g, o = hier(A)
    B = block_rhs(A.n, 16, 1000)
    Bf = B.astype(np.float32)
    X = torch.zeros(A.n, 16, dtype=torch.float32, device="cuda")
    g.vcycle_block(dev(Bf, torch.float32), X)
    Xg = host(X)
    Y = torch.zeros(A.n, 16, dtype=torch.float64, device="cuda")
    g.vcycle_block(dev(B), Y)
    Yg = host(Y)
    for c in (0, 7, 15):
        ref = o.vcycle(Bf[:, c].astype(np.float64), np.zeros(A.n))
        assert np.linalg.norm(Xg[:, c] - ref) <= 2e-5 * np.linalg.norm(ref)
        ref = o.vcycle(B[:, c], np.zeros(A.n))
        assert np.linalg.norm(Yg[:, c] - ref) <= 1e-12 * np.linalg.norm(ref)
    Xs = torch.zeros(A.n, 16, dtype=torch.float64, device="cuda")
    res = g.solve_block(dev(B), Xs, method=0, tol=1e-10, maxit=100, precision=32)
    assert res.converged
    S = sp(A)
    Xh = host(Xs)
    for c in range(16):
        assert np.linalg.norm(B[:, c] - S @ Xh[:, c]) <= 1.01e-10 * np.linalg.norm(B[:, c])


@pytest.mark.parametrize("name", ["aniso2d_128", "fv3d_16", "graph_3000", "poisson3d_32"])
@pytest.mark.parametrize("precision", [64, 32])
def test_block_pcg_matches_oracle(lib, name, precision):
    A = PROBLEMS[name]()
    g, o = hier(A, 0.01)
    B = block_rhs(A.n, 16, 1100)
    X0 = np.zeros_like(B)
    X = dev(X0)
    res = g.solve_block(dev(B), X, method=1, tol=1e-10, maxit=400, precision=precision)
    assert res.status == 0 and res.converged
    _check_columns(A, B, X0, host(X), res, o, precision, method=1)


@pytest.mark.parametrize("nrhs", [1, 6])
def test_block_pcg_padded_and_initial_guess(lib, nrhs):
    A = I.aniso2d(64)
    g, o = hier(A, 0.1)
    B = block_rhs(A.n, nrhs, 1200)
    X0 = 0.25 * block_rhs(A.n, nrhs, 1300)
    X = dev(X0)
    res = g.solve_block(dev(B), X, method=1, tol=1e-10, maxit=400, precision=32)
    assert res.status == 0 and res.converged
    _check_columns(A, B, X0, host(X), res, o, 32, method=1)


@pytest.mark.parametrize("precision", [64, 32])
def test_block_pcg_column_alone_equals_column_in_block(lib, precision):
    A = I.fv3d_lognormal(20)
    g, _ = hier(A, 0.01)
    B = block_rhs(A.n, 16, 1400)
    X = torch.zeros(A.n, 16, dtype=torch.float64, device="cuda")
    res = g.solve_block(dev(B), X, method=1, tol=1e-10, maxit=300, precision=precision)
    assert res.converged
    Xb = X.cpu().numpy()
    for c in (0, 9, 15):
        Bc = np.zeros_like(B)
        Bc[:, c] = B[:, c]
        Xc = torch.zeros(A.n, 16, dtype=torch.float64, device="cuda")
        rc = g.solve_block(dev(Bc), Xc, method=1, tol=1e-10, maxit=300, precision=precision)
        assert rc.converged and rc.col_iters[c] == res.col_iters[c]
        assert Xc.cpu().numpy()[:, c].tobytes() == Xb[:, c].tobytes(), c
        assert torch.count_nonzero(Xc).item() == torch.count_nonzero(Xc[:, c]).item()


def test_block_pcg_zero_and_converged_columns_stay_fixed(lib):
    A = I.poisson2d(48)
    g, _ = hier(A)
    B = block_rhs(A.n, 8, 1500)
    B[:, 3] = 0.0
    X = torch.zeros(A.n, 8, dtype=torch.float64, device="cuda")
    res = g.solve_block(dev(B), X, method=1, tol=1e-10, maxit=100, precision=32)
    assert res.converged and res.col_iters[3] == 0 and res.col_relres[3] == 0.0
    assert torch.count_nonzero(X[:, 3]).item() == 0
    assert np.all(np.isfinite(X.cpu().numpy()))
