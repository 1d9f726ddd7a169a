"""Pins of the oracle's coarsest-level direct solve when the coarsest operator
is not positive definite (Section 2, amg_solve: direct solve on the coarsest
level).  The oracle factors with Cholesky and falls back to Gaussian
elimination with partial pivoting when a pivot is not positive; these tests
reach that fallback and check it against LAPACK (numpy.linalg.solve), the
backward-stability bound of partial pivoting, and the dense V-cycle
recursion with an explicit inverse.

Inputs that reach the branch:
  * a dense symmetric indefinite matrix with a positive diagonal and n <= 49,
    so the hierarchy has one level and the coarsest operator is the matrix;
  * 2D Poisson 16x16 with 0.1 subtracted from the diagonal (one negative
    eigenvalue): the three-level hierarchy's coarsest Galerkin operator is
    indefinite too, and stationary AMG still converges on it.
"""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I
from tests.test_oracle_solve import dense_vcycle_operators

EPS = np.finfo(np.float64).eps


def shifted_poisson2d(N: int, sigma: float) -> I.CSR:
    """5-point Poisson with sigma subtracted from every diagonal entry: still
    bitwise symmetric with a positive diagonal, indefinite once sigma exceeds
    the smallest eigenvalue 8 sin^2(pi / (2 (N + 1)))."""
    A = I.poisson2d(N)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    A.val[A.col == rows] -= sigma
    return A


def dense_indefinite(n: int, seed: int) -> I.CSR:
    """Dense symmetric matrix, off-diagonals uniform[-1, 1], diagonal
    uniform[0.05, 0.5]: positive diagonal, Cholesky fails, and partial
    pivoting has to swap rows (the off-diagonals outweigh the diagonal)."""
    u = I.uniform_pm1(seed, n * n).reshape(n, n)
    M = np.triu(u, 1)
    M = M + M.T
    d = 0.05 + 0.225 * (I.uniform_pm1(seed + 1, n) + 1.0)
    M[np.arange(n), np.arange(n)] = d
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    return I.CSR(n, rp, col, M.reshape(-1).copy())


def _cholesky_fails(D):
    try:
        np.linalg.cholesky(D)
    except np.linalg.LinAlgError:
        return True
    return False


@pytest.mark.parametrize("n,seed", [(7, 11), (24, 12), (40, 13), (49, 14)])
def test_single_level_lu_solve_matches_lapack(oracle_mod, n, seed):
    A = dense_indefinite(n, seed)
    D = A.to_dense()
    assert _cholesky_fails(D) and np.linalg.eigvalsh(D).min() < 0
    h = oracle_mod.OracleAMG(A)
    assert h.nlev == 1
    for rs in (1, 2, 3):
        b = I.rhs(n, rs)
        x = h.level_op(0, 4, b, None, n)
        xs = np.linalg.solve(D, b)
        kappa = np.linalg.cond(D)
        # partial pivoting is backward stable: small residual relative to |A||x|
        assert np.linalg.norm(b - D @ x) <= 64 * n * EPS * np.linalg.norm(D, 2) * np.linalg.norm(x)
        assert np.linalg.norm(x - xs) <= 64 * n * EPS * kappa * np.linalg.norm(xs)
    # a direct solve on a one-level hierarchy: one stationary iteration,
    # residual at the rounding level
    b = I.rhs(n, 4)
    x, res = h.solve(b, method=0, tol=1e-10, maxit=3)
    assert res.converged and res.iters == 1


def test_single_level_lu_solve_is_exact_on_a_permutation_case(oracle_mod):
    """[[e, 1, 0], [1, e, 1], [0, 1, e]] with e = 2^-10: the first pivot is
    tiny, partial pivoting swaps rows 0 and 1; the exact inverse applied to
    b = A (1, 2, 3)^T must return (1, 2, 3) to rounding."""
    e = 2.0 ** -10
    D = np.array([[e, 1, 0], [1, e, 1], [0, 1, e]], float)
    A = I.CSR(3, np.array([0, 2, 5, 7], np.int32), np.array([0, 1, 0, 1, 2, 1, 2], np.int32),
              np.array([e, 1, 1, e, 1, 1, e], float))
    h = oracle_mod.OracleAMG(A)
    xt = np.array([1.0, 2.0, 3.0])
    x = h.level_op(0, 4, D @ xt, None, 3)
    assert np.max(np.abs(x - xt)) <= 1e-14


def test_indefinite_coarsest_level_multilevel(oracle_mod):
    A = shifted_poisson2d(16, 0.1)
    D0 = A.to_dense()
    assert (np.linalg.eigvalsh(D0) < 0).sum() == 1
    h = oracle_mod.OracleAMG(A)
    L = h.nlev - 1
    assert L >= 2
    DL = h.export(L, "AHAT").to_dense()
    assert _cholesky_fails(DL) and np.linalg.eigvalsh(DL).min() < 0
    nL = DL.shape[0]
    for rs in (5, 6):
        bL = I.rhs(nL, rs)
        xL = h.level_op(L, 4, bL, None, nL)
        xs = np.linalg.solve(DL, bL)
        assert np.linalg.norm(xL - xs) <= 64 * nL * EPS * np.linalg.cond(DL) * np.linalg.norm(xs)
    # the whole V-cycle equals the dense recursion built with an explicit
    # inverse of the coarsest operator
    E, B = dense_vcycle_operators(h)
    n = A.n
    Ev = np.stack([h.vcycle(np.zeros(n), e) for e in np.eye(n)], 1)
    Bv = np.stack([h.vcycle(e, np.zeros(n)) for e in np.eye(n)], 1)
    assert np.max(np.abs(Ev - E)) < 1e-11
    assert np.max(np.abs(Bv - B)) < 1e-11 * max(1.0, np.max(np.abs(B)))
    # stationary AMG converges (spectral radius of E below one) to the
    # direct solution; CG breaks down, p^T A p <= 0 on an indefinite matrix
    assert max(abs(np.linalg.eigvals(E))) < 1.0
    b = I.rhs(n, 1)
    x, res = h.solve(b, method=0, tol=1e-10, maxit=100)
    assert res.converged
    xs = np.linalg.solve(D0, b)
    assert np.linalg.norm(x - xs) <= 10 * np.linalg.cond(D0) * 1e-10 * np.linalg.norm(xs)
    x, res = h.solve(b, method=1, tol=1e-10, maxit=100)
    assert res.status == -6
