"""Pins of the oracle's hybrid Gauss-Seidel relaxation (the relaxation of the
paper's experiments, Section 5): Gauss-Seidel inside contiguous row blocks,
Jacobi across them; forward sweeps before the coarse correction and backward
sweeps after it.

* one row per block is Jacobi with weight 1;
* one block holding every row is textbook Gauss-Seidel: the lower (forward)
  or upper (backward) triangular solve of a library routine;
* any block size equals per-block triangular solves with the other blocks'
  old values moved to the right-hand side;
* the V-cycle with forward pre- and backward post-sweeps is a symmetric
  operator (a forward post-sweep is not), so it can precondition CG;
* solves converge; with one block (textbook Gauss-Seidel) in fewer iterations
  than with weighted Jacobi on Poisson (small blocks leave most couplings to
  an unweighted Jacobi part and converge more slowly).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1512_04629_amd import inputs as I

FWD, BWD = 7, 8


def _sweep(h, b, x, op):
    return h.level_op(0, op, b, x, h.n)


def test_block_one_is_jacobi_weight_one(oracle_mod):
    A = I.aniso2d(10)
    h = oracle_mod.OracleAMG(A)
    h.set_relaxation("hybrid_gs", 1)
    rng = np.random.default_rng(1)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    D = A.to_dense()
    ref = x + (b - D @ x) / np.diag(D)
    for op in (FWD, BWD):
        assert np.allclose(_sweep(h, b, x, op), ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["poisson2d", "aniso2d", "graph"])
def test_one_block_is_textbook_gauss_seidel(oracle_mod, name):
    A = {"poisson2d": lambda: I.poisson2d(9), "aniso2d": lambda: I.aniso2d(8),
         "graph": lambda: I.random_graph_laplacian(70)}[name]()
    h = oracle_mod.OracleAMG(A)
    h.set_relaxation("hybrid_gs", A.n)
    rng = np.random.default_rng(2)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    D = A.to_dense()
    lower, upper = np.tril(D), np.triu(D)
    fwd = sla.solve_triangular(lower, b - np.triu(D, 1) @ x, lower=True)
    bwd = sla.solve_triangular(upper, b - np.tril(D, -1) @ x, lower=False)
    assert np.allclose(_sweep(h, b, x, FWD), fwd, rtol=1e-12, atol=1e-12)
    assert np.allclose(_sweep(h, b, x, BWD), bwd, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("block", [2, 5, 16, 37])
def test_blocks_are_triangular_solves_with_old_values_outside(oracle_mod, block):
    A = I.poisson2d(12)
    h = oracle_mod.OracleAMG(A)
    h.set_relaxation("hybrid_gs", block)
    rng = np.random.default_rng(3)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    D = A.to_dense()
    for op, lower in ((FWD, True), (BWD, False)):
        ref = np.empty(A.n)
        for r0 in range(0, A.n, block):
            blk = slice(r0, min(r0 + block, A.n))
            Dbb = D[blk, blk]
            tri = np.tril(Dbb) if lower else np.triu(Dbb)
            rhs = b[blk] - D[blk] @ x + (D[blk, blk] @ x[blk]) - (Dbb - tri) @ x[blk]
            ref[blk] = sla.solve_triangular(tri, rhs, lower=lower)
        assert np.allclose(_sweep(h, b, x, op), ref, rtol=1e-12, atol=1e-12), op


def _precond_matrix(h, n):
    M = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = h.vcycle(e, np.zeros(n))
    return M


def test_symmetric_cycle_and_a_wrong_direction_breaks_it(oracle_mod):
    A = I.poisson2d(10)
    h = oracle_mod.OracleAMG(A)
    h.set_relaxation("hybrid_gs", 7)
    M = _precond_matrix(h, A.n)
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    # positive definite too (CG needs it)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    # the same sweep twice (forward after as well) is not symmetric
    n = A.n
    Mf = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        x = h.level_op(0, FWD, e, np.zeros(n), n)
        Mf[:, k] = h.level_op(0, FWD, e, x, n)
    assert not np.allclose(Mf, Mf.T, atol=1e-6)


def test_gauss_seidel_solves_converge_faster_than_jacobi(oracle_mod):
    A = I.poisson3d(14)
    b = I.rhs(A.n, 6)
    its = {}
    for kind, block in (("jacobi", 1), ("hybrid_gs", 64), ("hybrid_gs", A.n)):
        h = oracle_mod.OracleAMG(A)
        h.set_relaxation(kind, block)
        for method in (oracle_mod.STATIONARY, oracle_mod.PCG):
            x, r = h.solve(b, method=method, tol=1e-10, maxit=200)
            assert r.converged
            assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-10 * np.linalg.norm(b)
            its[(block, method)] = r.iters
    for method in (oracle_mod.STATIONARY, oracle_mod.PCG):
        assert its[(A.n, method)] < its[(1, method)]
    with pytest.raises(ValueError):
        oracle_mod.OracleAMG(A).set_relaxation("hybrid_gs", 0)
