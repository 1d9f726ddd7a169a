"""Pins of the oracle's method of non-Galerkin coarse grids (Section 2.1 and
amg_setup's optional sparsify): each coarse product is sparsified as soon as
it is formed and the result replaces it, so the next level is built from it.

* gamma 0 everywhere gives the Galerkin hierarchy bit for bit;
* every coarse operator is the dense product P^T A_l P of the hierarchy's own
  finer operator, sparsified: pattern inside the product's, symmetric, kept
  off-diagonal entries equal to the product's, row sums preserved, every
  dropped entry outside the brute-force minimal pattern and weak in both rows;
* the next level is built from the sparsified operator: its C/F split and
  interpolation equal those of a fresh hierarchy whose fine matrix is that
  operator.
"""
import math

import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_oracle_sparsify import PROBLEMS, dense_pattern

U = 2.0 ** -53


def _same(a, b):
    return (np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
            and a.val.tobytes() == b.val.tobytes())


def _csr_from(h, l):
    from paper_1512_04629_amd.inputs import CSR
    m = h.export(l, "A")
    return CSR(m.nrows, m.row_ptr.copy(), m.col.copy(), m.val.copy())


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_gamma_zero_is_the_galerkin_hierarchy(oracle_mod, name):
    A = PROBLEMS[name]()
    g = oracle_mod.OracleAMG(A)
    ng = oracle_mod.OracleAMG(A, nongalerkin_gamma=[0.0] * 30)
    assert g.nlev == ng.nlev
    for l in range(g.nlev):
        assert _same(g.export(l, "A"), ng.export(l, "A"))
        if l < g.nlev - 1:
            assert _same(g.export(l, "P"), ng.export(l, "P"))


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.1, 1.0])
def test_coarse_operators_are_sparsified_products(oracle_mod, name, gamma):
    A = PROBLEMS[name]()
    h = oracle_mod.OracleAMG(A, nongalerkin_gamma=[0.0] + [gamma] * 30)
    for l in range(h.nlev - 1):
        Af = h.export(l, "A").to_dense()
        P = h.export(l, "P").to_dense()
        prod = P.T @ Af @ P
        C = h.export(l + 1, "A")
        Cd = C.to_dense()
        n = C.nrows
        patC = dense_pattern(C)
        patProd = ((np.abs(P).T @ (Af != 0).astype(float) @ np.abs(P)) > 0)
        assert not (patC & ~patProd).any()
        assert np.array_equal(Cd, Cd.T)
        scale = np.abs(P).T @ np.abs(Af) @ np.abs(P)
        off = patC & ~np.eye(n, dtype=bool)
        assert np.all(np.abs(Cd[off] - prod[off]) <= 1e-13 * scale[off] + 1e-300)
        # minimal pattern from the finer operator (brute force) and the keep rule
        cf = h.cf(l).astype(bool)
        Phat = np.zeros_like(P)
        Phat[np.nonzero(cf)[0], np.arange(cf.sum())] = 1.0
        X = (Phat.T @ (Af != 0).astype(float) @ np.abs(P)) > 0
        M = X | X.T
        assert not (M & ~patC).any()
        m = np.max(np.abs(prod - np.diag(np.diag(prod))) * patProd, axis=1)
        dropped = patProd & ~patC & ~np.eye(n, dtype=bool)
        for i, j in zip(*np.nonzero(dropped)):
            tol = 1e-12 * scale[i, j]
            assert abs(prod[i, j]) < gamma * m[i] + tol and abs(prod[i, j]) < gamma * m[j] + tol
        # row sums preserved (lumping to the diagonal)
        for i in range(n):
            row = C.val[C.row_ptr[i]:C.row_ptr[i + 1]]
            assert abs(math.fsum(row) - math.fsum(prod[i][patProd[i]])) <= 1e-12 * scale[i].sum()


def test_next_level_is_built_from_the_sparsified_operator(oracle_mod):
    A = I.poisson3d(16)
    h = oracle_mod.OracleAMG(A, nongalerkin_gamma=[0.0, 0.0, 0.5, 0.5, 0.5, 0.5])
    g = oracle_mod.OracleAMG(A)
    assert h.sizes(2)["nnz"] < g.sizes(2)["nnz"]
    for l in (1, 2):
        if l >= h.nlev - 1:
            break
        fresh = oracle_mod.OracleAMG(_csr_from(h, l), nongalerkin_gamma=[0.0, 0.5, 0.5, 0.5, 0.5])
        assert np.array_equal(fresh.cf(0), h.cf(l))
        assert _same(fresh.export(0, "P"), h.export(l, "P"))
        assert _same(fresh.export(1, "A"), h.export(l + 1, "A"))


def test_nongalerkin_solves(oracle_mod):
    """The non-Galerkin hierarchy still solves (Section 2.1: it trades an
    A-orthogonal coarse correction for fewer nonzeros)."""
    A = I.poisson3d(16)
    b = I.rhs(A.n, 4)
    h = oracle_mod.OracleAMG(A, nongalerkin_gamma=[0.0, 0.0] + [0.1] * 10)
    x, r = h.solve(b, method=oracle_mod.PCG, tol=1e-10, maxit=100)
    assert r.converged
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-10 * np.linalg.norm(b)
