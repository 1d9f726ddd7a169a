"""Pins of the oracle's PMIS coarsening (the parallel aggressive coarsening of
De Sterck, Yang and Heys that Section 1 cites) and of the hierarchy built on
it.

* the weights' generator is SplitMix64: the oracle's C implementation gives
  the published first outputs and agrees with the input module's separate
  implementation;
* the round-based split equals the sequential greedy characterisation of the
  same independent set: visit the points in decreasing weight order (equal
  weights: smaller index first); a point still undecided becomes C and makes F
  every undecided point that depends strongly on it; points no point depends
  on start as F.  (A point becomes F in the rounds exactly when it depends
  strongly on a C point that beats it, which is the greedy rule.);
* a C point depends strongly on another C point only if it beats it (it was
  chosen first and the other point does not depend on it), so C is
  independent where S is symmetric; every F point that some point depends on
  depends strongly on a C point;
* interpolation and Galerkin pins of the Ruge-Stueben hierarchy hold with the
  PMIS split, and PCG converges on it.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1512_04629_amd import inputs as I

from .test_oracle_setup import PROBLEMS, check_galerkin_dense, check_interpolation, poisson1d

SEEDS = [0, 11]


def _S(h, l):
    S = h.export(l, "S")
    return sp.csr_matrix((np.ones(len(S.col)), S.col, S.row_ptr), shape=(S.nrows, S.nrows))


def greedy_split(S, seed, w=None):
    n = S.shape[0]
    St = S.T.tocsr()
    lam = np.diff(St.indptr)
    if w is None:
        w = lam.astype(np.float64) + I.uniform01(seed, n)
    U, C, F = 0, 1, 2
    state = np.where(lam == 0, F, U)
    for i in sorted(range(n), key=lambda i: (-w[i], i)):
        if state[i] != U:
            continue
        state[i] = C
        for j in St.indices[St.indptr[i]:St.indptr[i + 1]]:
            if state[j] == U:
                state[j] = F
    return (state == C).astype(np.int32)


def test_splitmix64_published_outputs_and_input_module(oracle_mod):
    lib = oracle_mod._load()
    assert [lib.or_splitmix64(0, k) for k in (1, 2, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                          0x06C45D188009454F]
    for seed in (1, 12345, 2 ** 64 - 1):
        ref = I.splitmix64(seed, 64)
        assert [lib.or_splitmix64(seed, k + 1) for k in range(64)] == [int(v) for v in ref]


ALL = dict(PROBLEMS, poisson1d=lambda: poisson1d(200), poisson3d8=lambda: I.poisson3d(8))


@pytest.mark.parametrize("name", sorted(ALL))
@pytest.mark.parametrize("seed", SEEDS)
def test_pmis_equals_greedy_characterisation(oracle_mod, name, seed):
    h = oracle_mod.OracleAMG(ALL[name](), coarsening="pmis", seed=seed)
    assert h.nlev >= 2
    for l in range(h.nlev - 1):
        assert np.array_equal(h.cf(l), greedy_split(_S(h, l), seed + l)), l


@pytest.mark.parametrize("name", ["poisson1d", "poisson2d", "poisson3d8", "aniso2d", "graph"])
def test_pmis_tie_break_smaller_index_wins(oracle_mod, name):
    """Random weights practically never tie; integer weights (lambda alone)
    tie everywhere, and the rounds still equal the greedy order in which equal
    weights are visited by ascending index."""
    h = oracle_mod.OracleAMG(ALL[name](), coarsening="pmis", seed=0)
    lib = oracle_mod._load()
    for l in range(min(h.nlev - 1, 2)):
        S = h.export(l, "S")
        Sm = _S(h, l)
        w = np.diff(Sm.T.tocsr().indptr).astype(np.float64)
        cf = np.zeros(S.nrows, np.int32)
        assert lib.or_pmis_rounds(S.nrows, S.row_ptr, S.col, w, cf) == 0
        assert np.array_equal(cf, greedy_split(Sm, 0, w)), l


@pytest.mark.parametrize("name", sorted(ALL))
def test_pmis_independent_and_covering(oracle_mod, name):
    seed = 3
    h = oracle_mod.OracleAMG(ALL[name](), coarsening="pmis", seed=seed)
    for l in range(h.nlev - 1):
        S = _S(h, l)
        cf = h.cf(l).astype(bool)
        lam = np.diff(S.T.tocsr().indptr)
        w = lam.astype(np.float64) + I.uniform01(seed + l, S.shape[0])
        G = S.tocoo()
        both = cf[G.row] & cf[G.col]
        i, j = G.row[both], G.col[both]
        assert np.all((w[i] > w[j]) | ((w[i] == w[j]) & (i < j)))
        if (S != S.T).nnz == 0:
            assert not both.any()
        hits = S @ cf.astype(np.float64)
        for i in np.nonzero(~cf & (lam > 0))[0]:
            assert hits[i] > 0, i


def test_pmis_one_dimensional_coarsening_ratio(oracle_mod):
    """1D Laplacian: S is the path graph, so C is a maximal independent set of
    the path: no two C neighbours and no two consecutive F points (an F point
    sits between its C neighbours), so between 1/3 and 1/2 of the points are C."""
    h = oracle_mod.OracleAMG(poisson1d(300), coarsening="pmis", seed=5)
    cf = h.cf(0)
    assert not np.any(cf[1:] & cf[:-1])
    f = 1 - cf
    assert not np.any(f[2:] & f[1:-1] & f[:-2])
    assert 300 / 3 - 1 <= cf.sum() <= 300 / 2 + 1


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_pmis_hierarchy_interpolation_and_galerkin(oracle_mod, name):
    h = oracle_mod.OracleAMG(PROBLEMS[name](), coarsening="pmis", seed=1)
    check_interpolation(h)
    check_galerkin_dense(h)


def test_pmis_seed_changes_split_and_pcg_converges(oracle_mod):
    A = I.poisson3d(12)
    a = oracle_mod.OracleAMG(A, coarsening="pmis", seed=1)
    b = oracle_mod.OracleAMG(A, coarsening="pmis", seed=2)
    assert not np.array_equal(a.cf(0), b.cf(0))
    rhs = I.rhs(A.n, 3)
    x, r = a.solve(rhs, method=oracle_mod.PCG, tol=1e-10, maxit=200)
    assert r.converged
    assert np.linalg.norm(rhs - A.to_scipy() @ x) <= 1.01e-10 * np.linalg.norm(rhs)
    with pytest.raises(ValueError):
        oracle_mod.OracleAMG(A, coarsening="hmis")
