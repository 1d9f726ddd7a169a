"""Pins of the oracle's Hybrid Galerkin sparsification (Section 3,
sparse_hybrid_setup, hybrid branch): the minimal pattern of level l comes from
the sparsified finer operator \\hat A_{l-1} instead of the Galerkin A_{l-1}.

* brute force: M_l = edges(Phat^T \\hat A_{l-1} P + P^T \\hat A_{l-1} Phat) with
  dense nonnegative products;
* special case: where the finer level is not sparsified (\\hat A_{l-1} = A_{l-1})
  Hybrid equals Sparse Galerkin bit for bit;
* M and the kept pattern are nested inside Sparse Galerkin's; every
  sparsified operator keeps the Theorem 1 invariants (symmetry, copied kept
  entries, row sums, Gershgorin margins);
* reintroduction under Hybrid Galerkin equals a fresh Hybrid sparsify at the
  lowered tolerances (a coarser level's M follows the operator just changed).
"""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_oracle_sparsify import PROBLEMS, _check_invariants, dense_pattern, mask_to_dense


def _brute_M(h, l):
    A = (h.export(l - 1, "AHAT").to_dense() != 0).astype(float)
    P = np.abs(h.export(l - 1, "P").to_dense())
    cf = h.cf(l - 1).astype(bool)
    Phat = np.zeros_like(P)
    Phat[np.nonzero(cf)[0], np.arange(cf.sum())] = 1.0
    X = (Phat.T @ A @ P) > 0
    return X | X.T


def _same(a, b):
    return (np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
            and a.val.tobytes() == b.val.tobytes())


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.1, 1.0])
def test_hybrid_minimal_pattern_brute_force_and_invariants(oracle_mod, name, gamma):
    h = oracle_mod.OracleAMG(PROBLEMS[name]())
    h.set_method(True)
    h.sparsify([0.0] + [gamma] * (h.nlev - 1))
    for l in range(1, h.nlev):
        assert np.array_equal(mask_to_dense(h, l, h.mask(l, "M")), _brute_M(h, l)), l
        _check_invariants(h, l, gamma)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_hybrid_nests_inside_sparse_galerkin(oracle_mod, name):
    A = PROBLEMS[name]()
    s, hy = oracle_mod.OracleAMG(A), oracle_mod.OracleAMG(A)
    hy.set_method(True)
    g = [0.0] + [0.1] * (s.nlev - 1)
    s.sparsify(g)
    hy.sparsify(g)
    for l in range(1, s.nlev):
        ms, mh = s.mask(l, "M").astype(bool), hy.mask(l, "M").astype(bool)
        assert not (mh & ~ms).any()
        ps, ph = dense_pattern(s.export(l, "AHAT")), dense_pattern(hy.export(l, "AHAT"))
        assert not (ph & ~ps).any()
    # level 1's finer operator is A_0 in both methods
    assert _same(s.export(1, "AHAT"), hy.export(1, "AHAT"))


def test_hybrid_equals_sparse_below_an_unsparsified_level(oracle_mod):
    """gamma_1 = gamma_2 = 0: \\hat A_2 = A_2, so M_3 and \\hat A_3 agree with Sparse
    Galerkin; from level 4 on Hybrid may drop more."""
    A = I.poisson2d(48)
    s, hy = oracle_mod.OracleAMG(A), oracle_mod.OracleAMG(A)
    hy.set_method(True)
    L = s.nlev
    assert L >= 5
    g = [0.0, 0.0, 0.0] + [0.1] * (L - 3)
    s.sparsify(g)
    hy.sparsify(g)
    for l in range(0, 4):
        assert _same(s.export(l, "AHAT"), hy.export(l, "AHAT")), l
        if l >= 1:
            assert np.array_equal(s.mask(l, "M"), hy.mask(l, "M")), l


def test_method_switch_rebuilds_M(oracle_mod):
    A = I.aniso2d(32)
    h = oracle_mod.OracleAMG(A)
    ref = [h.mask(l, "M").copy() for l in range(1, h.nlev)]
    h.set_method(True)
    h.sparsify([0.0] + [1.0] * (h.nlev - 1))
    h.set_method(False)
    for l in range(1, h.nlev):
        assert np.array_equal(h.mask(l, "M"), ref[l - 1])


def test_hybrid_reintroduce_equals_fresh_sparsify(oracle_mod):
    A = I.poisson3d(14)
    h = oracle_mod.OracleAMG(A)
    h.set_method(True)
    L = h.nlev
    h.sparsify([0.0, 0.0] + [1.0] * (L - 2))
    rc, first = h.reintroduce(s=1)
    assert rc == 0 and first == 2
    ref = oracle_mod.OracleAMG(A)
    ref.set_method(True)
    ref.sparsify([0.0, 0.0, 0.1] + [1.0] * (L - 3))
    for l in range(L):
        assert _same(h.export(l, "AHAT"), ref.export(l, "AHAT")), l
        if l >= 1:
            assert np.array_equal(h.mask(l, "M"), ref.mask(l, "M")), l
