"""Pins of the oracle's sparsification (Algorithm 3 keep set with the
diagonal-lumping loop of Algorithm 3b, Sparse Galerkin) and reintroduction
(Section 6): brute-force minimal pattern, Theorem 1 and its Remark,
row-sum and symmetry invariants, and the worked Example of Section 6."""
import math
import os

import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53

PROBLEMS = {
    "poisson2d": lambda: I.poisson2d(24),
    "poisson3d": lambda: I.poisson3d(10),
    "aniso2d": lambda: I.aniso2d(24),
    "fv3d": lambda: I.fv3d_lognormal(8),
    "graph": lambda: I.random_graph_laplacian(600),
}


def dense_pattern(S):
    pat = np.zeros((S.nrows, S.ncols), dtype=bool)
    rows = np.repeat(np.arange(S.nrows), np.diff(S.row_ptr))
    pat[rows, S.col] = True
    return pat


def mask_to_dense(h, l, mask):
    A = h.export(l, "A")
    d = np.zeros((A.nrows, A.ncols), dtype=bool)
    rows = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr))
    d[rows, A.col] = mask.astype(bool)
    return d


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_minimal_pattern_brute_force(oracle_mod, name):
    """M_l = edges(Phat^T A P + P^T A Phat) with A = A_{l-1} (Algorithm 3),
    computed with dense nonnegative products so that no cancellation hides a
    structural entry."""
    h = oracle_mod.OracleAMG(PROBLEMS[name]())
    for l in range(1, h.nlev):
        A = (h.export(l - 1, "A").to_dense() != 0).astype(float)
        P = np.abs(h.export(l - 1, "P").to_dense())
        cf = h.cf(l - 1).astype(bool)
        Phat = np.zeros_like(P)
        Phat[np.nonzero(cf)[0], np.arange(cf.sum())] = 1.0
        X = (Phat.T @ A @ P) > 0
        M = X | X.T
        got = mask_to_dense(h, l, h.mask(l, "M"))
        assert np.array_equal(got, M)
        assert not (M & ~dense_pattern(h.export(l, "A"))).any()


@pytest.mark.parametrize("name", ["poisson2d", "poisson3d"])
def test_minimal_pattern_is_full_on_level1_red_black(oracle_mod, name):
    """With red-black coarsening of the 5/7-point stencil every entry of A_1
    lies in M_1, so level 1 cannot drop anything at any gamma."""
    h = oracle_mod.OracleAMG(PROBLEMS[name]())
    assert h.mask(1, "M").all()
    h.sparsify([0.0] + [1.0] * (h.nlev - 1))
    assert h.sizes(1)["nnz_hat"] == h.sizes(1)["nnz"]


def _check_invariants(h, l, gamma):
    A = h.export(l, "A")
    Ah = h.export(l, "AHAT")
    Ad, Hd = A.to_dense(), Ah.to_dense()
    n = A.nrows
    # symmetric, bitwise
    assert np.array_equal(Hd, Hd.T)
    # kept entries are copied unchanged; diagonal stays in the pattern
    patA, patH = dense_pattern(A), dense_pattern(Ah)
    assert not (patH & ~patA).any()
    off = patH & ~np.eye(n, dtype=bool)
    assert np.array_equal(Hd[off], Ad[off])
    assert patH[np.arange(n), np.arange(n)].all()
    # M is never dropped
    M = mask_to_dense(h, l, h.mask(l, "M"))
    assert not (M & ~patH).any()
    # dropped entries are exactly those outside M that are weak in both rows
    m = np.max(np.abs(Ad - np.diag(np.diag(Ad))), axis=1)
    dropped = patA & ~patH
    for i, j in zip(*np.nonzero(dropped)):
        assert not M[i, j]
        assert abs(Ad[i, j]) < gamma * m[i] and abs(Ad[i, j]) < gamma * m[j]
    kept_off = patH & ~M & ~np.eye(n, dtype=bool)
    for i, j in zip(*np.nonzero(kept_off)):
        assert abs(Ad[i, j]) >= gamma * m[i] or abs(Ad[i, j]) >= gamma * m[j]
    # row sums preserved up to one rounding per lumped entry
    for i in range(n):
        a_row = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
        h_row = Ah.val[Ah.row_ptr[i]:Ah.row_ptr[i + 1]]
        d_i = int(dropped[i].sum())
        bound = (d_i + 1) * U * math.fsum(np.abs(a_row)) + 1e-300
        assert abs(math.fsum(h_row) - math.fsum(a_row)) <= bound
    # Gershgorin margin never decreases (Theorem 1 proof: discs never move left)
    margin_a = np.diag(Ad) - (np.abs(Ad).sum(1) - np.abs(np.diag(Ad)))
    margin_h = np.diag(Hd) - (np.abs(Hd).sum(1) - np.abs(np.diag(Hd)))
    assert np.all(margin_h >= margin_a - 1e-13 * np.abs(np.diag(Ad)))
    return Ad, Hd, margin_a


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.01, 0.1, 1.0])
def test_sparsify_invariants(oracle_mod, name, gamma):
    h = oracle_mod.OracleAMG(PROBLEMS[name]())
    h.sparsify([0.0] + [gamma] * (h.nlev - 1))
    for l in range(1, h.nlev):
        Ad, Hd, margin = _check_invariants(h, l, gamma)
        # Theorem 1 and the Remark: for a diagonally dominant SPD A_l with a
        # strictly dominant row the lumped operator is SPD.
        if np.all(margin >= -1e-13 * np.abs(np.diag(Ad))) and np.any(margin > 1e-12):
            np.linalg.cholesky(Hd)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_gamma_zero_is_galerkin_and_patterns_nest(oracle_mod, name):
    h = oracle_mod.OracleAMG(PROBLEMS[name]())
    L = h.nlev
    h.sparsify([0.0] * L)
    for l in range(L):
        A, Ah = h.export(l, "A"), h.export(l, "AHAT")
        assert np.array_equal(A.row_ptr, Ah.row_ptr) and np.array_equal(A.col, Ah.col)
        assert A.val.tobytes() == Ah.val.tobytes()
    pats = []
    for g in (0.01, 0.1, 1.0):
        h.sparsify([0.0] + [g] * (L - 1))
        pats.append([dense_pattern(h.export(l, "AHAT")) for l in range(L)])
    for l in range(L):
        assert not (pats[1][l] & ~pats[0][l]).any()
        assert not (pats[2][l] & ~pats[1][l]).any()


def test_reintroduce_equals_fresh_sparsify(oracle_mod):
    """Entries are restored from the retained Galerkin operator (Section 3.1):
    lowering gamma and re-sparsifying gives bitwise the operator a fresh
    sparsify at the lower gamma gives."""
    A = I.poisson3d(12)
    h = oracle_mod.OracleAMG(A)
    L = h.nlev
    h.sparsify([0.0, 0.0] + [1.0] * (L - 2))
    rc, first = h.reintroduce(s=1)
    assert rc == 0 and first == 2
    assert h.gamma(2) == 0.1
    ref = oracle_mod.OracleAMG(A)
    ref.sparsify([0.0, 0.0, 0.1] + [1.0] * (L - 3))
    for l in range(L):
        a, b = h.export(l, "AHAT"), ref.export(l, "AHAT")
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
        assert a.val.tobytes() == b.val.tobytes()


def test_adaptive_example_gamma_ladder(oracle_mod):
    """Replays the Example of Section 6 on a hierarchy with six coarse
    operators (2D Poisson 160^2 has levels 0..6)."""
    fx = {}
    for line in open(os.path.join(GOLDEN, "adaptive_example_gamma.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            fx[k] = [float(t) for t in v]
    h = oracle_mod.OracleAMG(I.poisson2d(160))
    assert h.nlev == 7
    h.sparsify([0.0] + fx["initial"])
    gam = lambda: [h.gamma(l) for l in range(1, 7)]
    assert gam() == fx["initial"]
    rc, first = h.reintroduce(s=int(fx["s"][0]), gamma_min=fx["gamma_min"][0])
    assert rc == 0 and first == int(fx["changed1"][0])
    assert gam() == fx["after1"]
    rc, first = h.reintroduce(s=int(fx["s"][0]), gamma_min=fx["gamma_min"][0])
    assert rc == 0 and first == int(fx["changed2"][0])
    assert gam() == fx["after2"]
    # the ladder ends when every coarse gamma is 0
    for _ in range(20):
        rc, first = h.reintroduce(s=2)
        if rc == 1:
            break
    assert rc == 1 and first == -1 and gam() == [0.0] * 6


def test_gamma_out_of_range_rejected(oracle_mod):
    h = oracle_mod.OracleAMG(I.poisson2d(16))
    with pytest.raises(ValueError):
        h.sparsify([0.0, 1.5] + [0.0] * (h.nlev - 2))
    with pytest.raises(ValueError):
        h.sparsify([0.0, float("nan")] + [0.0] * (h.nlev - 2))
