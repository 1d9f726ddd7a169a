"""Pins of the oracle's strong-neighbour lumping (Algorithm 3, second loop):
a dropped entry (i,j) is shared among the strong neighbours m of j that row
i keeps, in proportion |a_jm|; each share goes to (i,m) and (m,i) and comes
off (m,m) (added once to (i,i) when m = i); with no such neighbour it goes
to the diagonal.

* a 4x4 worked example whose values were derived by hand from that rule;
* a dropped entry whose row j has no strong entry goes to the diagonal, as
  Algorithm 3b would put it;
* on hierarchies: the result is bitwise symmetric, keeps every row sum
  (within rounding), has the same pattern as diagonal lumping, and
  gamma = 0 leaves the operators unchanged; PCG still converges.
"""
import math

import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_oracle_sparsify import PROBLEMS, dense_pattern


def _csr(rows):
    n = len(rows)
    rp, ci, v = [0], [], []
    for r in rows:
        for j, a in sorted(r.items()):
            ci.append(j); v.append(a)
        rp.append(len(ci))
    return I.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64))


def test_worked_example_four_by_four(oracle_mod):
    # A = [[4,-1,-1,-.5],[-1,4,-1,0],[-1,-1,4,-1],[-.5,0,-1,4]], (0,3) and (3,0) dropped.
    # Strong sets (theta 1/4): row 3 -> {0, 2}; row 0 -> {1, 2, 3}.
    # (0,3): W = {0, 2}, shares of -0.5 in 0.5 : 1  -> (0,0) += -1/6; (0,2),(2,0) += -1/3, (2,2) -= -1/3
    # (3,0): W = {2, 3} ((3,1) is not stored), shares 1 : 0.5 -> (3,2),(2,3) += -1/3, (2,2) -= -1/3;
    #        (3,3) += -1/6
    A = _csr([{0: 4.0, 1: -1.0, 2: -1.0, 3: -0.5}, {0: -1.0, 1: 4.0, 2: -1.0},
              {0: -1.0, 1: -1.0, 2: 4.0, 3: -1.0}, {0: -0.5, 2: -1.0, 3: 4.0}])
    keep = np.ones(len(A.col), np.uint8)
    keep[3] = 0                      # (0,3)
    keep[len(A.col) - 3] = 0         # (3,0)
    got = oracle_mod.strong_lump(A, keep)
    t = 1.0 / 3.0
    want = [4 - 1 / 6, -1, -1 - t,          # row 0: (0,0) (0,1) (0,2)
            -1, 4, -1,                      # row 1
            -1 - t, -1, 4 + 2 * t, -1 - t,  # row 2
            -1 - t, 4 - 1 / 6]              # row 3: (3,2) (3,3)
    assert np.allclose(got, want, rtol=0, atol=1e-15)


def test_no_strong_neighbour_goes_to_the_diagonal(oracle_mod):
    # row 1 has no negative coupling, so no strong entry: (0,1) and (1,0) lump
    A = _csr([{0: 2.0, 1: 0.5}, {0: 0.5, 1: 2.0}])
    got = oracle_mod.strong_lump(A, np.array([1, 0, 0, 1], np.uint8))
    assert np.array_equal(got, [2.5, 2.5])


def _check(h, l, gamma):
    A = h.export(l, "A")
    Ah = h.export(l, "AHAT")
    D, Dh = A.to_dense(), Ah.to_dense()
    assert np.array_equal(Dh, Dh.T), "not bitwise symmetric"
    for i in range(A.nrows):
        a = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
        ah = Ah.val[Ah.row_ptr[i]:Ah.row_ptr[i + 1]]
        assert abs(math.fsum(ah) - math.fsum(a)) <= 1e-13 * math.fsum(np.abs(a)), i
    return dense_pattern(Ah)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.01, 0.1, 1.0])
def test_invariants_and_pattern(oracle_mod, name, gamma):
    A = PROBLEMS[name]()
    s, d = oracle_mod.OracleAMG(A), oracle_mod.OracleAMG(A)
    s.set_lumping("strong")
    gam = [0.0] + [gamma] * (s.nlev - 1)
    s.sparsify(gam)
    d.sparsify(gam)
    for l in range(1, s.nlev):
        pat = _check(s, l, gamma)
        assert np.array_equal(pat, dense_pattern(d.export(l, "AHAT"))), l


def test_gamma_zero_is_identity_and_solves_converge(oracle_mod):
    A = I.poisson3d(14)
    h = oracle_mod.OracleAMG(A)
    h.set_lumping("strong")
    h.sparsify([0.0] * 20)
    for l in range(h.nlev):
        a, ah = h.export(l, "A"), h.export(l, "AHAT")
        assert a.val.tobytes() == ah.val.tobytes()
    h.sparsify([0.0, 0.0] + [1.0] * 20)
    b = I.rhs(A.n, 3)
    x, r = h.solve(b, method=oracle_mod.PCG, tol=1e-10, maxit=300)
    assert r.converged
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-10 * np.linalg.norm(b)
    with pytest.raises(ValueError):
        h.set_lumping("neighbours")
