"""The device setup (amg_setup_device: strength, C/F split, direct
interpolation and Galerkin product, Section 2's amg_setup, in device kernels)
through the C ABI.

Bars (bit-exact, as for the host setup):
  * Ruge-Stueben coarsening: every level's A, P, R and C/F split equal the
    oracle's and the host setup's;
  * PMIS coarsening: every level equals the oracle's PMIS hierarchy with the
    same seed;
  * solves and sparsification on a device-built hierarchy meet the bars of
    the host-built one (equal iteration counts, solution within 1e-10;
    sparsified patterns and kept values bit-exact);
  * malformed input is rejected with AMG_ERR_BAD_MATRIX naming the row.
"""
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


class _Csr:
    """A library export (nrows, ncols, row_ptr, col, val) in the oracle's form."""

    def __init__(self, t):
        _, _, self.row_ptr, self.col, self.val = t


def _export(h, l, which):
    m = h.export(l, which)
    return _Csr(m) if isinstance(m, tuple) else m


def same_hierarchy(g, o, split_of_o):
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        assert same_csr(g.export(l, "A"), _export(o, l, "A")), ("A", l)
        if l < o.nlev - 1:
            assert same_csr(g.export(l, "P"), _export(o, l, "P")), ("P", l)
            assert same_csr(g.export(l, "R"), _export(o, l, "R")), ("R", l)
            assert np.array_equal(g.split(l), split_of_o(l)), ("split", l)


def oracle(A, **kw):
    from oracle import oracle as O
    return O.OracleAMG(A, **kw)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_rs_device_setup_equals_oracle(lib, name):
    A = PROBLEMS[name]()
    g = lib.Hierarchy(A, setup="device", coarsening="rs")
    o = oracle(A)
    same_hierarchy(g, o, o.cf)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("seed", [0, 7])
def test_pmis_device_setup_equals_oracle(lib, name, seed):
    A = PROBLEMS[name]()
    g = lib.Hierarchy(A, setup="device", coarsening="pmis", seed=seed)
    o = oracle(A, coarsening="pmis", seed=seed)
    same_hierarchy(g, o, o.cf)


@pytest.mark.parametrize("coarsening", ["rs", "pmis"])
def test_device_setup_several_tiles(lib, coarsening):
    A = I.poisson3d(41)       # 68,921 rows: many workgroups and a ragged last one
    g = lib.Hierarchy(A, setup="device", coarsening=coarsening, seed=3)
    o = oracle(A, coarsening=coarsening, seed=3)
    same_hierarchy(g, o, o.cf)


def test_device_setup_from_device_tensors(lib):
    A = I.fv3d_lognormal(14)
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(A.col.astype(np.int32)).cuda()
    v = torch.from_numpy(A.val.astype(np.float64)).cuda()
    g = lib.Hierarchy((A.n, rp, ci, v), setup="device", coarsening="rs")
    h = lib.Hierarchy(A)
    same_hierarchy(g, h, h.split)


def test_pmis_solve_and_sparsify_parity(lib):
    A = I.poisson3d(24)
    b = I.rhs(A.n, 5)
    g = lib.Hierarchy(A, setup="device", coarsening="pmis", seed=1)
    o = oracle(A, coarsening="pmis", seed=1)
    gam = [0.0, 0.0] + [0.1] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    compare_levels(g, o)
    for method in (0, 1):
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        kw = dict(method=method, tol=1e-10, maxit=400)
        rg = g.solve(dev(b), xd, **kw)
        xo, ro = o.solve(b, **kw)
        assert ro.converged
        _assert_solve_parity(host(xd), rg, xo, ro, kw["tol"])


def test_pmis_adaptive_reintroduction_parity(lib):
    A = I.aniso2d(64)
    b = I.rhs(A.n, 9)
    g = lib.Hierarchy(A, setup="device", coarsening="pmis", seed=4)
    o = oracle(A, coarsening="pmis", seed=4)
    gam = [0.0, 0.0] + [1.0] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    kw = dict(method=1, tol=1e-10, maxit=300, adaptive=True, k=2, s=1, rho_max=0.0)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(dev(b), xd, **kw)
    xo, ro = o.solve(b, **kw)
    assert ro.reintroductions >= 1
    _assert_solve_parity(host(xd), rg, xo, ro, kw["tol"])
    compare_levels(g, o)


def test_single_level_and_level_cap(lib):
    A = I.poisson2d(6)          # 36 rows <= 49: no coarsening
    g = lib.Hierarchy(A, setup="device", coarsening="pmis")
    assert g.nlev == 1
    B = I.poisson2d(30)
    g = lib.Hierarchy(B, setup="device", coarsening="rs", max_levels=2)
    o = oracle(B, max_levels=2)
    assert g.nlev == o.nlev == 2
    same_hierarchy(g, o, o.cf)
    x = torch.zeros(B.n, dtype=torch.float64, device="cuda")
    r = g.solve(dev(I.rhs(B.n, 1)), x, method=1, tol=1e-10, maxit=200)
    assert r.converged


def _bad(A, **kw):
    from paper_1512_04629_amd.inputs import CSR
    return CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy(), **kw)


def test_malformed_input_rejected(lib):
    A = I.poisson2d(8)
    row = 10
    b0, e0 = A.row_ptr[row], A.row_ptr[row + 1]
    cases = []
    m = _bad(A); m.col[b0], m.col[b0 + 1] = m.col[b0 + 1], m.col[b0]; cases.append(("ascending", m))
    m = _bad(A); m.val[b0] = m.val[b0] * 1.5; cases.append(("symmetric", m))
    m = _bad(A); m.val[np.nonzero(m.col[b0:e0] == row)[0][0] + b0] = 0.0; cases.append(("diagonal", m))
    m = _bad(A); m.val[b0] = np.nan; cases.append(("non-finite", m))
    m = _bad(A); m.col[b0] = A.n + 5; cases.append(("range", m))
    for what, m in cases:
        with pytest.raises(lib.AmgError) as e:
            lib.Hierarchy(m, setup="device", coarsening="pmis")
        assert e.value.status == -2, what
        assert what in str(e.value), (what, str(e.value))
    # row_ptr that does not end at nnz
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([A.col, [0]]).astype(np.int32)).cuda()
    v = torch.from_numpy(np.concatenate([A.val, [1.0]])).cuda()
    with pytest.raises(lib.AmgError) as e:
        lib.Hierarchy((A.n, rp, ci, v), setup="device")
    assert e.value.status == -2 and "row_ptr" in str(e.value)
    with pytest.raises(ValueError):
        lib.Hierarchy(A, coarsening="pmis")


def test_full_size_rs_device_setup_equals_host_setup(lib):
    """128^3 7-point Poisson (2,097,152 rows): the device-built hierarchy is the
    host-built one bit for bit, level by level."""
    A = I.poisson3d(128)
    g = lib.Hierarchy(A, setup="device", coarsening="rs")
    h = lib.Hierarchy(A)
    same_hierarchy(g, h, h.split)
