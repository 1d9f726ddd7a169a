"""Strong-neighbour lumping (Algorithm 3, second loop) on the device against
the oracle.  Every entry of a sparsified operator is its Galerkin value plus
its shares added in ascending order of their source entry, on the device as
in the oracle, so the operators agree bit for bit, diagonal included; this
holds for both launch shapes (a wave per row, and a workgroup per row with
the row staged in LDS, whose rows longer than the stage go the one-wave
way), each forced in turn, and for the denominators' wave-per-row stage that
levels of short rows take.  Solves: equal iteration counts, solution within
1e-10."""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_gpu_parity import PROBLEMS, _assert_solve_parity, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    amg.load_library()
    return amg


def pair(A, hybrid=False):
    from oracle import oracle as O
    from paper_1512_04629_amd import amg
    g, o = amg.Hierarchy(A), O.OracleAMG(A)
    g.set_lumping("strong")
    o.set_lumping("strong")
    if hybrid:
        g.set_method(True)
        o.set_method(True)
    return g, o


def same_operators(g, o):
    for l in range(o.nlev):
        nr, nc, rp, ci, v = g.export(l, "AHAT")
        ref = o.export(l, "AHAT")
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col), ("pattern", l)
        assert v.tobytes() == ref.val.tobytes(), ("values", l)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("gamma", [0.1, 1.0])
@pytest.mark.parametrize("hybrid", [False, True])
def test_sparsify_bitwise(lib, name, gamma, hybrid):
    A = PROBLEMS[name]()
    g, o = pair(A, hybrid)
    gam = [0.0] + [gamma] * (o.nlev - 1)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    same_operators(g, o)


SHAPES = {"wave": dict(wide_mean_row=1e300), "workgroup": dict(wide_mean_row=0.0),
          "workgroup_256": dict(small_rows=0)}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("path", sorted(SHAPES))
def test_both_launch_shapes_bitwise(lib, name, path):
    """wave: one wave per row on every level; workgroup: a workgroup per row
    (the default); workgroup_256: the share kernel's 256-thread workgroups on
    every level (by default levels of fewer than 4,096 rows, most of these
    problems', take 1,024)."""
    A = PROBLEMS[name]()
    g, o = pair(A)
    g.set_lump_shapes(**SHAPES[path])
    gam = [0.0] + [0.1] * (o.nlev - 1)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    same_operators(g, o)


@pytest.mark.parametrize("path", ["default", "wave", "staged_wave_denominators"])
def test_rows_longer_than_the_stage(lib, path):
    """A graph whose first coarse level has 259 nearly full rows: 148 longer
    than the 256 entries a row's stage holds, 111 not, so one launch takes
    both branches of the staged kernels (the denominators' wave-per-row stage
    forced onto it in the third case)."""
    A = I.random_graph_laplacian(1800, degree=10)
    g, o = pair(A)
    if path == "wave":
        g.set_lump_shapes(wide_mean_row=1e300)
    if path == "staged_wave_denominators":
        g.set_lump_shapes(den_wave_mean_row=1e300)
    a = o.export(1, "A")
    lens = np.diff(a.row_ptr)
    assert (lens > 256).sum() > 0 and (lens <= 256).sum() > 0
    gam = [0.0, 0.1]
    g.sparsify_levels(gam)
    o.sparsify(gam)
    same_operators(g, o)


def test_adaptive_solve_parity(lib):
    A = I.poisson3d(20)
    b = I.rhs(A.n, 4)
    g, o = pair(A)
    gam = [0.0, 0.0] + [1.0] * (o.nlev - 2)
    g.sparsify_levels(gam)
    o.sparsify(gam)
    kw = dict(method=1, tol=1e-10, maxit=300, adaptive=True, k=2, s=1, rho_max=0.0)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rg = g.solve(dev(b), xd, **kw)
    xo, ro = o.solve(b, **kw)
    assert ro.reintroductions >= 1
    _assert_solve_parity(host(xd), rg, xo, ro, kw["tol"])
    same_operators(g, o)


def test_fp32_cycle_and_switching_back(lib):
    A = I.aniso2d(96)
    b = dev(I.rhs(A.n, 5))
    g, o = pair(A)
    g.sparsify(0.1, 2)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r = g.solve(b, x, method=1, tol=1e-10, maxit=300, precision=32)
    assert r.converged
    g.set_lumping("diagonal")
    g.sparsify(0.1, 2)
    from oracle import oracle as O
    d = O.OracleAMG(A)
    d.sparsify_from(0.1, 2)
    for l in range(1, d.nlev):
        assert np.array_equal(g.export(l, "AHAT")[3], d.export(l, "AHAT").col)
    with pytest.raises(ValueError):
        g.set_lumping("neighbours")
    with pytest.raises(lib.AmgError):
        g._check(g._lib.amg_set_lumping(g._h, 2))
