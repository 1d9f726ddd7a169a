"""Pins of the oracle's solve phase: the V-cycle of Section 2 (amg_solve),
stationary AMG, AMG-preconditioned CG and the adaptive solve of Section 6."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_1512_04629_amd import inputs as I
from tests.test_oracle_setup import poisson1d

OMEGA = 2.0 / 3.0


def test_two_grid_factor_1d_is_one_ninth(oracle_mod):
    """1D Poisson, red-black split, linear (= direct) interpolation, V(1,1)
    weighted Jacobi with omega = 2/3: the two-grid error propagator has
    spectral radius exactly 1/9 (Fourier symbol
    (1-4s/3)^2 s + (4s/3-1/3)^2 (1-s) = 1/9 for every frequency s)."""
    for n in (31, 63, 127):
        h = oracle_mod.OracleAMG(poisson1d(n), max_levels=2, max_coarse=1)
        E = np.stack([h.vcycle(np.zeros(n), e) for e in np.eye(n)], 1)
        rho = max(abs(np.linalg.eigvals(E)))
        assert abs(rho - 1.0 / 9.0) < 1e-12


def dense_vcycle_operators(h):
    """E_0 and B_0 of the V-cycle built from the exported operators by the
    recursion E_l = S_l (I - P_l B_{l+1} P_l^T Ahat_l) S_l,
    B_l = (I - E_l) Ahat_l^{-1}, S_l = I - omega D_l^{-1} Ahat_l, E_L = 0."""
    L = h.nlev - 1
    B = np.linalg.inv(h.export(L, "AHAT").to_dense())
    for l in range(L - 1, -1, -1):
        Ah = h.export(l, "AHAT").to_dense()
        P = h.export(l, "P").to_dense()
        n = Ah.shape[0]
        S = np.eye(n) - OMEGA * np.diag(1.0 / np.diag(Ah)) @ Ah
        E = S @ (np.eye(n) - P @ B @ P.T @ Ah) @ S
        B = (np.eye(n) - E) @ np.linalg.inv(Ah)
    return E, B


@pytest.mark.parametrize("make,gammas", [
    (lambda: I.poisson2d(12), (0.0,)),
    (lambda: I.poisson3d(7), (0.0, 0.1, 1.0)),
    (lambda: I.aniso2d(14), (0.01, 1.0)),
    (lambda: I.fv3d_lognormal(6), (0.1,)),
    (lambda: I.random_graph_laplacian(300), (0.1,)),
])
def test_vcycle_matches_dense_recursion(oracle_mod, make, gammas):
    A = make()
    n = A.n
    h = oracle_mod.OracleAMG(A)
    for g in gammas:
        h.sparsify([0.0, 0.0] + [g] * (h.nlev - 2))
        E, B = dense_vcycle_operators(h)
        Ev = np.stack([h.vcycle(np.zeros(n), e) for e in np.eye(n)], 1)
        Bv = np.stack([h.vcycle(e, np.zeros(n)) for e in np.eye(n)], 1)
        assert np.max(np.abs(Ev - E)) < 1e-12
        assert np.max(np.abs(Bv - B)) < 1e-12 * max(1.0, np.max(np.abs(B)))


def test_stationary_factor_matches_spectral_radius(oracle_mod):
    A = I.poisson2d(20)
    h = oracle_mod.OracleAMG(A)
    E, _ = dense_vcycle_operators(h)
    rho = max(abs(np.linalg.eigvals(E)))
    x = I.rhs(A.n, 3)
    b = np.zeros(A.n)
    ratios = []
    prev = np.linalg.norm(x)
    for _ in range(40):
        x = h.vcycle(b, x)
        cur = np.linalg.norm(x)
        ratios.append(cur / prev)
        prev = cur
        if cur < 1e-250:
            break
    assert abs(ratios[-1] - rho) < 0.05 * rho


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("make", [lambda: I.poisson2d(32), lambda: I.aniso2d(24),
                                  lambda: I.fv3d_lognormal(8), lambda: I.random_graph_laplacian(800)])
def test_solution_matches_direct_solve(oracle_mod, method, make):
    A = make()
    b = I.rhs(A.n, 1)
    h = oracle_mod.OracleAMG(A)
    h.sparsify([0.0, 0.0] + [0.1] * (h.nlev - 2))
    x, res = h.solve(b, method=method, tol=1e-10, maxit=400)
    assert res.status == 0 and res.converged
    xs = np.linalg.solve(A.to_dense(), b)
    kappa = np.linalg.cond(A.to_dense())
    assert np.linalg.norm(x - xs) <= 10 * kappa * 1e-10 * np.linalg.norm(xs)
    r = b - A.to_scipy() @ x
    assert abs(np.linalg.norm(r) / np.linalg.norm(b) - res.relres) < 1e-14
    assert res.relres <= 1e-10 * 1.0001


@pytest.mark.parametrize("make", [lambda: I.poisson3d(12), lambda: I.aniso2d(32),
                                  lambda: I.random_graph_laplacian(2000)])
def test_pcg_iterations_match_scipy_cg(oracle_mod, make):
    """The oracle's PCG and scipy's CG with the oracle's V-cycle as the
    preconditioner take the same number of iterations (within one)."""
    A = make()
    b = I.rhs(A.n, 2)
    h = oracle_mod.OracleAMG(A)
    h.sparsify([0.0, 0.0] + [0.1] * (h.nlev - 2))
    x, res = h.solve(b, method=1, tol=1e-8, maxit=200)
    assert res.converged
    M = spla.LinearOperator((A.n, A.n), matvec=lambda r: h.vcycle(r, np.zeros(A.n)))
    count = [0]
    xs, info = spla.cg(A.to_scipy(), b, rtol=1e-8, atol=0.0, M=M, maxiter=200,
                       callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0
    assert abs(count[0] - res.iters) <= 1
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_pcg_terminates_within_n_steps(oracle_mod):
    A = I.random_graph_laplacian(60, degree=3)
    h = oracle_mod.OracleAMG(A, max_coarse=10)
    x, res = h.solve(I.rhs(A.n, 5), method=1, tol=1e-12, maxit=A.n)
    assert res.converged and res.iters <= A.n


def test_residual_history_and_info(oracle_mod):
    A = I.poisson2d(64)
    b = I.rhs(A.n, 1)
    h = oracle_mod.OracleAMG(A)
    h.sparsify_from(0.01, 2)
    x, res = h.solve(b, method=0, tol=1e-8, maxit=100)
    assert res.converged and res.status == 0
    hist = res.hist
    assert len(hist) == res.iters + 1
    assert hist[-1] <= 1e-8 * hist[0] < hist[-2]
    assert np.all(hist[1:] < hist[:-1])
    assert abs(res.rho_avg - res.relres ** (1.0 / res.iters)) < 1e-15


def test_adaptive_reintroduction_forced(oracle_mod):
    """With rho_max = 0 every window of k iterations reintroduces (while some
    coarse gamma is positive); the hierarchy the solve ends with is the one
    the same number of ladder steps gives on a fresh hierarchy, and every
    reintroduction restarts CG."""
    A = I.poisson3d(16)
    b = I.rhs(A.n, 2)
    h = oracle_mod.OracleAMG(A)
    L = h.nlev
    start = [0.0, 0.0] + [1.0] * (L - 2)
    h.sparsify(start)
    x, res = h.solve(b, method=1, tol=1e-12, maxit=200, adaptive=True, k=2, s=1, rho_max=0.0)
    assert res.converged
    windows = min(res.iters // 2, 3 * (L - 2))
    assert res.reintroductions == windows >= 3
    assert res.restarts == res.reintroductions
    ref = oracle_mod.OracleAMG(A)
    ref.sparsify(start)
    for _ in range(res.reintroductions):
        assert ref.reintroduce(s=1)[0] == 0
    for l in range(L):
        assert h.gamma(l) == ref.gamma(l)
        assert h.export(l, "AHAT").val.tobytes() == ref.export(l, "AHAT").val.tobytes()
    xs = np.linalg.solve(A.to_dense(), b) if A.n <= 5000 else None
    if xs is not None:
        assert np.linalg.norm(x - xs) < 1e-9 * np.linalg.norm(xs)


def test_adaptive_no_trigger_equals_plain_pcg(oracle_mod):
    A = I.poisson3d(14)
    b = I.rhs(A.n, 2)
    h = oracle_mod.OracleAMG(A)
    h.sparsify_from(0.1, 2)
    x1, r1 = h.solve(b, method=1, tol=1e-8, maxit=100, adaptive=False)
    x2, r2 = h.solve(b, method=1, tol=1e-8, maxit=100, adaptive=True, k=3, s=1, rho_max=0.99)
    assert r1.iters == r2.iters and r2.reintroductions == 0
    assert x1.tobytes() == x2.tobytes()


def test_failure_statuses(oracle_mod):
    A = I.poisson2d(16)
    h = oracle_mod.OracleAMG(A)
    b = I.rhs(A.n, 1)
    x, res = h.solve(b, method=1, tol=1e-14, maxit=1)
    assert res.status == -5 and res.iters == 1 and not res.converged
    bad = b.copy(); bad[3] = np.nan
    x, res = h.solve(bad, method=1, tol=1e-8, maxit=10)
    assert res.status == -6
    x, res = h.solve(np.zeros(A.n), method=1, tol=1e-8, maxit=10)
    assert res.status == 0 and res.iters == 0


def test_adaptive_diverged_window_reverts(oracle_mod):
    """Stationary AMG on the random graph Laplacian with gamma = 1 on every
    coarse level diverges; the first window (k = 3) therefore reintroduces
    entries and restarts from the window-start iterate (Section 6: the most
    recent x is kept unless the iterations diverged).  Replayed step by step
    with the non-adaptive solver."""
    A = I.random_graph_laplacian(5000)
    b = I.rhs(A.n, 1)
    start = lambda h: h.sparsify([0.0] + [1.0] * (h.nlev - 1))
    h = oracle_mod.OracleAMG(A)
    start(h)
    x_ad, res = h.solve(b, method=0, tol=1e-14, maxit=5, adaptive=True, k=3, s=1)
    assert res.reintroductions == 1 and res.status == -5
    ref = oracle_mod.OracleAMG(A)
    start(ref)
    x3, r3 = ref.solve(b, method=0, tol=1e-14, maxit=3)
    assert r3.relres > 1.0                       # the first window diverged
    assert ref.reintroduce(s=1)[0] == 0
    x_ref, _ = ref.solve(b, method=0, tol=1e-14, maxit=2)   # from the reverted x = 0
    assert x_ad.tobytes() == x_ref.tobytes()


def test_openmp_timing_build_gives_the_same_bits(oracle_mod):
    """The OpenMP timing build of the oracle (the CPU baseline) returns the
    parity build's results bit for bit: row loops are split between threads
    but every row and every fixed 8,192-entry block of an inner product is
    summed by one thread in index order."""
    A = I.poisson3d(24)           # 13,824 rows: two dot-product blocks
    b = I.rhs(A.n, 2)
    out = []
    for parallel in (False, True):
        h = oracle_mod.OracleAMG(A, parallel=parallel)
        h.sparsify_from(0.1, 2)
        x, res = h.solve(b, method=1, tol=1e-10, maxit=100, adaptive=True, k=3, s=1)
        xs, rs = h.solve(b, method=0, tol=1e-8, maxit=100)
        out.append((x.tobytes(), res.iters, res.hist.tobytes(), xs.tobytes(), rs.iters))
    assert out[0] == out[1]
