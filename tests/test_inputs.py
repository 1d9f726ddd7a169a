"""Pins of the seeded problem generators (shared by the oracle and the library)."""
import math

import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I


def test_splitmix64_published_vectors():
    # First outputs of SplitMix64 seeded with 0, as published with the
    # reference implementation of the generator.
    z = I.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_ranges_and_offsets():
    u = I.uniform01(5, 1000)
    assert u.min() >= 0.0 and u.max() < 1.0
    # the stream is counter based: a window equals the slice of a longer draw
    assert np.array_equal(I.uniform01(5, 10, start=990), u[990:])
    r = I.rhs(1000, 2)
    assert r.min() >= -1.0 and r.max() < 1.0


def test_normal_moments():
    z = I.normal(11, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


@pytest.mark.parametrize("N", [3, 7, 20])
def test_poisson_nnz_closed_forms(N):
    assert I.poisson2d(N).nnz == N * N + 4 * N * (N - 1)
    assert I.poisson3d(N).nnz == N ** 3 + 6 * N * N * (N - 1)
    assert I.aniso2d(N).nnz == (3 * N - 2) ** 2


def test_poisson3d_table1_level0():
    # Table 1, level 0: 1,000,000 rows and 6,940,000 nonzeros at 100^3.
    A = I.poisson3d(100)
    assert (A.n, A.nnz) == (1000000, 6940000)


def _check_csr(A):
    rp, ci = A.row_ptr, A.col
    assert rp[0] == 0 and np.all(np.diff(rp) >= 1)
    for i in range(A.n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i in row
    d = A.to_dense()
    assert np.array_equal(d, d.T)  # bitwise symmetric
    return d


@pytest.mark.parametrize("make", [lambda: I.poisson2d(6), lambda: I.poisson3d(4),
                                  lambda: I.aniso2d(6), lambda: I.fv3d_lognormal(4),
                                  lambda: I.random_graph_laplacian(200)])
def test_generators_spd_sorted_symmetric(make):
    A = make()
    d = _check_csr(A)
    assert np.linalg.eigvalsh(d).min() > 0


def test_interior_row_sums_zero():
    for A, N, dim in ((I.poisson2d(8), 8, 2), (I.poisson3d(6), 6, 3), (I.aniso2d(8), 8, 2)):
        d = A.to_dense()
        idx = np.indices((N,) * dim).reshape(dim, -1)[::-1]
        interior = np.all((idx > 0) & (idx < N - 1), axis=0)
        assert np.max(np.abs(d.sum(1)[interior])) < 1e-14


def _q1_element_stiffness(K):
    """Bilinear element stiffness on the unit square by 2x2 Gauss quadrature."""
    g = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]
    Ke = np.zeros((4, 4))
    for x in g:
        for y in g:
            grads = []
            for (cx, cy) in corners:
                fx = (x if cx else 1 - x)
                fy = (y if cy else 1 - y)
                dfx = 1.0 if cx else -1.0
                dfy = 1.0 if cy else -1.0
                grads.append(np.array([dfx * fy, fx * dfy]))
            for a in range(4):
                for b in range(4):
                    Ke[a, b] += 0.25 * grads[a] @ K @ grads[b]
    return Ke, corners


def test_q1_rotated_stencil_by_element_assembly():
    # Section 5: K = Q^T D Q with Q the rotation by theta, D = diag(1, eps).
    eps, th = 1e-3, math.pi / 8
    Q = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
    K = Q.T @ np.diag([1.0, eps]) @ Q
    Ke, corners = _q1_element_stiffness(K)
    # assemble the stencil of the node at the origin from its four elements
    st = {}
    for ex in (-1, 0):
        for ey in (-1, 0):
            a = corners.index((-ex, -ey))  # local index of the origin in this element
            for b, (cx, cy) in enumerate(corners):
                off = (ex + cx, ey + cy)
                st[off] = st.get(off, 0.0) + Ke[a, b]
    ref = I.q1_rotated_stencil(eps, th)
    for off, v in ref.items():
        assert abs(st[off] - v) < 1e-12, off
    # the values quoted for theta = pi/8, eps = 1e-3
    assert round(ref[(0, 0)], 6) == 1.334667
    assert round(ref[(1, 0)], 6) == -0.520033
    assert round(ref[(0, 1)], 6) == 0.186367
    assert round(ref[(1, 1)], 6) == -0.343433
    assert round(ref[(-1, 1)], 6) == 0.009767


def test_fv_harmonic_weights():
    A = I.fv3d_lognormal(5, seed=40)
    d = A.to_dense()
    k = np.exp(I.normal(40, 125))
    # face between cells 0 and 1 (x neighbours)
    assert d[0, 1] == -(2.0 * k[0] * k[1] / (k[0] + k[1]))
    # corner cell 0: three boundary faces (2k) and three interior faces
    assert abs(d[0, 0] - (3 * 2 * k[0] - d[0, 1] - d[0, 5] - d[0, 25])) < 1e-12 * d[0, 0]
    assert np.all(d.sum(1) > -1e-12)
