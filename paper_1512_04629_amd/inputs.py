"""Seeded synthetic inputs: the model problems and right-hand sides.

This module builds the linear systems the solver is run on; it holds none of
the multigrid method's arithmetic (no strength, coarsening, interpolation,
Galerkin product, sparsification or cycling).  Both the CPU oracle and the
device library are fed the arrays produced here, so each problem is generated
once and handed to both sides unchanged.

Problems (all SPD, homogeneous Dirichlet boundaries eliminated so that the
unknowns are the interior nodes, numbered lexicographically with x fastest):

* ``poisson2d``  – 5-point finite differences, stencil {4, -1}.
* ``poisson3d``  – 7-point finite differences, stencil {6, -1}; at N=100 this is
  the matrix of Table 1 (level 0: 1,000,000 rows, 6,940,000 nonzeros).
* ``aniso2d``    – bilinear (Q1) finite elements for -div(K grad u) with the
  rotated tensor K = Q^T D Q, Q the rotation by theta and D = diag(1, eps)
  (Section 5, rotated anisotropic diffusion); 9-point stencil.
* ``fv3d_lognormal`` – cell-centred finite volumes on N^3 cells with i.i.d.
  lognormal cell coefficients and harmonic-mean face weights (7-point).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): one sequential stream per seed,
state_k = seed + k * 0x9E3779B97F4A7C15 (k = 1, 2, ...), each state passed
through the published finaliser.  A double in [0, 1) is (z >> 11) * 2^-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream for ``seed``."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 output."""
    z = splitmix64(seed, count, start)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, count: int) -> np.ndarray:
    """Doubles in [-1, 1): 2u - 1 with u from :func:`uniform01`."""
    return 2.0 * uniform01(seed, count) - 1.0


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller, one normal per pair of uniforms.

    Uniform pair (u1, u2) = outputs (2i, 2i+1); u1 is mapped to (0, 1] by
    1 - u1 so that the logarithm is finite; the cosine branch is used.
    """
    u = uniform01(seed, 2 * count)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


@dataclass
class CSR:
    """Square CSR matrix: int32 row pointers and sorted columns, float64 values."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _structured(shape: tuple[int, ...], offsets: list[tuple[int, ...]],
                values: list) -> CSR:
    """Assemble a constant-pattern stencil on a lexicographic grid.

    ``offsets`` are per-axis displacements ordered (x, y, z, ...); ``values``
    holds either a scalar per offset or an array of length n giving the value
    in each row.  Neighbours outside the grid are dropped (Dirichlet).  The
    columns of every row come out sorted because the stencil is visited in
    increasing linear displacement.
    """
    d = len(shape)
    n = int(np.prod(shape))
    strides = [1]
    for k in range(1, d):
        strides.append(strides[-1] * shape[k - 1])
    lin = [sum(o[k] * strides[k] for k in range(d)) for o in offsets]
    order = np.argsort(lin, kind="stable")
    coords = np.indices(shape[::-1]).reshape(d, -1)[::-1]  # coords[k] = axis-k index, x fastest
    masks, cols, vals = [], [], []
    for t in order:
        o = offsets[t]
        m = np.ones(n, dtype=bool)
        for k in range(d):
            if o[k] != 0:
                c = coords[k] + o[k]
                m &= (c >= 0) & (c < shape[k])
        masks.append(m)
        cols.append(np.arange(n, dtype=np.int64) + lin[t])
        v = values[t]
        vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
    masks = np.stack(masks)                      # (stencil, n)
    counts = masks.sum(axis=0)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    fill = row_ptr[:-1].copy()
    for s in range(len(order)):
        m = masks[s]
        pos = fill[m]
        col[pos] = cols[s][m]
        val[pos] = vals[s][m]
        fill[m] += 1
    return CSR(n, row_ptr.astype(np.int32), col, val)


def poisson2d(N: int) -> CSR:
    """5-point Laplacian on an N x N interior grid: nnz = N^2 + 4N(N-1)."""
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    return _structured((N, N), offs, [4.0, -1.0, -1.0, -1.0, -1.0])


def poisson3d(N: int) -> CSR:
    """7-point Laplacian on an N^3 interior grid: nnz = N^3 + 6N^2(N-1)."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return _structured((N, N, N), offs, [6.0] + [-1.0] * 6)


def q1_rotated_stencil(eps: float, theta: float) -> dict:
    """Assembled Q1 stencil of -div(K grad u), K = Q^T diag(1, eps) Q.

    With a = K_xx, b = K_yy, c = K_xy the interior stencil of the bilinear
    element (independent of the mesh width in 2D) is: centre 4(a+b)/3,
    east/west (b-2a)/3, north/south (a-2b)/3, NE/SW -(a+b)/6 - c/2,
    NW/SE -(a+b)/6 + c/2.  Keys are (dx, dy).
    """
    cs, sn = math.cos(theta), math.sin(theta)
    a = cs * cs + eps * sn * sn
    b = sn * sn + eps * cs * cs
    c = (1.0 - eps) * cs * sn
    return {
        (0, 0): 4.0 * (a + b) / 3.0,
        (-1, 0): (b - 2.0 * a) / 3.0, (1, 0): (b - 2.0 * a) / 3.0,
        (0, -1): (a - 2.0 * b) / 3.0, (0, 1): (a - 2.0 * b) / 3.0,
        (1, 1): -(a + b) / 6.0 - c / 2.0, (-1, -1): -(a + b) / 6.0 - c / 2.0,
        (-1, 1): -(a + b) / 6.0 + c / 2.0, (1, -1): -(a + b) / 6.0 + c / 2.0,
    }


def aniso2d(N: int, eps: float = 1e-3, theta: float = math.pi / 8) -> CSR:
    """Rotated anisotropic Q1 9-point operator on N x N interior nodes: nnz = (3N-2)^2."""
    st = q1_rotated_stencil(eps, theta)
    offs = list(st.keys())
    return _structured((N, N), offs, [st[o] for o in offs])


def fv3d_lognormal(N: int, seed: int = 40) -> CSR:
    """Cell-centred FV diffusion on N^3 cells, coefficients exp(N(0,1)) i.i.d.

    Interior face weight 2 k_i k_j / (k_i + k_j) (harmonic mean, written so
    that the (i,j) and (j,i) weights are the same double); a boundary face
    contributes 2 k_i to the diagonal (half a cell to the Dirichlet face).
    The diagonal is the sum of the cell's six face weights, in the order
    -x, +x, -y, +y, -z, +z.
    """
    n = N ** 3
    k = np.exp(normal(seed, n)).reshape(N, N, N)  # [z, y, x]
    diag = np.zeros((N, N, N))
    offs = [(0, 0, 0)]
    vals = [None]
    for axis, (dx, dy, dz) in ((2, (1, 0, 0)), (1, (0, 1, 0)), (0, (0, 0, 1))):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, N - 1)
        hi[axis] = slice(1, N)
        kl, kh = k[tuple(lo)], k[tuple(hi)]
        w = 2.0 * kl * kh / (kl + kh)
        wm = np.zeros((N, N, N))       # weight of the face on the minus side
        wp = np.zeros((N, N, N))       # weight of the face on the plus side
        wp[tuple(lo)] = w
        wm[tuple(hi)] = w
        bm = np.zeros((N, N, N), dtype=bool)
        bp = np.zeros((N, N, N), dtype=bool)
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = N - 1
        bm[tuple(first)] = True
        bp[tuple(last)] = True
        fm = np.where(bm, 2.0 * k, wm)
        fp = np.where(bp, 2.0 * k, wp)
        diag = diag + fm
        diag = diag + fp
        offs += [(-dx, -dy, -dz), (dx, dy, dz)]
        vals += [-wm.reshape(-1), -wp.reshape(-1)]
    vals[0] = diag.reshape(-1)
    return _structured((N, N, N), offs, vals)


def random_graph_laplacian(n: int, degree: int = 6, seed: int = 7,
                           shift_every: int = 17) -> CSR:
    """Weighted Laplacian of a random graph plus a sparse diagonal shift.

    Each vertex i draws ``degree`` partners j = floor(u n) and weights
    0.5 + u' (u, u' uniform from SplitMix64 ``seed``); self loops are skipped,
    repeated edges have their weights added.  Every undirected edge weight is
    one double written at (i,j) and (j,i), so the matrix is bitwise symmetric.
    The diagonal is the sum of the incident weights (summed in increasing
    neighbour order) plus 1 on every ``shift_every``-th row, so the matrix is
    a symmetric diagonally dominant M-matrix with strictly dominant rows, hence
    SPD.  Row lengths vary from row to row.
    """
    m = n * degree
    u = uniform01(seed, 2 * m)
    src = np.repeat(np.arange(n, dtype=np.int64), degree)
    dst = np.minimum((u[0::2] * n).astype(np.int64), n - 1)
    w = 0.5 + u[1::2]
    keep = src != dst
    src, dst, w = src[keep], dst[keep], w[keep]
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    key = lo * n + hi
    order = np.argsort(key, kind="stable")
    key, w = key[order], w[order]
    uniq, start = np.unique(key, return_index=True)
    wsum = np.add.reduceat(w, start) if len(w) else w
    lo, hi = uniq // n, uniq % n
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    vals = np.concatenate([-wsum, -wsum])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    # per-row sums of incident weights in increasing neighbour order
    counts = np.bincount(rows, minlength=n)
    rp_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp_off[1:])
    negw = -vals
    diag = np.add.reduceat(negw, rp_off[:-1]) if len(negw) else np.zeros(n)
    diag = np.where(counts > 0, diag, 0.0)
    diag = diag + np.where(np.arange(n) % shift_every == 0, 1.0, 0.0)
    diag = np.where(diag > 0, diag, 1.0)
    # merge the diagonal into the sorted rows
    all_rows = np.concatenate([rows, np.arange(n)])
    all_cols = np.concatenate([cols, np.arange(n)])
    all_vals = np.concatenate([vals, diag])
    order = np.lexsort((all_cols, all_rows))
    all_rows, all_cols, all_vals = all_rows[order], all_cols[order], all_vals[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(all_rows, minlength=n), out=rp[1:])
    return CSR(n, rp.astype(np.int32), all_cols.astype(np.int32), all_vals.astype(np.float64))


def rhs(n: int, seed: int) -> np.ndarray:
    """Right-hand side with entries uniform in [-1, 1)."""
    return uniform_pm1(seed, n)


def make_problem(kind: str, N: int) -> CSR:
    if kind == "poisson2d":
        return poisson2d(N)
    if kind == "poisson3d":
        return poisson3d(N)
    if kind == "aniso2d":
        return aniso2d(N)
    if kind == "fv3d":
        return fv3d_lognormal(N)
    if kind == "graph":
        return random_graph_laplacian(N)
    raise ValueError(f"unknown problem kind {kind!r}")
