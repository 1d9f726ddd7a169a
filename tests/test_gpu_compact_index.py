"""Compressed column indices of the fixed operators (amg_set_compact_indices:
16-bit offsets, and for the SELL-64 copies of stencil-like operators 8-bit
positions in a table of offsets per slice): a storage form of the same
matrices, so every result is bitwise the one the 32-bit indices give.  Bars: V-cycles (FP64, FP32) and PCG solves bit for bit
equal with the indices on and off; the form is used where the spans fit
(banded 3D Poisson) and refused where they do not (a random graph).  The
LDS-staged kernels alternate the order of their row blocks from pass to
pass: results bitwise independent of it."""
import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

from .test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    amg.load_library()
    return amg


def _stream_levels(h):
    """levels whose fixed operator A_l is read with compressed column indices"""
    return [l for l in range(h.nlev) if h.index_width(l, "A") < 4]


def test_compact_indices_bitwise_equal_results(lib):
    A = I.poisson3d(64)          # levels 0 and 1 run on the LDS-staged kernels
    b = dev(I.rhs(A.n, 4))
    h = lib.Hierarchy(A)
    assert 0 in _stream_levels(h) and 1 in _stream_levels(h)
    # A_0 (7 offsets per slice) in the 8-bit offset-table form, R_0 in 16 bits
    assert h.index_width(0, "R") == 2 and h.index_width(0, "AHAT") == 1 and h.index_width(1, "A") == 1
    h.sparsify(0.1, 2)
    out = {}
    for on in (True, False):
        h.set_compact_indices(on)
        assert (h.index_width(0, "A") < 4) == on
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        h.vcycle(b, x)
        x32 = torch.zeros(A.n, dtype=torch.float32, device="cuda")
        h.vcycle32(b.float(), x32)
        xs = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        r = h.solve(b, xs, method=1, tol=1e-10, maxit=100)
        xm = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        rm = h.solve(b, xm, method=1, tol=1e-10, maxit=100, precision=32)
        out[on] = (host(x), host(x32), host(xs), r.iters, host(xm), rm.iters)
    a, c = out[True], out[False]
    for u, v in zip(a, c):
        if isinstance(u, np.ndarray):
            assert u.tobytes() == v.tobytes()
        else:
            assert u == v


def test_wide_spans_keep_32bit_indices(lib):
    A = I.random_graph_laplacian(300000, degree=6)
    h = lib.Hierarchy(A)
    assert h.index_width(0, "A") == 4
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(I.rhs(A.n, 1)), x)
    assert torch.isfinite(x).all()


def test_toggle_refused_while_a_batch_exists(lib):
    A = I.poisson3d(20)
    with torch.cuda.stream(torch.cuda.Stream()):
        h = lib.Hierarchy(A)
        eng = h.batch(4, 64)
        with pytest.raises(lib.AmgError):
            h.set_compact_indices(False)
        eng.close()
        h.set_compact_indices(False)
        h.close()


def test_stream_direction_does_not_change_results(lib):
    """Consecutive passes over one operator visit its row blocks in opposite
    orders (for the Infinity Cache); every row's result is the same either
    way, so two consecutive launches of a level operation give the same bits,
    with 16-bit and with 32-bit indices, on the LDS-staged levels."""
    A = I.poisson3d(64)
    h = lib.Hierarchy(A)
    h.sparsify(0.1, 2)
    levels = _stream_levels(h)
    assert levels
    gen = torch.Generator(device="cuda").manual_seed(11)
    for on in (True, False):
        h.set_compact_indices(on)
        for l in levels:
            n = h.level_info(l)["n"]
            b = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
            x = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
            for op in ("JACOBI", "RESIDUAL", "SPMV_A", "SPMV_AHAT"):
                outs = []
                for _ in range(3):
                    y = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
                    h.level_op(l, op, inp=b, x=x, out=y)
                    outs.append(host(y))
                assert outs[0].tobytes() == outs[1].tobytes() == outs[2].tobytes(), (on, l, op)
            if l + 1 < h.nlev:
                nc = h.level_info(l + 1)["n"]
                xc = torch.rand(nc, dtype=torch.float64, device="cuda", generator=gen)
                for op, inp, xx, m in (("RESTRICT", x, None, nc), ("INTERPOLATE", xc, x, n)):
                    outs = []
                    for _ in range(2):
                        y = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
                        h.level_op(l, op, inp=inp, x=xx, out=y)
                        outs.append(host(y))
                    assert outs[0].tobytes() == outs[1].tobytes(), (on, l, op)


def test_repeated_solves_give_the_same_bits(lib):
    """Every pass over an operator flips its direction, also through the
    copies that alias it and in the launches that form dot products (their
    per-block partials go to the block's own index): the same PCG solve run
    three times in a row on one handle, each starting with the passes in the
    other directions, gives the same iterate, residual history and dots."""
    A = I.poisson3d(64)
    b = dev(I.rhs(A.n, 4))
    h = lib.Hierarchy(A)
    assert h.row_format(0, "A") == "sell"
    h.sparsify(0.1, 2)
    outs = []
    for _ in range(3):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        r = h.solve(b, x, method=1, tol=1e-10, maxit=100, adaptive=True, k=3, s=1)
        outs.append((host(x).tobytes(), r.iters, r.hist.tobytes(), r.relres))
    assert outs[0] == outs[1] == outs[2]
