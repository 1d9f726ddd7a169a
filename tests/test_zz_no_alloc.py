"""amg_solve_noalloc, the solve for callers that cannot allocate device
memory, against amg_solve through the C ABI.

The handles are built with an allocator callback that counts its calls, so
the test sees every device allocation the library asks for.  On each case a
fresh sparsification is solved first with amg_solve_noalloc (on a handle that
has never solved, so none of amg_solve's work vectors exist yet) and then,
after the same sparsification, with amg_solve: the allocation-free call asks
for no memory, and the two give the same status, counts, residual history and
solution bit for bit.  The cases run in a row on the one static work array,
each smaller than the one before.  Sizes beyond the array, the FP32 cycle and
kernel profiling are rejected before any device work.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1512_04629_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_04629_amd import amg
    return amg.load_library()


class CountingAllocator:
    def __init__(self):
        from paper_1512_04629_amd import amg
        self.allocs = 0
        self.live = {}

        def alloc(nbytes, stream, user):
            self.allocs += 1
            p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            self.live[p] = nbytes
            return p

        def free(ptr, nbytes, stream, user):
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = amg.ALLOC_FN(alloc)
        self.free_fn = amg.FREE_FN(free)


def make_handle(lib, A, counter):
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    ci = np.ascontiguousarray(A.col, np.int32)
    v = np.ascontiguousarray(A.val, np.float64)
    h = C.c_void_p()
    st = lib.amg_setup_from_csr(A.n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, None,
                                C.c_void_p(torch.cuda.current_stream().cuda_stream), counter.alloc_fn,
                                counter.free_fn, None, C.byref(h))
    assert st == 0, lib.amg_last_error(None)
    return h


def params(method, tol, maxit, adaptive, precision=64):
    from paper_1512_04629_amd import amg
    return amg.SolveParams(method, tol, maxit, int(adaptive), 3, 1, 0.5, 0.01, precision)


def run(lib, fn, h, b, p):
    from paper_1512_04629_amd import amg
    x = torch.zeros(b.numel(), dtype=torch.float64, device="cuda")
    info = amg.SolveInfo()
    hist = np.full(p.maxit + 1, np.nan)
    st = fn(h, b.data_ptr(), x.data_ptr(), C.byref(p), C.byref(info), hist.ctypes.data)
    torch.cuda.synchronize()
    return st, info, hist[: info.iters + 1].copy(), x.cpu().numpy()


CASES = [
    # (problem, gamma on levels >= 2, method, tol, adaptive); n decreasing
    ("poisson3d_64", lambda: I.poisson3d(64), 0.1, 1, 1e-8, True),
    ("aniso2d_160", lambda: I.aniso2d(160), 0.1, 1, 1e-8, True),
    ("poisson2d_64", lambda: I.poisson2d(64), 0.01, 0, 1e-8, False),
]


def test_noalloc_solve_equals_solve_in_a_row(lib):
    counter = CountingAllocator()
    sizes = []
    for name, make, gamma, method, tol, adaptive in CASES:
        A = make()
        sizes.append(A.n)
        print(f"no-alloc case {name}: n={A.n} gamma={gamma} method={method} adaptive={adaptive}", flush=True)
        h = make_handle(lib, A, counter)
        try:
            b = torch.as_tensor(I.rhs(A.n, 2)).cuda()
            p = params(method, tol, 300, adaptive)
            assert lib.amg_sparsify(h, gamma, 2) == 0
            torch.cuda.synchronize()
            before = counter.allocs
            st0, info0, hist0, x0 = run(lib, lib.amg_solve_noalloc, h, b, p)
            assert counter.allocs == before, (name, counter.allocs - before)
            assert lib.amg_sparsify(h, gamma, 2) == 0
            st1, info1, hist1, x1 = run(lib, lib.amg_solve, h, b, p)
            assert counter.allocs > before       # amg_solve allocates its work vectors
            print(f"  status {st0}/{st1} iterations {info0.iters}/{info1.iters} "
                  f"reintroductions {info0.reintroductions}/{info1.reintroductions}", flush=True)
            assert st0 == st1 == 0
            assert (info0.iters, info0.restarts, info0.reintroductions, info0.converged) == \
                   (info1.iters, info1.restarts, info1.reintroductions, info1.converged)
            assert info0.relres == info1.relres and info0.relres <= tol
            assert hist0.tobytes() == hist1.tobytes()
            assert x0.tobytes() == x1.tobytes()
        finally:
            lib.amg_destroy(h)
    assert sizes == sorted(sizes, reverse=True)


def test_noalloc_rejections(lib):
    from paper_1512_04629_amd import amg
    counter = CountingAllocator()
    A = I.poisson2d(32)
    h = make_handle(lib, A, counter)
    try:
        b = torch.as_tensor(I.rhs(A.n, 1)).cuda()
        st, _, _, _ = run(lib, lib.amg_solve_noalloc, h, b, params(1, 1e-8, 50, False, precision=32))
        assert st == -1 and b"FP64" in lib.amg_last_error(h)
        assert lib.amg_profile_enable(h, 1, -1, -1) == 0
        st, _, _, _ = run(lib, lib.amg_solve_noalloc, h, b, params(1, 1e-8, 50, False))
        assert st == -7
        assert lib.amg_profile_enable(h, 0, -1, -1) == 0
        st, info, _, _ = run(lib, lib.amg_solve_noalloc, h, b, params(1, 1e-8, 50, False))
        assert st == 0 and info.converged
    finally:
        lib.amg_destroy(h)
    A = I.poisson3d(129)                      # 2,146,689 rows > 2,097,152
    h = make_handle(lib, A, counter)
    try:
        b = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        st, _, _, _ = run(lib, lib.amg_solve_noalloc, h, b, params(1, 1e-8, 5, False))
        assert st == -1 and b"2097152" in lib.amg_last_error(h)
    finally:
        lib.amg_destroy(h)
    assert amg.ABI_SYMBOLS.count("amg_solve_noalloc") == 1
