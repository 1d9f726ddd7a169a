"""Continuous batching (amg_batch) and the solve server, through the C ABI.

Bars:
  * a request's solution is bitwise the same served in a mix (slots refilled
    while others iterate, several problems overlapping on their streams) as
    solved alone: the 16-column block PCG with that right-hand side in one
    column and zeros elsewhere, same precision;
  * against the oracle's PCG of the same right-hand side: FP64 equal
    iteration counts, FP32 cycle at most 3 more; true residual <= 1.01e-10
    ||b|| and ||A (x - x_or)|| <= 2.02e-10 ||b||;
  * admission: with a budget that holds one engine at a time every request
    still completes and no more than one engine is ever live.
"""
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
    amg.load_library()
    return amg


PROBLEMS = {
    "p2d_48": lambda: I.poisson2d(48),
    "aniso_40": lambda: I.aniso2d(40),
    "p3d_14": lambda: I.poisson3d(14),
}


def make_requests(problems, count, seed, rate=None):
    from paper_1512_04629_amd.serve import Request
    keys = sorted(problems)
    pick = I.splitmix64(seed, count) % np.uint64(len(keys))
    gaps = -np.log(1.0 - I.uniform01(seed + 1, count)) / rate if rate else np.zeros(count)
    t = np.cumsum(gaps)
    reqs = []
    for i in range(count):
        key = keys[int(pick[i])]
        n = problems[key].n
        b = torch.as_tensor(I.rhs(n, 1000 + i)).cuda()
        reqs.append(Request(i, key, b, float(t[i]) if rate else 0.0,
                            x=torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    return reqs


def alone(h, b, precision, slots=16):
    """The request solved alone: block PCG, the right-hand side in column 0."""
    n = h.n
    B = torch.zeros(n, slots, dtype=torch.float64, device="cuda")
    B[:, 0] = b
    X = torch.zeros_like(B)
    res = h.solve_block(B, X, method=1, tol=1e-10, maxit=300, precision=precision)
    return X[:, 0].clone(), int(res.col_iters[0])


@pytest.mark.parametrize("precision", [32, 64])
def test_served_results_equal_alone_and_oracle(lib, precision):
    from oracle import oracle as O
    from paper_1512_04629_amd.serve import SolveServer
    import scipy.sparse as S
    probs = {k: f() for k, f in PROBLEMS.items()}
    srv = SolveServer(probs, hbm_budget=64 << 30, slots=16, precision=precision, tol=1e-10, maxit=300)
    reqs = make_requests(probs, 60, seed=5, rate=3000.0)
    st = srv.run(reqs)
    assert all(r.status == 0 for r in reqs), [r.status for r in reqs]
    assert st.steps > 0 and st.max_live_engines <= len(probs)
    srv.close_engines()
    oracles = {}
    for r in reqs[::7]:
        h = srv.hier[r.key]
        xa, ia = alone(h, r.b, precision)
        assert r.iters == ia
        assert r.x.cpu().numpy().tobytes() == xa.cpu().numpy().tobytes(), r.rid
        A = probs[r.key]
        if r.key not in oracles:
            o = O.OracleAMG(A)
            o.sparsify([0.0, 0.0] + [0.01] * (o.nlev - 2))
            oracles[r.key] = o
        b = r.b.cpu().numpy()
        xo, ro = oracles[r.key].solve(b, method=O.PCG, tol=1e-10, maxit=300)
        Sp = S.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
        x = r.x.cpu().numpy()
        nb = np.linalg.norm(b)
        assert np.linalg.norm(b - Sp @ x) <= 1.01e-10 * nb
        assert np.linalg.norm(Sp @ (x - xo)) <= 2.02e-10 * nb
        if precision == 64:
            assert r.iters == ro.iters, (r.iters, ro.iters)
        else:
            assert ro.iters <= r.iters <= ro.iters + 3, (r.iters, ro.iters)
    srv.close()


def test_admission_with_a_one_engine_budget(lib):
    from paper_1512_04629_amd.serve import Request, SolveServer
    probs = {k: f() for k, f in PROBLEMS.items()}
    srv = SolveServer(probs, hbm_budget=64 << 30, slots=8, precision=32)
    # one request per problem, so that every engine (and the FP32 copies of
    # every hierarchy, which then stay resident) has been made once
    warm = [Request(i, k, torch.as_tensor(I.rhs(probs[k].n, 50 + i)).cuda(), 0.0,
                    x=torch.zeros(probs[k].n, dtype=torch.float64, device="cuda"))
            for i, k in enumerate(sorted(probs))]
    srv.run(warm)
    srv.close_engines()
    resident = srv.device_bytes()
    sizes = sorted(h.batch_bytes(8, 32) for h in srv.hier.values())
    assert sizes[0] + sizes[1] > sizes[-1]          # the budget below holds one engine at a time
    srv.budget = resident + sizes[-1]
    reqs = make_requests(probs, 30, seed=9)
    st = srv.run(reqs)
    assert all(r.status == 0 for r in reqs)
    assert st.max_live_engines == 1 and st.engines_evicted >= 2
    assert st.peak_bytes <= srv.budget
    srv.close()


def test_batch_api_contract(lib):
    from paper_1512_04629_amd import amg
    A = I.poisson2d(32)
    h = amg.Hierarchy(A)
    h.sparsify(0.01, 2)
    eng = h.batch(slots=4, precision=32, tol=1e-10, maxit=100)
    with pytest.raises(amg.AmgError):
        h.solve(torch.zeros(A.n, dtype=torch.float64, device="cuda"),
                torch.zeros(A.n, dtype=torch.float64, device="cuda"))
    with pytest.raises(amg.AmgError):
        h.batch(slots=4)
    bs = [torch.as_tensor(I.rhs(A.n, 30 + i)).cuda() for i in range(5)]
    bs[2].zero_()
    slots = [eng.submit(b) for b in bs[:4]]
    assert sorted(slots) == [0, 1, 2, 3]
    with pytest.raises(amg.AmgError):
        eng.submit(bs[4])                      # all slots taken
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(amg.AmgError):
        eng.collect(0, x)                      # not finished
    assert eng.step()
    with pytest.raises(amg.AmgError):
        eng.step()                             # previous step not completed
    fin = eng.poll(wait=True)
    assert fin == [slots[2]]                   # the zero right-hand side: x = 0 at once
    it, rr, stt = eng.collect(slots[2], x)
    assert (it, rr, stt) == (0, 0.0, 0) and torch.count_nonzero(x).item() == 0
    s4 = eng.submit(bs[4])                     # refilled while the others iterate
    assert s4 == slots[2]
    done = {}
    for _ in range(200):
        if not eng.step():
            break
        for c in eng.poll(wait=True):
            xc = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            done[c] = (eng.collect(c, xc), xc)
    assert sorted(done) == [0, 1, 2, 3]
    assert all(v[0][2] == 0 and v[0][1] <= 1e-10 for v in done.values())
    assert list(eng.states()) == [0, 0, 0, 0]
    assert eng.poll(wait=False) == []
    # maxit reached: status NOT_CONVERGED, slot still collectable
    eng.close()
    eng = h.batch(slots=4, precision=64, tol=1e-14, maxit=2)
    eng.submit(bs[0])
    eng.step(); eng.poll(True)
    eng.step(); fin = eng.poll(True)
    assert fin == [0]
    it, rr, stt = eng.collect(0, x)
    assert it == 2 and stt == -5 and rr > 1e-14
    eng.close()
    # the handle works normally again once the engine is gone
    res = h.solve(bs[0], x.zero_(), tol=1e-10)
    assert res.converged
    h.close()


def test_batch_bytes_match_allocations(lib):
    from paper_1512_04629_amd import amg
    A = I.aniso2d(64)
    h = amg.Hierarchy(A)
    h.sparsify(0.1, 2)
    for prec in (32, 64):
        before = h.device_bytes()
        predicted = h.batch_bytes(16, prec)
        eng = h.batch(slots=16, precision=prec)
        assert h.device_bytes() - before == predicted
        eng.close()
        if prec == 32:
            # the FP32 copies stay with the hierarchy
            assert h.batch_bytes(16, 32) < predicted
    h.close()


@pytest.mark.parametrize("precision", [32, 64])
def test_graph_replays_and_multi_iteration_steps_equal_eager(lib, precision):
    """The same submissions served with captured iterations and several
    iterations per step give the bits of eager single-iteration steps."""
    from paper_1512_04629_amd import amg
    A = I.aniso2d(48)
    stream = torch.cuda.Stream()          # captured graphs need a stream other than the null stream
    with torch.cuda.stream(stream):
        h = amg.Hierarchy(A)
    torch.cuda.synchronize()
    bs = [torch.as_tensor(I.rhs(A.n, 70 + i)).cuda() for i in range(10)]
    torch.cuda.synchronize()

    def serve(graphs, iters):
        with torch.cuda.stream(stream):
            eng = h.batch(slots=4, precision=precision, tol=1e-10, maxit=200, graphs=graphs)
        out, queue, owner = {}, list(range(len(bs))), {}
        while len(out) < len(bs):
            while queue and (eng.states() == 0).any():
                i = queue.pop(0)
                owner[eng.submit(bs[i])] = i
            assert eng.step(iters)
            torch.cuda.synchronize()               # eager work between replays
            for c in eng.poll(wait=True):
                x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                it, rr, st = eng.collect(c, x)
                assert st == 0
                out[owner.pop(c)] = (it, x)
        eng.close()
        torch.cuda.synchronize()
        return out

    ref = serve(False, 1)
    for graphs, iters in ((True, 1), (True, 3), (False, 4), (True, 7)):
        got = serve(graphs, iters)
        for i in range(len(bs)):
            assert got[i][0] == ref[i][0]
            assert got[i][1].cpu().numpy().tobytes() == ref[i][1].cpu().numpy().tobytes(), (graphs, iters, i)
    h.close()
