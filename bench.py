"""Benchmark: sparsified AMG-PCG on the 3D Poisson problem, one MI355X.

One step = the whole hot path on resident inputs: Sparse Galerkin
sparsification of every coarse level (keep set + diagonal lumping, from the
retained Galerkin operators) followed by an adaptive AMG-preconditioned CG
solve to a 1e-8 relative residual (with reintroduction when the windowed
convergence factor exceeds 0.5).  The Galerkin setup is a host-side
prerequisite done once before timing (reported as setup_s).

    python bench.py [--steps K] [--warmup W] [--gamma G] [--no-cpu-baseline]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1512_04629_amd", "csrc", "kernels.hip")
BLOCK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters_fv3d.json")
BLOCK_KERNEL_SRC = os.path.join(ROOT, "paper_1512_04629_amd", "csrc", "block_kernels.hip")
LUMP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters_lump.json")
LUMP_KERNEL_SRC = os.path.join(ROOT, "paper_1512_04629_amd", "csrc", "lump_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def launch_bytes(h, kernel: str, level: int) -> int:
    """Algorithmic HBM bytes of one launch: what the method must move, FP64
    values and int32 column indices and row pointers, each array entry counted
    once (a gathered vector is counted as n entries).  This is the figure the
    roofline fraction uses, whatever storage the kernel reads (a SELL-64 copy
    with padding, 16-bit column offsets): the HBM counters report that."""
    li = h.level_info(level)
    n, nnz_hat, nc, nnz_p = li["n"], li["nnz_hat"], li["n_coarse"], li["nnz_P"]
    nnz_a = li["nnz"]
    e = 12  # an FP64 value and an int32 column index per entry

    if kernel == "JACOBI":
        # x gathered, b, dinv read, x' written
        return e * nnz_hat + 4 * (n + 1) + 32 * n
    if kernel == "JACOBI_ZERO":
        # zero-guess level: residual of the prescaled sweep omega D^-1 b that
        # the producer (restriction / CG update) wrote: x gathered, b read, r
        # written (the fused first-iteration form moves 8n more; counted as
        # this lower figure)
        return e * nnz_hat + 4 * (n + 1) + 24 * n
    if kernel == "RESIDUAL":
        # level 0 is the Galerkin A_0 (never sparsified), below it Ahat_l
        nz = nnz_a if level == 0 else nnz_hat
        return e * nz + 4 * (n + 1) + 24 * n
    if kernel == "SPMV_DOT":
        return e * nnz_a + 4 * (n + 1) + 16 * n
    if kernel == "RESTRICT":
        # b_c = R r; below the coarsest level also x_c = omega dinv_c b_c
        extra = 16 * nc if level + 2 < h.nlev else 0
        return e * nnz_p + 4 * (nc + 1) + 8 * n + 8 * nc + extra
    if kernel == "INTERP":
        return e * nnz_p + 4 * (n + 1) + 8 * nc + 16 * n
    return 0


def launch_bytes32(h, kernel: str, level: int) -> int:
    """launch_bytes for the FP32 cycle: 4-byte values and vectors, int32 column
    indices and row pointers (whatever index width the kernel reads)."""
    li = h.level_info(level)
    n, nnz_hat, nc, nnz_p = li["n"], li["nnz_hat"], li["n_coarse"], li["nnz_P"]
    e = 8  # an FP32 value and an int32 column index per entry

    if kernel == "JACOBI":
        return e * nnz_hat + 4 * (n + 1) + 16 * n
    if kernel in ("JACOBI_ZERO", "RESIDUAL"):
        return e * nnz_hat + 4 * (n + 1) + 12 * n
    if kernel == "RESTRICT":
        extra = 8 * nc if level + 2 < h.nlev else 0
        return e * nnz_p + 4 * (nc + 1) + 4 * n + 4 * nc + extra
    if kernel == "INTERP":
        return e * nnz_p + 4 * (n + 1) + 4 * nc + 8 * n
    return 0


def kernel_source_sha(src: str = KERNEL_SRC) -> str:
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_for(kernel: str, level: int, path: str = TRAFFIC_FILE, src: str = KERNEL_SRC, N: int | None = None):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if
    there are none for this kernel (on the 3D Poisson N^3 hierarchy, if N is
    given) or the kernel source changed since."""
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_sha") != kernel_source_sha(src):
        return None
    key = f"{kernel}@{level}" if N is None else f"N{N}:{kernel}@{level}"
    ent = data.get("kernels", {}).get(key)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=128, help="grid side of the 3D Poisson problem")
    ap.add_argument("--gamma", type=float, default=0.1, help="drop tolerance on levels >= 2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--seeds", type=int, default=8, help="right-hand sides of the gamma comparison")
    ap.add_argument("--reps", type=int, default=5, help="timed solves per right-hand side in the gamma comparison")
    ap.add_argument("--hbm-steps", type=int, default=10, help="timed steps of the 192^3 HBM-only figure")
    ap.add_argument("--no-hbm-only", action="store_true", help="skip the 192^3 HBM-only figure")
    ap.add_argument("--no-alone", action="store_true",
                    help="skip the dominant kernel's launches outside the cycle (profiler runs of the cycle alone)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the per-gamma time-to-solution comparison (short profiler runs)")
    ap.add_argument("--budget-gb", type=float, default=32.0,
                    help="serve: HBM budget for resident hierarchies plus batch engines (GiB)")
    ap.add_argument("--requests", type=int, default=512, help="serve: number of requests")
    ap.add_argument("--workload", default="poisson3d", choices=("poisson3d", "aniso2d", "fv3d", "serve", "setup", "lumping", "methods"),
                    help="poisson3d: the headline 3D Poisson FP64 AMG-PCG run; aniso2d: rotated "
                         "anisotropic Q1 1024^2, FP32-preconditioned vs FP64 PCG to 1e-10; fv3d: "
                         "lognormal-coefficient FV 192^3 with 16 right-hand sides per launch, FP32 "
                         "correction cycle in FP64 iterative refinement to 1e-10; serve: 512 requests "
                         "over 14 resident hierarchies, continuous batching, FP32-preconditioned vs "
                         "FP64 PCG to 1e-10; setup: device-resident hierarchy setup (PMIS) of the "
                         "3D Poisson problem, vs the host and RS setups; lumping: sparsification of "
                         "the 3D Poisson hierarchy with strong-neighbour lumping, vs diagonal lumping; "
                         "methods: Galerkin, Sparse Galerkin, Hybrid Galerkin and non-Galerkin "
                         "hierarchies compared on 3D Poisson and rotated anisotropic diffusion")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "aniso2d":
        return bench_aniso(args)
    if args.workload == "fv3d":
        return bench_fv3d(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "setup":
        return bench_setup(args)
    if args.workload == "lumping":
        return bench_lumping(args)
    if args.workload == "methods":
        return bench_methods(args)
    return bench_poisson(args)


def crossing_margin(hist, tol: float) -> float:
    """Smallest |log(rho_k / tol)| over the stop tests a solve took (rho_k its
    relative residual after iteration k): how far its iteration count is from
    flipping under a rounding-level change of the residuals."""
    import numpy as np
    h = np.asarray(hist, float)
    rel = h[1:] / h[0]
    rel = rel[np.isfinite(rel) & (rel > 0)]
    return float(np.min(np.abs(np.log(rel / tol)))) if rel.size else float("inf")


def host_description() -> dict:
    """The host the CPU baseline ran on: nproc, the cores this process may use,
    and lscpu's model, sockets, cores and threads."""
    import subprocess
    d = {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
         "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                             "CPU max MHz"):
                d["lscpu " + k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        d["lscpu"] = "unavailable"
    return d


def omp_threads() -> int:
    v = os.environ.get("OMP_NUM_THREADS")
    try:
        return max(1, int(v.split(",")[0])) if v else len(os.sched_getaffinity(0))
    except ValueError:
        return len(os.sched_getaffinity(0))


def dominant_kernel(h, step):
    """(kernel class, level) with the most HIP-event time over one step."""
    h.profile_enable(True)
    step()
    best = None
    for kern in ("JACOBI", "JACOBI_ZERO", "RESIDUAL", "RESTRICT", "INTERP", "SPMV_DOT"):
        for l in range(h.nlev):
            cnt, ms = h.profile_read(kern, l)
            if cnt and (best is None or ms > best[2]):
                best = (kern, l, ms, cnt)
    h.profile_enable(False)
    return best[0], best[1]


def timed_steps(h, step, steps, warmup, kern, level):
    """Times `steps` steps after `warmup` untimed ones; the launches of one
    kernel class on one level are bracketed by HIP events on the handle's
    stream.  (ms per step, last result, launches, ms in those launches)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    h.profile_enable(True, kern, level)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cnt, ms_total = h.profile_read(kern, level)
    h.profile_enable(False)
    return elapsed / steps * 1e3, res, cnt, ms_total


def bench_poisson(args):
    """The headline workload: 3D Poisson 7-point N^3, Sparse Galerkin
    sparsification at gamma on levels >= 2 + adaptive AMG-PCG to 1e-8."""
    import numpy as np
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    N = args.N
    A = I.poisson3d(N)
    b_host = I.rhs(A.n, 2)
    b = torch.as_tensor(b_host).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    # every solve starts from x0 = 0 (the library zeroes x and takes r0 = b)
    solve_kw = dict(method=amg.PCG, tol=1e-8, maxit=200, adaptive=True, k=3, s=1, rho_max=0.5,
                    gamma_min=0.01, zero_guess=True)
    log(f"[bench] setup 3D Poisson {N}^3 (n={A.n}, nnz={A.nnz})")
    t0 = time.perf_counter()
    h = amg.Hierarchy(A)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup done in {setup_s:.2f} s, {h.nlev} levels")

    def step(gamma=args.gamma, rhs=b):
        h.sparsify(gamma, 2)
        return h.solve(rhs, x, **solve_kw)

    # sparsified vs Galerkin: time-to-1e-8 per gamma over several right-hand
    # sides, with the crossing margin of every solve's iteration count
    compare = {}
    seeds = list(range(2, 2 + args.seeds))
    rhs = {sd: torch.as_tensor(I.rhs(A.n, sd)).cuda() for sd in seeds}
    for gamma in (() if args.no_compare else (0.0, 0.01, 0.1, 1.0)):
        h.sparsify(gamma, 2)
        bpc = h.bytes_per_cycle()
        nnz_levels = [h.level_info(l)["nnz_hat"] for l in range(h.nlev)]
        per_seed = []
        for sd in seeds:
            res = step(gamma, rhs[sd])
            torch.cuda.synchronize()
            times = []
            for _ in range(args.reps):
                t0 = time.perf_counter()
                res = step(gamma, rhs[sd])
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
            ms = float(np.median(times))
            per_seed.append(dict(seed=sd, ms=round(ms, 3), iters=res.iters, reintroductions=res.reintroductions,
                                 relres=res.relres, converged=res.converged,
                                 margin=round(crossing_margin(res.hist, solve_kw["tol"]), 5),
                                 ms_per_iter=round(ms / max(res.iters, 1), 4)))
        med = lambda k: float(np.median([r[k] for r in per_seed]))  # noqa: E731
        compare[str(gamma)] = dict(
            ms_to_1e8=round(med("ms"), 3), ms_min=round(min(r["ms"] for r in per_seed), 3),
            iters=med("iters"), ms_per_iter=round(med("ms_per_iter"), 4), reps=args.reps,
            min_margin=min(r["margin"] for r in per_seed), converged=all(r["converged"] for r in per_seed),
            nnz_per_level=nnz_levels, bytes_per_vcycle=bpc, per_seed=per_seed)
        log(f"[bench] gamma={gamma}: median {med('ms'):.2f} ms, {med('iters'):.0f} iters, "
            f"{med('ms_per_iter'):.3f} ms/iter, {bpc / 1e6:.0f} MB/cycle, "
            f"min margin {compare[str(gamma)]['min_margin']:.3g}")
    summary = None
    g0, gg = compare.get("0.0"), compare.get(str(args.gamma))
    if g0 and gg:
        wins = sum(1 for a, c in zip(g0["per_seed"], gg["per_seed"]) if c["ms"] < a["ms"])
        fewer = sum(1 for a, c in zip(g0["per_seed"], gg["per_seed"]) if c["iters"] < a["iters"])
        more = sum(1 for a, c in zip(g0["per_seed"], gg["per_seed"]) if c["iters"] > a["iters"])
        summary = dict(
            gamma=args.gamma, seeds=len(seeds),
            speedup_median=round(g0["ms_to_1e8"] / gg["ms_to_1e8"], 4),
            per_iteration_speedup=round(g0["ms_per_iter"] / gg["ms_per_iter"], 4),
            iteration_ratio=round(g0["iters"] / gg["iters"], 4),
            bytes_per_cycle_ratio=round(gg["bytes_per_vcycle"] / g0["bytes_per_vcycle"], 4),
            seeds_faster=wins, seeds_fewer_iterations=fewer, seeds_more_iterations=more)
        log(f"[bench] gamma={args.gamma} vs Galerkin: {summary}")

    # timed region: K steps (right-hand side seed 2), the dominant kernel's
    # launches bracketed by HIP events
    dom_kernel, dom_level = dominant_kernel(h, step)
    log(f"[bench] dominant kernel {dom_kernel} on level {dom_level}")
    ms_per_step, res, cnt, ms_total = timed_steps(h, step, args.steps, args.warmup, dom_kernel, dom_level)
    value = 1e3 / ms_per_step
    per_launch_s = ms_total / max(cnt, 1) / 1e3
    nbytes = launch_bytes(h, dom_kernel, dom_level)
    achieved = nbytes / per_launch_s / 1e9
    traffic = traffic_for(dom_kernel, dom_level, N=N)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step; {dom_kernel}@{dom_level}: "
        f"{per_launch_s * 1e6:.1f} us/launch, {achieved:.0f} GB/s")

    # the step's two phases timed apart with HIP events on the library's stream
    # (torch's current stream): the sparsify pass over every coarse level, and
    # the adaptive solve
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    sp_ms, so_ms = [], []
    for _ in range(max(args.steps // 2, 3)):
        ev[0].record()
        h.sparsify(args.gamma, 2)
        ev[1].record()
        h.solve(b, x, **solve_kw)
        ev[2].record()
        torch.cuda.synchronize()
        sp_ms.append(ev[0].elapsed_time(ev[1]))
        so_ms.append(ev[1].elapsed_time(ev[2]))
    phases = dict(sparsify_ms=round(float(np.median(sp_ms)), 4), solve_ms=round(float(np.median(so_ms)), 4),
                  runs=len(sp_ms), how="medians; HIP events around amg_sparsify and around amg_solve from x0 = 0")
    log(f"[bench] phases: sparsify {phases['sparsify_ms']:.3f} ms, solve {phases['solve_ms']:.3f} ms")

    # the dominant kernel alone on its operator, launched through amg_level_op:
    # back to back (the 256 MB Infinity Cache may hold part of the operator),
    # and with 1 GiB streamed between launches so that every launch reads it
    # from HBM.  The zero-guess sweep has no level operation of its own; the
    # sweep with a guess streams the same operator and stands in for it.
    cache_runs = {}
    alone_kernel = {"JACOBI": "JACOBI", "RESIDUAL": "RESIDUAL", "JACOBI_ZERO": "JACOBI"}.get(dom_kernel)
    if alone_kernel and not args.no_alone:
        alone_bytes = launch_bytes(h, alone_kernel, dom_level)
        nl = h.level_info(dom_level)["n"]
        gen = torch.Generator(device="cuda").manual_seed(5)
        bl = torch.rand(nl, dtype=torch.float64, device="cuda", generator=gen)
        xl = torch.rand(nl, dtype=torch.float64, device="cuda", generator=gen)
        ol = torch.empty_like(xl)
        big = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        big2 = torch.empty_like(big)
        cache_runs["kernel"] = f"{alone_kernel} level {dom_level}"
        cache_runs["bytes_per_launch"] = alone_bytes
        cache_runs["how"] = ("back_to_back: 10 launches in a row, the operator partly or wholly read from the "
                             "256 MB Infinity Cache (frac may exceed 1 against the HBM peak); mall_flushed: a "
                             "1 GiB copy before each launch, so the operator comes from HBM")
        for label, flush in (("back_to_back", False), ("mall_flushed", True)):
            h.level_op(dom_level, alone_kernel, inp=bl, x=xl, out=ol)
            torch.cuda.synchronize()
            h.profile_enable(True, alone_kernel, dom_level)
            for _ in range(10):
                if flush:
                    big2.copy_(big)
                h.level_op(dom_level, alone_kernel, inp=bl, x=xl, out=ol)
            torch.cuda.synchronize()
            c3, m3 = h.profile_read(alone_kernel, dom_level)
            h.profile_enable(False)
            gbs = alone_bytes / (m3 / c3 / 1e3) / 1e9
            cache_runs[label] = dict(us_per_launch=round(m3 / c3 * 1e3, 3), achieved=round(gbs, 1),
                                     frac=round(gbs / HBM_PEAK_GBS, 4), launches=c3)
            log(f"[bench] {alone_kernel}@{dom_level} alone, {label}: {m3 / c3 * 1e3:.1f} us, {gbs:.0f} GB/s")
        del big, big2

    # practical ceiling: a plain device-to-device copy of 1 GiB (read + written bytes / time)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9
    # and a read-only pass: a sum over the same 1 GiB (warmed up with the same
    # expression: the first use of the elementwise add stalls the host)
    acc = src.sum()
    acc = acc + src.sum()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        acc = acc + src.sum()
    e1.record()
    torch.cuda.synchronize()
    read_gbs = 10 * src.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    log(f"[bench] device copy of 1 GiB: {copy_gbs:.0f} GB/s (read + write); sum of 1 GiB: {read_gbs:.0f} GB/s")

    # SpMV bandwidth of the fine-level operator (the CG product A p)
    h.profile_enable(True, "SPMV_DOT", 0)
    step()
    c2, m2 = h.profile_read("SPMV_DOT", 0)
    h.profile_enable(False)
    spmv_gbs = launch_bytes(h, "SPMV_DOT", 0) / (m2 / c2 / 1e3) / 1e9 if c2 else None
    nlev = h.nlev
    h.close()
    del x, b, rhs

    # the same step on 3D Poisson 192^3, whose fine operators (A_0 592 MB,
    # A_1 926 MB of algorithmic bytes) are several times the 256 MB Infinity
    # Cache: its dominant kernel's rate is an HBM-only figure
    hbm_only = None
    if N < 192 and not args.no_hbm_only:
        hbm_only = hbm_only_roofline(args, 192)

    out = {
        "metric": "solves/s to 1e-8 relative residual (Sparse Galerkin sparsify + adaptive AMG-PCG); "
                  "time-to-1e-8 sparsified vs Galerkin; SpMV HBM GB/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Poisson 7-point FD {N}^3 (n={A.n}, nnz={A.nnz}), RHS uniform[-1,1] seed 2; "
                        f"RS theta=0.25, direct interpolation, coarsen to <50 rows; Sparse Galerkin "
                        f"gamma={args.gamma} on levels>=2 with diagonal lumping; V(1,1) Jacobi "
                        f"omega=2/3; adaptive AMG-PCG (k=3, s=1, rho_max=0.5) to 1e-8",
            "levels": nlev,
            "gamma": args.gamma,
        },
        "iters": res.iters,
        "relres": res.relres,
        "setup_s": round(setup_s, 3),
        "phases": phases,
        "time_to_1e8_ms": compare,
        "sparsified_vs_galerkin": summary,
        "speedup_vs_galerkin": summary["speedup_median"] if summary else None,
        "spmv_gbs_level0": round(spmv_gbs, 1) if spmv_gbs else None,
        "practical_ceiling": {"copy_gbs": round(copy_gbs, 1), "read_gbs": round(read_gbs, 1),
                              "how": "1 GiB device-to-device copy, bytes read + written per second; "
                                     "sum over 1 GiB, bytes read per second"},
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom_kernel} level {dom_level}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": nbytes,
            "bytes_rule": "12 nnz + 4 (n+1) + 32 n (Jacobi; 24 n residual): FP64 values, int32 indices",
            "us_per_launch": round(per_launch_s * 1e6, 3),
            "launches": cnt,
            "alone": cache_runs,
            "hbm_only": hbm_only,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, A, b_host)
    print(json.dumps(out), flush=True)


def hbm_only_roofline(args, N2: int) -> dict:
    """The headline step on 3D Poisson N2^3: its dominant kernel timed with
    HIP events over `steps` timed steps, against the algorithmic bytes."""
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    A = I.poisson3d(N2)
    log(f"[bench] HBM-only figure: setup 3D Poisson {N2}^3 (n={A.n}, nnz={A.nnz})")
    h = amg.Hierarchy(A)
    b = torch.as_tensor(I.rhs(A.n, 2)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    kw = dict(method=amg.PCG, tol=1e-8, maxit=200, adaptive=True, k=3, s=1, rho_max=0.5, gamma_min=0.01,
              zero_guess=True)

    def step():
        h.sparsify(args.gamma, 2)
        return h.solve(b, x, **kw)

    kern, lvl = dominant_kernel(h, step)
    ms_step, res, cnt, ms_total = timed_steps(h, step, args.hbm_steps, 2, kern, lvl)
    per = ms_total / max(cnt, 1) / 1e3
    nb = launch_bytes(h, kern, lvl)
    li = h.level_info(lvl)
    ach = nb / per / 1e9
    log(f"[bench] {N2}^3: {ms_step:.3f} ms/step, {res.iters} iters; {kern}@{lvl}: {per * 1e6:.1f} us, "
        f"{ach:.0f} GB/s, frac {ach / HBM_PEAK_GBS:.3f}")
    out = dict(workload=f"3D Poisson 7-point {N2}^3 (n={A.n}, nnz={A.nnz}), the same step", kernel=f"{kern} level {lvl}",
               operator_mb=round(12 * li["nnz_hat"] / 1e6, 1), bytes_per_launch=nb, us_per_launch=round(per * 1e6, 3),
               launches=cnt, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
               traffic=traffic_for(kern, lvl, N=N2), ms_per_step=round(ms_step, 4), iters=res.iters,
               steps=args.hbm_steps)
    h.close()
    return out


def cpu_baseline(args, A, b_host) -> dict:
    """The oracle on the host's cores, setup excluded: the OpenMP timing build
    on every core this process may use, and the single-threaded parity build,
    each on a bounded number of full steps (sparsify + adaptive PCG); both
    builds must return the same bits."""
    from oracle import oracle as O
    runs = {}
    for parallel in (True, False):
        if not parallel and A.n > 3_000_000:
            continue
        label = "openmp" if parallel else "single_thread"
        log(f"[bench] CPU baseline ({label}): oracle setup (untimed) ...")
        o = O.OracleAMG(A, parallel=parallel)
        done, xs = 0, None
        t0 = time.perf_counter()
        while done < args.cpu_steps:
            o.sparsify_from(args.gamma, 2)
            xs, r = o.solve(b_host, method=O.PCG, tol=1e-8, maxit=200, adaptive=True, k=3, s=1)
            done += 1
            if time.perf_counter() - t0 > 20.0:
                break
        sec = time.perf_counter() - t0
        runs[label] = dict(value=round(done / sec, 5), steps=done, seconds=round(sec, 3),
                           cores=omp_threads() if parallel else 1, x=xs)
        log(f"[bench] CPU baseline ({label}): {done / sec:.4f} solves/s over {done} steps")
        del o
    same = None
    if "single_thread" in runs:
        same = runs["openmp"]["x"].tobytes() == runs["single_thread"]["x"].tobytes()
    for r in runs.values():
        r.pop("x")
    omp = runs["openmp"]
    return {
        "value": omp["value"],
        "unit": "solves/s",
        "cores": omp["cores"],
        "kind": "oracle",
        "sample": f"{omp['steps']} full steps (sparsify gamma={args.gamma} + adaptive PCG to 1e-8) of the same "
                  f"workload, C oracle OpenMP timing build, setup excluded",
        "single_thread": runs.get("single_thread"),
        "same_bits_as_single_thread": same,
        "host": host_description(),
    }


def bench_setup(args):
    """Device-resident setup of the 3D Poisson problem N^3 (default 128^3):
    strength, PMIS split, direct interpolation and the Galerkin products of
    every level in device kernels, from the matrix already in HBM.  One step
    = one whole hierarchy built (and released).  Also reported: the RS device
    setup (same hierarchy as the host setup), the host setup, and the
    sparsified adaptive PCG solve to 1e-8 on each hierarchy (time to
    solution = setup + solve)."""
    import numpy as np
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    N = args.N
    A = I.poisson3d(N)
    b_host = I.rhs(A.n, 2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
        ci = torch.from_numpy(A.col.astype(np.int32)).cuda()
        v = torch.from_numpy(A.val).cuda()
        b = torch.from_numpy(b_host).cuda()
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")

        def build(coarsening="pmis", where="device"):
            if where == "host":
                return amg.Hierarchy(A)
            return amg.Hierarchy((A.n, rp, ci, v), setup="device", coarsening=coarsening, seed=1)

        log(f"[bench] device setup of 3D Poisson {N}^3 (n={A.n}, nnz={A.nnz})")
        for _ in range(args.warmup):
            build().close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            build().close()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ms_per_step = elapsed / args.steps * 1e3
        log(f"[bench] {args.steps} PMIS device setups: {ms_per_step:.2f} ms each")
        # kernel classes by HIP events over the same number of setups
        amg.setup_profile_enable(True)
        for _ in range(args.steps):
            build().close()
        torch.cuda.synchronize()
        prof = amg.setup_profile_read()
        amg.setup_profile_enable(False)
        dom = max(prof, key=lambda k: prof[k][1])
        cnt, ms, nbytes = prof[dom]
        achieved = nbytes / (ms / 1e3) / 1e9
        log(f"[bench] dominant class {dom}: {cnt} groups, {ms / args.steps:.2f} ms per setup, "
            f"{achieved:.0f} GB/s")

        compare = {}
        solve_kw = dict(method=amg.PCG, tol=1e-8, maxit=300, adaptive=True, k=3, s=1, rho_max=0.5,
                        gamma_min=0.01)
        for label, co, where in (("device_pmis", "pmis", "device"), ("device_rs", "rs", "device"),
                                 ("host_rs", "rs", "host")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = build(co, where)
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            sizes = [(h.level_info(l)["n"], h.level_info(l)["nnz"]) for l in range(h.nlev)]
            h.sparsify(args.gamma, 2)
            x.zero_()
            res = h.solve(b, x, **solve_kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                h.sparsify(args.gamma, 2)
                x.zero_()
                res = h.solve(b, x, **solve_kw)
            torch.cuda.synchronize()
            solve_ms = (time.perf_counter() - t0) / reps * 1e3
            compare[label] = dict(setup_ms=round(setup_s * 1e3, 2), levels=h.nlev,
                                  operator_complexity=round(sum(z for _, z in sizes) / sizes[0][1], 4),
                                  solve_iters=res.iters, solve_ms=round(solve_ms, 3), relres=res.relres,
                                  time_to_solution_ms=round(setup_s * 1e3 + solve_ms, 2))
            log(f"[bench] {label}: setup {setup_s * 1e3:.1f} ms, {h.nlev} levels, solve {res.iters} it "
                f"{solve_ms:.2f} ms")
            h.close()

    out = {
        "metric": "hierarchies set up per second (device-resident AMG setup: strength, PMIS, direct "
                  "interpolation, Galerkin products on every level)",
        "value": round(args.steps / elapsed, 4),
        "unit": "setups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Poisson 7-point FD {N}^3 (n={A.n}, nnz={A.nnz}) resident in HBM; strength "
                        f"theta=0.25, PMIS (SplitMix64 weights, seed 1), direct interpolation, "
                        f"Galerkin products to <50 rows; then Sparse Galerkin gamma={args.gamma} and "
                        f"adaptive AMG-PCG to 1e-8 on each hierarchy for the time to solution",
        },
        "setup_classes_ms_per_setup": {k: round(prof[k][1] / args.steps, 3) for k in prof},
        "compare": compare,
        "roofline": {
            "bound": "hbm",
            "kernel": f"setup class {dom}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": round(nbytes / max(cnt, 1)),
            "us_per_launch": round(ms / max(cnt, 1) * 1e3, 3),
            "launches": cnt,
        },
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] CPU baseline: one oracle PMIS setup ...")
        t0 = time.perf_counter()
        O.OracleAMG(A, coarsening="pmis", seed=1)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(1.0 / cpu_s, 5),
            "unit": "setups/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"one whole setup (PMIS seed 1, same {N}^3 problem) by the single-threaded C oracle",
        }
        log(f"[bench] CPU baseline {cpu_s:.2f} s per setup")
    print(json.dumps(out), flush=True)


GAMMAS = (0.01, 0.1, 1.0)


def bench_methods(args):
    """The paper's comparison (Section 5) on one GPU: the Galerkin hierarchy,
    Sparse and Hybrid Galerkin post-passes over it (Section 3, diagonal
    lumping, adaptive reintroduction), and non-Galerkin hierarchies whose
    coarse products are sparsified during setup (Section 2.1), on levels >= 2
    with gamma in {0.01, 0.1, 1}.  Per method: adaptive AMG-PCG to 1e-8 (k=3,
    s=1), its iterations, reintroductions, time to solution (median and
    minimum of 5), operator complexity and algorithmic bytes per V-cycle (the
    one-GPU image of the communication the paper counts)."""
    import numpy as np
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    kw = dict(method=amg.PCG, tol=1e-8, maxit=300, adaptive=True, k=3, s=1, rho_max=0.5, gamma_min=0.01)
    problems = ((f"poisson3d_{args.N}", lambda: I.poisson3d(args.N), 2),
                ("aniso2d_1024", lambda: I.aniso2d(1024), 3))
    results = {}
    best = None
    for name, make, seed in problems:
        A = make()
        b = torch.as_tensor(I.rhs(A.n, seed)).cuda()
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        log(f"[bench] methods: {name} (n={A.n}, nnz={A.nnz})")
        rows = {}

        def measure(h, prepare):
            def run():
                prepare()
                x.zero_()
                return h.solve(b, x, **kw)
            run()
            ts = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = run()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            # kernel time per level and iteration (HIP events on every launch of one solve)
            prepare()
            x.zero_()
            h.profile_enable(True)
            rp_ = h.solve(b, x, **kw)
            torch.cuda.synchronize()
            per_level = []
            for l in range(h.nlev):
                tot = 0.0
                for kern in amg.KERNEL:
                    if kern in ("SPARSIFY", "LUMP_DEN", "LUMP_SHARES"):
                        continue
                    tot += h.profile_read(kern, l)[1]
                per_level.append(round(tot / max(rp_.iters, 1) * 1e3, 2))
            h.profile_enable(False)
            prepare()
            nnz = [h.level_info(l)["nnz_hat"] for l in range(h.nlev)]
            return dict(ms_to_1e8=round(float(np.median(ts)), 3), ms_min=round(min(ts), 3), iters=r.iters,
                        us_per_iteration_by_level=per_level,
                        reintroductions=r.reintroductions, converged=bool(r.converged), relres=r.relres,
                        operator_complexity=round(sum(nnz) / A.nnz, 4), bytes_per_vcycle=h.bytes_per_cycle(),
                        nnz_per_level=nnz, levels=h.nlev), run

        h = amg.Hierarchy(A)
        variants = [("galerkin", None, False)] + [(f"sparse_galerkin_{g}", g, False) for g in GAMMAS] + \
                   [(f"hybrid_galerkin_{g}", g, True) for g in GAMMAS]
        for label, gamma, hybrid in variants:
            def prepare(gamma=gamma, hybrid=hybrid):
                h.set_method(hybrid)
                h.sparsify(0.0 if gamma is None else gamma, 2)
            rows[label], run = measure(h, prepare)
            log(f"[bench]   {label}: {rows[label]['ms_to_1e8']:.2f} ms, {rows[label]['iters']} it, "
                f"{rows[label]['reintroductions']} reint, complexity {rows[label]['operator_complexity']:.3f}")
            if name.startswith("poisson3d") and (best is None or rows[label]["ms_to_1e8"] < best[2]):
                best = (label, dict(gamma=gamma, hybrid=hybrid, nongalerkin=False), rows[label]["ms_to_1e8"])
        h.close()
        for g in GAMMAS:
            label = f"nongalerkin_{g}"
            ng = [0.0, 0.0] + [g] * 30
            t0 = time.perf_counter()
            hn = amg.Hierarchy(A, nongalerkin_gamma=ng)
            setup_s = time.perf_counter() - t0
            rows[label], run = measure(hn, lambda: hn.sparsify(0.0, 2))
            rows[label]["setup_s"] = round(setup_s, 3)
            log(f"[bench]   {label}: {rows[label]['ms_to_1e8']:.2f} ms, {rows[label]['iters']} it, "
                f"complexity {rows[label]['operator_complexity']:.3f}")
            if name.startswith("poisson3d") and rows[label]["ms_to_1e8"] < best[2]:
                best = (label, dict(gamma=g, hybrid=False, nongalerkin=True), rows[label]["ms_to_1e8"])
            hn.close()
        results[name] = rows

    # the fastest method on 3D Poisson: timed steps, dominant kernel by HIP events
    label, cfg, _ = best
    A = I.poisson3d(args.N)
    b_host = I.rhs(A.n, 2)
    b = torch.as_tensor(b_host).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    ng = [0.0, 0.0] + [cfg["gamma"]] * 30
    h = amg.Hierarchy(A, nongalerkin_gamma=ng) if cfg["nongalerkin"] else amg.Hierarchy(A)

    def step():
        if not cfg["nongalerkin"]:
            h.set_method(cfg["hybrid"])
            h.sparsify(0.0 if cfg["gamma"] is None else cfg["gamma"], 2)
        else:
            h.sparsify(0.0, 2)
        x.zero_()
        return h.solve(b, x, **kw)

    h.profile_enable(True)
    step()
    dom = None
    for kern in ("JACOBI", "JACOBI_ZERO", "RESIDUAL", "RESTRICT", "INTERP", "SPMV_DOT"):
        for l in range(h.nlev):
            c, ms = h.profile_read(kern, l)
            if c and (dom is None or ms > dom[2]):
                dom = (kern, l, ms)
    h.profile_enable(False)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.profile_enable(True, dom[0], dom[1])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cnt, ms_total = h.profile_read(dom[0], dom[1])
    h.profile_enable(False)
    nbytes = launch_bytes(h, dom[0], dom[1])
    per_launch_s = ms_total / max(cnt, 1) / 1e3
    achieved = nbytes / per_launch_s / 1e9
    log(f"[bench] fastest on Poisson: {label}, {elapsed / args.steps * 1e3:.3f} ms per solve; "
        f"{dom[0]}@{dom[1]} {per_launch_s * 1e6:.1f} us, {achieved:.0f} GB/s")
    out = {
        "metric": "solves/s to 1e-8 (adaptive AMG-PCG) with the fastest of the Galerkin, Sparse Galerkin, "
                  "Hybrid Galerkin and non-Galerkin hierarchies",
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Poisson 7-point FD {args.N}^3 (RHS seed 2) and 2D rotated anisotropic Q1 1024^2 "
                        f"(RHS seed 3); RS theta=0.25, direct interpolation; gamma on levels >= 2 in "
                        f"{list(GAMMAS)}, diagonal lumping; adaptive AMG-PCG (k=3, s=1, rho_max=0.5) to 1e-8; "
                        f"timed: {label} on 3D Poisson",
            "method": label,
        },
        "methods": results,
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom[0]} level {dom[1]}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(dom[0], dom[1]) if not cfg["nongalerkin"] else None,
            "bytes_per_launch": nbytes,
            "us_per_launch": round(per_launch_s * 1e6, 3),
            "launches": cnt,
        },
    }
    h.close()
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log(f"[bench] CPU baseline: oracle hierarchy (not timed), then one {label} solve ...")
        o = O.OracleAMG(A, nongalerkin_gamma=ng) if cfg["nongalerkin"] else O.OracleAMG(A)
        if not cfg["nongalerkin"]:
            o.set_method(cfg["hybrid"])
            o.sparsify_from(0.0 if cfg["gamma"] is None else cfg["gamma"], 2)
        t0 = time.perf_counter()
        o.solve(b_host, method=O.PCG, tol=1e-8, maxit=300, adaptive=True, k=3, s=1)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(1.0 / cpu_s, 5),
            "unit": "solves/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"one adaptive PCG solve with the {label} hierarchy of the same {args.N}^3 problem by the "
                      f"single-threaded C oracle, its setup excluded",
        }
        log(f"[bench] CPU baseline {cpu_s:.2f} s per solve")
    print(json.dumps(out), flush=True)


def lump_shares_bytes(h, l: int) -> int:
    """Bytes the strong-lumping share kernel must move on level l at least:
    row pointers of A_l and of its sparsified pattern, A_l's columns, values
    and keep flags, the denominators of the dropped entries, the thresholds,
    the kept columns, and every kept value read and written once."""
    s = h.level_info(l)
    n, nnz, kept = s["n"], s["nnz"], s["nnz_hat"]
    return 8 * (n + 1) + 13 * nnz + 8 * (nnz - kept) + 8 * n + 4 * kept + 16 * kept


def bench_lumping(args):
    """Sparsification with strong-neighbour lumping (Algorithm 3, second loop)
    of the 3D Poisson hierarchy: one step is one pass over every coarse level
    (keep flags, copy, thresholds, denominators, shares, inverse diagonal);
    compared with diagonal lumping (Algorithm 3b) on three problem families."""
    import numpy as np
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    N = args.N
    A = I.poisson3d(N)
    log(f"[bench] lumping: host setup of 3D Poisson {N}^3 (n={A.n}, nnz={A.nnz})")
    h = amg.Hierarchy(A)
    h.set_lumping("strong")
    for _ in range(args.warmup):
        h.sparsify(args.gamma, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h.sparsify(args.gamma, 2)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    log(f"[bench] {args.steps} strong-lumping sparsifications: {ms_per_step:.3f} ms each")
    levels = [l for l in range(h.nlev) if h.gamma(l) > 0]
    kinds = ("SPARSIFY", "LUMP_DEN", "LUMP_SHARES")
    times = {}
    for kind in kinds:
        h.profile_enable(True, kind)
        for _ in range(args.steps):
            h.sparsify(args.gamma, 2)
        torch.cuda.synchronize()
        c = ms = 0
        for l in range(h.nlev):
            cl, tl = h.profile_read(kind, l)
            c += cl
            ms += tl
        h.profile_enable(False)
        times[kind] = (c, ms)
    cnt, ms = times["LUMP_SHARES"]
    nbytes = args.steps * sum(lump_shares_bytes(h, l) for l in levels)
    achieved = nbytes / (ms / 1e3) / 1e9
    traffic = None   # HBM bytes per launch from the committed counters, if they match this source
    if os.path.exists(LUMP_TRAFFIC_FILE):
        tc = json.load(open(LUMP_TRAFFIC_FILE))
        ent = tc.get("kernels", {}).get("LUMP_SHARES")
        if ent and tc.get("kernel_source_sha") == kernel_source_sha(LUMP_KERNEL_SRC) \
                and ent["launches_per_pass"] == len(levels):
            traffic = round(ent["hbm_bytes_per_pass"] / ent["launches_per_pass"])
    log(f"[bench] share kernel: {cnt} launches, {ms / args.steps:.3f} ms per pass, {achieved:.1f} GB/s "
        f"of compulsory bytes; denominators {times['LUMP_DEN'][1] / args.steps:.3f} ms per pass")

    compare = {}
    if not args.no_compare:
        for name, make in ((f"poisson3d_{N}", lambda: A), ("aniso2d_1024", lambda: I.aniso2d(1024)),
                           ("fv3d_lognormal_96", lambda: I.fv3d_lognormal(96))):
            M = make()
            hh = h if M is A else amg.Hierarchy(M)
            b = torch.as_tensor(I.rhs(M.n, 2)).cuda()
            x = torch.zeros(M.n, dtype=torch.float64, device="cuda")
            hh.set_lumping("diagonal")
            hh.sparsify(0.0, 2)
            x.zero_()
            g = hh.solve(b, x, method=amg.PCG, tol=1e-8, maxit=300)
            rows = {"galerkin_pcg_iters": g.iters}
            for mode in ("diagonal", "strong"):
                hh.set_lumping(mode)
                for gam in (0.01, 0.1, 1.0):
                    hh.sparsify(gam, 2)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(5):
                        hh.sparsify(gam, 2)
                    torch.cuda.synchronize()
                    sp_ms = (time.perf_counter() - t0) / 5 * 1e3
                    cx = sum(hh.level_info(l)["nnz_hat"] for l in range(hh.nlev)) / M.nnz
                    x.zero_()
                    r = hh.solve(b, x, method=amg.PCG, tol=1e-8, maxit=300)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(3):
                        x.zero_()
                        r = hh.solve(b, x, method=amg.PCG, tol=1e-8, maxit=300)
                    torch.cuda.synchronize()
                    solve_ms = (time.perf_counter() - t0) / 3 * 1e3
                    rows[f"{mode}_gamma_{gam}"] = dict(sparsify_ms=round(sp_ms, 3), operator_complexity=round(cx, 4),
                                                       pcg_iters=r.iters, converged=bool(r.converged),
                                                       solve_ms=round(solve_ms, 3))
                    log(f"[bench] {name} {mode} gamma {gam}: sparsify {sp_ms:.2f} ms, complexity {cx:.3f}, "
                        f"PCG {r.iters} it {solve_ms:.2f} ms")
            compare[name] = rows
            if hh is not h:
                hh.close()
    h.close()

    out = {
        "metric": "sparsifications per second (Sparse Galerkin with strong-neighbour lumping, every coarse "
                  "level of the hierarchy)",
        "value": round(args.steps / elapsed, 4),
        "unit": "sparsifications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Poisson 7-point FD {N}^3 (n={A.n}, nnz={A.nnz}), Galerkin hierarchy (RS, direct "
                        f"interpolation) resident in HBM; gamma={args.gamma} on levels >= 2, dropped entries "
                        f"shared among strong neighbours (theta=0.25)",
        },
        "class_ms_per_step": {k: round(times[k][1] / args.steps, 4) for k in kinds},
        "compare": compare,
        "roofline": {
            "bound": "hbm",
            "kernel": "strong_lump_wide_kernel (shares)",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic,
            "bytes_per_launch": round(nbytes / max(cnt, 1)),
            "us_per_launch": round(ms / max(cnt, 1) * 1e3, 3),
            "launches": cnt,
        },
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] CPU baseline: oracle hierarchy (not timed), then one strong-lumping sparsification ...")
        o = O.OracleAMG(A)
        o.set_lumping("strong")
        t0 = time.perf_counter()
        o.sparsify_from(args.gamma, 2)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(1.0 / cpu_s, 5),
            "unit": "sparsifications/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"one strong-lumping sparsification (gamma {args.gamma}, levels >= 2) of the same "
                      f"{N}^3 hierarchy by the single-threaded C oracle, its setup excluded",
        }
        log(f"[bench] CPU baseline {cpu_s:.2f} s per sparsification")
    print(json.dumps(out), flush=True)


def bench_aniso(args):
    """Rotated anisotropic diffusion (eps = 1e-3, theta = pi/8), Q1 on 1024^2:
    AMG-PCG to 1e-10 with the V-cycle in FP64 vs in FP32, gamma in {0.01, 0.1};
    error of each solution against the FP64 oracle's."""
    import numpy as np
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    N = 1024 if args.N == 128 else args.N
    A = I.aniso2d(N)
    b_host = I.rhs(A.n, 3)
    b = torch.as_tensor(b_host).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    log(f"[bench] setup rotated anisotropic Q1 {N}^2 (n={A.n}, nnz={A.nnz})")
    t0 = time.perf_counter()
    h = amg.Hierarchy(A)
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.2f} s, {h.nlev} levels")
    # the configured iteration: PCG with the sparsified hierarchy (no adaptive window, whose
    # convergence-factor test this problem's factor of ~0.58 would trip at every window)
    kw = dict(method=amg.PCG, tol=1e-10, maxit=500)
    results = {}
    sols = {}
    for gamma in (0.01, 0.1):
        for prec in (64, 32):
            def step():
                h.sparsify(gamma, 2)
                x.zero_()
                return h.solve(b, x, precision=prec, **kw)
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                res = step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            sols[(gamma, prec)] = x.cpu().numpy()
            results[f"gamma={gamma},fp{prec}"] = dict(ms=round(ms, 3), solves_per_s=round(1e3 / ms, 3),
                                                      iters=res.iters, relres=res.relres,
                                                      reintroductions=res.reintroductions)
            log(f"[bench] gamma={gamma} fp{prec}: {ms:.2f} ms, {res.iters} iters, relres {res.relres:.2e}")
    # dominant kernel of the FP32-cycle solve at gamma 0.1, timed with HIP events
    h.sparsify(0.1, 2)

    def solve32():
        x.zero_()
        return h.solve(b, x, precision=32, **kw)

    h.profile_enable(True)
    solve32()
    dom = None
    for kern in ("JACOBI", "JACOBI_ZERO", "RESIDUAL", "RESTRICT", "INTERP", "SPMV_DOT"):
        for l in range(h.nlev):
            c, ms = h.profile_read(kern, l)
            if c and (dom is None or ms > dom[2]):
                dom = (kern, l, ms)
    h.profile_enable(False)
    h.profile_enable(True, dom[0], dom[1])
    for _ in range(args.steps):
        solve32()
    torch.cuda.synchronize()
    cnt, ms_total = h.profile_read(dom[0], dom[1])
    h.profile_enable(False)
    # the outer product and residual stay FP64; the cycle's kernels are FP32
    fp64_kernel = dom[0] == "SPMV_DOT" or (dom[0] == "RESIDUAL" and dom[1] == 0)
    nbytes = launch_bytes(h, dom[0], dom[1]) if fp64_kernel else launch_bytes32(h, dom[0], dom[1])
    per_launch_s = ms_total / max(cnt, 1) / 1e3
    achieved = nbytes / per_launch_s / 1e9
    log(f"[bench] FP32-cycle solve: dominant {dom[0]}@{dom[1]} ({'FP64' if fp64_kernel else 'FP32'}) "
        f"{per_launch_s * 1e6:.1f} us, {achieved:.0f} GB/s")
    roofline = {"bound": "hbm", "kernel": f"{dom[0]} level {dom[1]} ({'FP64' if fp64_kernel else 'FP32'})",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": nbytes,
                "us_per_launch": round(per_launch_s * 1e6, 3), "launches": cnt}
    cpu_baseline = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] FP64 oracle solutions for the error report ...")
        o = O.OracleAMG(A)
        for gamma in (0.01, 0.1):
            o.sparsify_from(gamma, 2)
            t0 = time.perf_counter()
            xo, ro = o.solve(b_host, method=O.PCG, tol=1e-10, maxit=500)
            cpu_s = time.perf_counter() - t0
            if gamma == 0.1:
                cpu_baseline = {"value": round(1.0 / cpu_s, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
                                "sample": f"one FP64 AMG-PCG solve to 1e-10 (gamma 0.1) of the same {N}^2 problem "
                                          f"by the single-threaded C oracle, its setup excluded"}
            for prec in (64, 32):
                d = results[f"gamma={gamma},fp{prec}"]
                d["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(sols[(gamma, prec)] - xo) / np.linalg.norm(xo))
                d["oracle_iters"] = ro.iters
    best = results["gamma=0.1,fp32"]
    out = {
        "metric": "solves/s to 1e-10 relative residual, FP32-preconditioned FP64 AMG-PCG vs FP64 "
                  "(rotated anisotropic Q1)",
        "value": best["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 V-cycle in f64 PCG", "data": "synthetic",
        "config": {"workload": f"2D rotated anisotropic diffusion eps=1e-3 theta=pi/8, Q1 9-point "
                               f"{N}^2 (n={A.n}, nnz={A.nnz}), RHS seed 3; Sparse Galerkin gamma on "
                               f"levels>=2; AMG-PCG to 1e-10", "levels": h.nlev},
        "setup_s": round(setup_s, 3),
        "runs": results,
        "fp32_speedup_gamma0.1": round(results["gamma=0.1,fp64"]["ms"] / best["ms"], 4),
        "fp32_speedup_gamma0.01": round(results["gamma=0.01,fp64"]["ms"] / results["gamma=0.01,fp32"]["ms"], 4),
        "roofline": roofline,
    }
    if cpu_baseline:
        out["cpu_baseline"] = cpu_baseline
    h.close()
    print(json.dumps(out), flush=True)


def block_launch_bytes(h, kernel: str, level: int, k: int, value_bytes: int, cg: bool = True) -> int:
    """Algorithmic bytes of one block launch on k columns: matrix values of
    value_bytes (4 for the FP32 cycle) plus int32 indices, each block entry
    counted once; the outer residual (RESIDUAL on level 0) reads the FP64
    operator and FP64 x, b.  cg: the block solve is PCG (else refinement)."""
    li = h.level_info(level)
    n, nnz_hat, nc, nnz_p = li["n"], li["nnz_hat"], li["n_coarse"], li["nnz_P"]
    m = value_bytes + 4
    vb = value_bytes
    if kernel == "RESIDUAL" and level == 0:
        # r = b - A x (FP64): x, b read; r and the next first sweep written at
        # the cycle's precision; dinv at the cycle's precision
        return 12 * li["nnz"] + 4 * (n + 1) + vb * n + k * n * (16 + 2 * vb)
    if kernel == "SPMV_DOT":
        # q = A p in FP64 (CG): p gathered, q written
        return 12 * li["nnz"] + 4 * (n + 1) + 16 * k * n
    if kernel == "JACOBI":
        # level 0: the last sweep writes z and reads the FP64 residual for r.z
        # (CG), or adds its result to the FP64 iterate (refinement: read + write)
        out = vb if level > 0 else (vb + 8 if cg else 16)
        return m * nnz_hat + 4 * (n + 1) + vb * n + k * n * (2 * vb + out)
    if kernel in ("JACOBI_ZERO", "RESIDUAL"):
        return m * nnz_hat + 4 * (n + 1) + k * n * 3 * vb
    if kernel == "RESTRICT":
        scale = level + 2 < h.nlev
        return m * nnz_p + 4 * (nc + 1) + k * n * vb + (vb * nc + 2 * k * nc * vb if scale else k * nc * vb)
    if kernel == "INTERP":
        return m * nnz_p + 4 * (n + 1) + k * nc * vb + 2 * k * n * vb
    return 0


def bench_fv3d(args):
    """3D cell-centred FV diffusion with lognormal cell coefficients on 192^3,
    16 right-hand sides solved together: every kernel processes all 16
    columns in one pass over its operator.  Timed step: the 16-column solve
    to 1e-10 with the V-cycle in FP32 preconditioning FP64 CG (one recurrence
    per column); also measured: FP32 cycle in FP64 iterative refinement (the
    stationary form), both with an FP64 cycle, and 16 single-right-hand-side
    FP64 / FP32-preconditioned AMG-PCG solves."""
    import numpy as np
    import scipy.sparse as S
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I

    N = 192 if args.N == 128 else args.N
    K = 16
    gamma = 0.01
    A = I.fv3d_lognormal(N, seed=40)
    log(f"[bench] fv3d {N}^3 (n={A.n}, nnz={A.nnz}); generating {K} right-hand sides")
    B_host = np.stack([I.rhs(A.n, 41 + c) for c in range(K)], axis=1)
    B = torch.as_tensor(B_host).cuda()
    X = torch.zeros(A.n, K, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    h = amg.Hierarchy(A)
    h.sparsify(gamma, 2)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup + sparsify {setup_s:.2f} s, {h.nlev} levels")

    def step(prec=32, method=amg.PCG):
        X.zero_()
        return h.solve_block(B, X, method=method, tol=1e-10, maxit=300, precision=prec)

    # dominant kernel of the timed solve by HIP-event time
    step()
    h.profile_enable(True)
    res = step()
    best = None
    for kern in ("JACOBI", "JACOBI_ZERO", "RESIDUAL", "RESTRICT", "INTERP", "SPMV_DOT"):
        for l in range(h.nlev):
            cnt, ms = h.profile_read(kern, l)
            if cnt and (best is None or ms > best[2]):
                best = (kern, l, ms, cnt)
    h.profile_enable(False)
    dom_kernel, dom_level = best[0], best[1]
    log(f"[bench] dominant kernel {dom_kernel} on level {dom_level}; {res.iters} iterations")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.profile_enable(True, dom_kernel, dom_level)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cnt, ms_total = h.profile_read(dom_kernel, dom_level)
    h.profile_enable(False)
    ms_per_step = elapsed / args.steps * 1e3
    per_launch_s = ms_total / max(cnt, 1) / 1e3
    nbytes = block_launch_bytes(h, dom_kernel, dom_level, K, 4)
    achieved = nbytes / per_launch_s / 1e9
    log(f"[bench] FP32-preconditioned block PCG: {ms_per_step:.2f} ms per 16 solves, {res.iters} iters; "
        f"{dom_kernel}@{dom_level} {per_launch_s * 1e6:.1f} us, {achieved:.0f} GB/s")
    # accuracy of every column, checked on the host in FP64
    Xh = X.cpu().numpy()
    Ssp = S.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    true_rel = [float(np.linalg.norm(B_host[:, c] - Ssp @ Xh[:, c]) / np.linalg.norm(B_host[:, c]))
                for c in range(K)]
    log(f"[bench] largest true relative residual {max(true_rel):.3e}")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3, r

    reps = max(1, min(args.steps, 3))
    others = {}
    sols = {}
    for label, prec, method in (() if args.no_compare else
                                (("fp64_block_pcg", 64, amg.PCG), ("fp32_block_ir", 32, amg.STATIONARY),
                                 ("fp64_block_ir", 64, amg.STATIONARY))):
        ms, r = timed(lambda: step(prec, method), reps)
        sols[label] = X.cpu().numpy()
        others[label] = dict(ms_for_16=round(ms, 3), iters=r.iters, relres=r.relres)
        log(f"[bench] {label}: {ms:.2f} ms, {r.iters} iters")
    xs = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    for prec in (() if args.no_compare else (64, 32)):
        def sixteen():
            its = []
            for c in range(K):
                xs.zero_()
                its.append(h.solve(B[:, c].contiguous(), xs, method=amg.PCG, tol=1e-10, maxit=300,
                                   precision=prec).iters)
            return its
        ms, its = timed(sixteen, 1)
        others[f"fp{prec}_single_pcg_x16"] = dict(ms_for_16=round(ms, 3), iters=its)
        log(f"[bench] 16 single-RHS PCG fp{prec}: {ms:.1f} ms")

    value = K * args.steps / elapsed
    out = {
        "metric": "right-hand sides solved per second to 1e-10 (16 per block; FP32 V-cycle preconditioning "
                  "FP64 CG per column)",
        "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 cycle in f64 CG", "data": "synthetic",
        "config": {"workload": f"3D cell-centred FV 7-point {N}^3 (n={A.n}, nnz={A.nnz}), lognormal(0,1) "
                               f"cell coefficients seed 40, harmonic-mean faces; 16 RHS uniform[-1,1] seeds "
                               f"41..56 in one n x 16 block; Sparse Galerkin gamma={gamma} on levels>=2; "
                               f"V(1,1) Jacobi; to 1e-10", "levels": h.nlev, "nrhs": K},
        "iters": res.iters,
        "col_iters": [int(v) for v in res.col_iters],
        "true_relres_max": max(true_rel),
        "compare": others,
        "fp32_vs_fp64_block_pcg_max_rel_diff": float(max(
            np.linalg.norm(Xh[:, c] - sols["fp64_block_pcg"][:, c]) / np.linalg.norm(sols["fp64_block_pcg"][:, c])
            for c in range(K))) if sols else None,
        "speedup_vs_16_fp64_single_pcg": round(others["fp64_single_pcg_x16"]["ms_for_16"] / ms_per_step, 4)
        if others else None,
        "speedup_vs_fp64_block_pcg": round(others["fp64_block_pcg"]["ms_for_16"] / ms_per_step, 4)
        if others else None,
        "setup_s": round(setup_s, 3),
        "roofline": {
            "bound": "hbm", "kernel": f"{dom_kernel} level {dom_level} (16-column block)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(dom_kernel, dom_level, BLOCK_TRAFFIC_FILE, BLOCK_KERNEL_SRC),
            "bytes_per_launch": nbytes, "us_per_launch": round(per_launch_s * 1e6, 3), "launches": cnt,
        },
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] CPU baseline: oracle setup (untimed) ...")
        o = O.OracleAMG(A)
        o.sparsify_from(gamma, 2)
        t0 = time.perf_counter()
        xo, ro = o.solve(B_host[:, 0], method=O.PCG, tol=1e-10, maxit=300)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(1.0 / cpu_s, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"right-hand side 1 of 16 (seed 41), FP64 AMG-PCG to 1e-10 ({ro.iters} iterations), "
                      f"single-threaded C oracle, setup excluded",
        }
        out["oracle_rel_err_col0"] = float(np.linalg.norm(Xh[:, 0] - xo) / np.linalg.norm(xo))
        log(f"[bench] CPU baseline {1.0 / cpu_s:.4f} solves/s")
    h.close()
    print(json.dumps(out), flush=True)


SERVE_LADDER = {
    "poisson2d": (100, 224, 500, 1000, 1414),
    "poisson3d": (22, 47, 100, 126),
    "aniso2d": (100, 224, 500, 1000, 1414),
}


def serve_requests(count):
    """(family, N) and right-hand-side seed of each request: family uniform
    over the three, size uniform over the family's ladder (SplitMix64 stream
    5), right-hand side seed 1000 + i."""
    from paper_1512_04629_amd import inputs as I
    fams = sorted(SERVE_LADDER)
    z = I.splitmix64(5, 2 * count)
    out = []
    for i in range(count):
        fam = fams[int(z[2 * i] % 3)]
        lad = SERVE_LADDER[fam]
        out.append((fam, lad[int(z[2 * i + 1] % len(lad))], 1000 + i))
    return out


def bench_serve(args):
    """Continuous-batching serving: requests for 14 (family, size) problems
    with n from 1e4 to 2e6, each hierarchy built once and resident, batch
    engines of 16 slots admitted against an HBM budget.  Capacity (all
    requests queued at once) of the FP32-preconditioned and the FP64 batched
    path; then Poisson arrivals at 0.8 x the FP64 capacity, served by both
    and by one-at-a-time FP64 PCG: solves/s and p50/p99 latency."""
    import numpy as np
    import scipy.sparse as S
    import torch

    from paper_1512_04629_amd import amg
    from paper_1512_04629_amd import inputs as I
    from paper_1512_04629_amd.serve import Request, SolveServer, percentile

    gens = {"poisson2d": I.poisson2d, "poisson3d": I.poisson3d, "aniso2d": I.aniso2d}
    spec = serve_requests(args.requests)
    keys = sorted({(f, N) for f, N, _ in spec})
    log(f"[bench] serve: {args.requests} requests over {len(keys)} problems")
    problems = {f"{f}_{N}": gens[f](N) for f, N in keys}
    budget = int(args.budget_gb * (1 << 30))
    t0 = time.perf_counter()
    srv = SolveServer(problems, hbm_budget=budget, slots=16, precision=32, tol=1e-10, maxit=300, gamma=0.01)
    setup_s = time.perf_counter() - t0
    log(f"[bench] {len(problems)} hierarchies built in {setup_s:.1f} s, {srv.device_bytes() / 2**30:.2f} GiB")
    rhs = [torch.as_tensor(I.rhs(problems[f"{f}_{N}"].n, seed)).cuda() for f, N, seed in spec]
    outs = [torch.zeros(b.numel(), dtype=torch.float64, device="cuda") for b in rhs]
    torch.cuda.synchronize()
    log("[bench] right-hand sides resident")

    def requests(arrivals):
        return [Request(i, f"{f}_{N}", rhs[i], float(arrivals[i]), x=outs[i].zero_())
                for i, (f, N, _) in enumerate(spec)]

    def serve(precision, arrivals):
        srv.close_engines()
        srv.precision = precision
        reqs = requests(arrivals)
        st = srv.run(reqs)
        bad = [r.rid for r in reqs if r.status != 0]
        lat = st.latencies
        per_key = {}
        for key in sorted({r.key for r in reqs}):
            rs = [r for r in reqs if r.key == key]
            occ = st.occupancy.get(key, [0, 1])
            per_key[key] = dict(count=len(rs), p50_ms=round(percentile([r.latency for r in rs], 50) * 1e3, 2),
                                p99_ms=round(percentile([r.latency for r in rs], 99) * 1e3, 2),
                                service_ms=round(float(np.mean([r.done - r.admitted for r in rs])) * 1e3, 2),
                                iters=round(float(np.mean([r.iters for r in rs])), 1),
                                slot_occupancy=round(occ[0] / max(occ[1], 1), 2))
        return reqs, dict(solves_per_s=round(len(reqs) / st.makespan, 3), makespan_s=round(st.makespan, 4),
                          p50_ms=round(percentile(lat, 50) * 1e3, 3), p99_ms=round(percentile(lat, 99) * 1e3, 3),
                          steps=st.steps, engines_created=st.engines_created, engines_evicted=st.engines_evicted,
                          peak_gib=round(st.peak_bytes / 2**30, 3), failed=len(bad),
                          iters_mean=round(float(np.mean([r.iters for r in reqs])), 2), per_problem=per_key)

    zero = np.zeros(args.requests)
    serve(32, zero)                                   # warm-up: engines, FP32 copies, allocator
    cap = {}
    for prec in (64, 32):
        _, cap[prec] = serve(prec, zero)
        log(f"[bench] capacity fp{prec}: {cap[prec]['solves_per_s']:.1f} solves/s, "
            f"p99 {cap[prec]['p99_ms']:.1f} ms")
    lam = 0.8 * cap[64]["solves_per_s"]
    gaps = -np.log(1.0 - I.uniform01(6, args.requests)) / lam
    arrivals = np.cumsum(gaps) - gaps[0]
    open_loop = {}
    for prec in (64, 32):
        reqs, open_loop[f"fp{prec}_batched"] = serve(prec, arrivals)
        log(f"[bench] lambda={lam:.1f}/s fp{prec} batched: p50 {open_loop[f'fp{prec}_batched']['p50_ms']:.2f} ms, "
            f"p99 {open_loop[f'fp{prec}_batched']['p99_ms']:.2f} ms")
    # accuracy of a sample of the FP32 results, on the host in FP64
    worst = 0.0
    for r in reqs[:: max(1, args.requests // 32)]:
        A = problems[r.key]
        Sp = S.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
        b = r.b.cpu().numpy()
        worst = max(worst, float(np.linalg.norm(b - Sp @ r.x.cpu().numpy()) / np.linalg.norm(b)))
    seq_reqs = requests(arrivals)
    st = srv.run_sequential(seq_reqs, precision=64)
    open_loop["fp64_one_at_a_time"] = dict(
        solves_per_s=round(len(seq_reqs) / st.makespan, 3), makespan_s=round(st.makespan, 4),
        p50_ms=round(percentile(st.latencies, 50) * 1e3, 3), p99_ms=round(percentile(st.latencies, 99) * 1e3, 3),
        failed=sum(r.status != 0 for r in seq_reqs))
    log(f"[bench] one-at-a-time fp64: p50 {open_loop['fp64_one_at_a_time']['p50_ms']:.2f} ms, "
        f"p99 {open_loop['fp64_one_at_a_time']['p99_ms']:.2f} ms")
    out = {
        "metric": "solves/s to 1e-10 and p50/p99 latency, continuous-batching server (FP32 V-cycle "
                  "preconditioning FP64 CG vs FP64)",
        "value": cap[32]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(cap[32]["makespan_s"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 cycle in f64 CG", "data": "synthetic",
        "config": {"workload": f"{args.requests} requests, family uniform over 2D 5-point / 3D 7-point / 2D "
                               f"rotated anisotropic Q1, size uniform over N in {SERVE_LADDER} (n 1e4..2e6), "
                               f"RHS uniform[-1,1] seed 1000+i; Sparse Galerkin gamma=0.01; 16-slot engines; "
                               f"PCG to 1e-10; HBM budget {args.budget_gb} GiB",
                   "problems": len(problems)},
        "capacity": {f"fp{p}_batched": cap[p] for p in (64, 32)},
        "arrival_rate_per_s": round(lam, 3),
        "open_loop": open_loop,
        "fp32_capacity_speedup": round(cap[32]["solves_per_s"] / cap[64]["solves_per_s"], 4),
        "true_relres_max_sample": worst,
        "setup_s": round(setup_s, 2),
        "resident_gib": round(srv.device_bytes() / 2**30, 3),
    }
    # the kernels the server runs, measured alone: the largest problem's engine with all 16 slots
    # busy, FP32 cycle, iterations launched one by one so that HIP events can bracket them
    srv.close_engines()
    big = max(srv.hier, key=lambda k: srv.hier[k].n)
    hb = srv.hier[big]
    bt = hb.batch(16, 32, 1e-10, 300, graphs=False)
    rhs16 = [torch.as_tensor(I.rhs(hb.n, 9000 + i)).cuda() for i in range(16)]
    torch.cuda.synchronize()   # the copies ran on the default stream, the engine reads on its own
    for t in rhs16:
        bt.submit(t)
    bt.step(2)
    bt.poll(True)
    hb.profile_enable(True)
    bt.step(3)
    bt.poll(True)
    dom = None
    for kern in ("JACOBI", "JACOBI_ZERO", "RESIDUAL", "RESTRICT", "INTERP", "SPMV_DOT"):
        for l in range(hb.nlev):
            c, ms = hb.profile_read(kern, l)
            if c and (dom is None or ms > dom[2]):
                dom = (kern, l, ms)
    hb.profile_enable(True, dom[0], dom[1])
    bt.step(8)
    bt.poll(True)
    cnt, ms_total = hb.profile_read(dom[0], dom[1])
    hb.profile_enable(False)
    bt.close()
    nbytes = block_launch_bytes(hb, dom[0], dom[1], 16, 4)
    per_launch_s = ms_total / max(cnt, 1) / 1e3
    achieved = nbytes / per_launch_s / 1e9
    log(f"[bench] {big} engine alone: dominant {dom[0]}@{dom[1]} {per_launch_s * 1e6:.1f} us, {achieved:.0f} GB/s")
    out["roofline"] = {"bound": "hbm", "kernel": f"{dom[0]} level {dom[1]} (16-column block, {big})",
                       "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": nbytes,
                       "us_per_launch": round(per_launch_s * 1e6, 3), "launches": cnt}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] CPU baseline: oracle PCG on the requests in order (setups untimed) ...")
        oracles, solved, cpu_s = {}, 0, 0.0
        for i, (f, N, seed) in enumerate(spec):
            key = f"{f}_{N}"
            if key not in oracles:
                o = O.OracleAMG(problems[key])
                o.sparsify([0.0, 0.0] + [0.01] * (o.nlev - 2))
                oracles[key] = o
            b = rhs[i].cpu().numpy()
            t1 = time.perf_counter()
            oracles[key].solve(b, method=O.PCG, tol=1e-10, maxit=300)
            cpu_s += time.perf_counter() - t1
            solved += 1
            if cpu_s > 20.0:
                break
        out["cpu_baseline"] = {"value": round(solved / cpu_s, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {solved} requests in order, FP64 AMG-PCG to 1e-10, "
                                         f"single-threaded C oracle, setups excluded"}
        log(f"[bench] CPU baseline {solved / cpu_s:.3f} solves/s over {solved} requests")
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
