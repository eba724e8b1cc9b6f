#!/usr/bin/env python3
"""Benchmark of the matrix-free line-preconditioned CG solver on one MI355X.

Main timed loop (the `value`): full FP64 solves of the 512 x 512 x 128
periodic problem (anisotropy ratio 1e5, vertical grading 1.05, right-hand
side U[-1, 1) from seed 1) to relative residual 1e-8 with the two fused
sweeps per iteration.  One step = one complete solve (start-up kernels, all
iterations, exit correction, flag read-backs) with b already in HBM.
value = unknowns * iterations / wall time of the timed steps.

Every launch of kernel A (the dominant kernel) in the timed steps is
bracketed by HIP event nodes on the stream it runs on; its mean duration and
its algorithmic bytes per launch give the `roofline` object.  Kernel B's
launches are timed the same way in a few profiled solves after the timed
steps.  `cpu_baseline` times the
CPU oracle (plain C, one thread) on a bounded sample of the same workload.
Extras (not timed in `value`): production graph path, unfused comparator,
matrix-free vs CSR operator, the 64 x 64 x 32 latency case, mixed precision
vs FP64 at 1024 x 1024 x 128, and a plain copy kernel as the HBM ceiling.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import re
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "unknowns·iter/s + HBM GB/s; mixed vs FP64 @1e-8 resid; served p50/p99 latency"
PEAK_HBM_GBPS = 8000.0
# Algorithmic bytes per unknown per launch (FP64): every vector touched once.
# The first kernel B of a zero-start solve reads b instead of r and q (24 B),
# the first kernel A reads only z (32 B).
BYTES = {"fused_apply": 56, "fused_prec": 32, "iteration": 88, "unfused_iteration": 160,
         "apply": 16, "precond": 16, "fused_apply_first": 16, "fused_apply_second": 48,
         "fused_prec_first": 16}


def solve_kernel_bytes(kernel, iterations, n):
    """Algorithmic bytes of all launches of a fused kernel in one zero-start
    solve of `iterations` iterations (A runs k times, B k+1 times).  A's
    first launch reads z and writes q (u, zero, is not written; p = z is
    not stored: z's vector serves as p), its second reads p, q, z and
    writes u, p, q (u is not read), later ones move all seven vectors."""
    if kernel == "fused_apply":
        if iterations <= 1:
            return n * BYTES["fused_apply_first"] * iterations
        return n * (BYTES["fused_apply_first"] + BYTES["fused_apply_second"] +
                    BYTES["fused_apply"] * (iterations - 2))
    return n * (BYTES["fused_prec_first"] + BYTES["fused_prec"] * iterations)


def fp64_solve_bytes(k, n):
    """Algorithmic bytes of a zero-start FP64 fused solve of k >= 1 iterations
    with the line preconditioner: kernels A and B (solve_kernel_bytes) and
    the exit correction u += alpha p (read u, p, write u: 24 bytes/unknown;
    16 after a single iteration, when u is still unset and not read)."""
    return (solve_kernel_bytes("fused_apply", k, n) + solve_kernel_bytes("fused_prec", k, n) +
            n * (24 if k >= 2 else 16))


def mixed_solve_bytes(inner, steps, n):
    """Algorithmic bytes of a zero-start mixed-precision solve with `steps`
    refinement steps and `inner` FP32 inner iterations in all (the counts a
    pcg_result reports).  An inner solve of k iterations moves 44k - 16
    bytes/unknown: kernel B 8 + 16k (its first launch reads b and writes z),
    kernel A 8 + 24 + 28(k - 2) (first: read z, write q; second: u not
    read); its exit correction is folded into the update.  (Exact when every
    inner solve runs at least two iterations; one of a single iteration
    moves 4 bytes/unknown more.)  The FP64 steps:
    steps + 1 residuals r32 = (b - A x) scale, 20 each (read x, b, write
    r32; the first reads b only: 12), and `steps` updates
    x += (u32 + alpha p32) / scale, 24 each (read x, u32, p32, write x; the
    first does not read x: 16)."""
    if steps == 0:
        return n * (12 + 8)   # one residual, then x = 0 written
    return n * (44 * inner - 16 * steps + (12 + 20 * steps) + (16 + 24 * (steps - 1)))


def solve_roofline(bytes_per_solve, ms_per_solve):
    """Whole-solve bandwidth: algorithmic bytes over wall time per solve
    (launch gaps, flag read-backs and finalize launches included)."""
    gbps = bytes_per_solve / (ms_per_solve * 1e-3) / 1e9
    return dict(bound="hbm", algorithmic_bytes_per_solve=bytes_per_solve, achieved=gbps,
                peak=PEAK_HBM_GBPS, unit="GB/s", frac=gbps / PEAK_HBM_GBPS)


KERNEL_PATTERN = {
    "fused_apply": r"k_fused_apply<double, \d+, (true|false), false, (true|false), (true|false)>",
    "fused_prec": r"k_fused_prec<double, \d+, (true|false), false, (true|false), (true|false), "
                  r"(true|false)>",
    # the first launch of each in a solve runs its own kernel
    "fused_apply_first": r"k_fused_apply_first<double, \d+, (true|false), false, (true|false), "
                         r"(true|false), \d+, (true|false)>",
    "fused_prec_first": r"k_fused_prec_first<double, \d+, (true|false), false, (true|false), "
                        r"(true|false), \d+, (true|false)>"}
STREAM_BYTES = 64 << 20       # vectors at least this large use nontemporal accesses
CACHE_Z_BYTES = 384 << 20     # ... and kernel B stores z cached up to this size


def kernel_symbol(kernel, lanes_per_column, n, nz, elem=8, stretched=False, nrhs=1):
    """Template instance of a fused kernel that runs for this launch shape:
    M levels per lane, 16-byte vector path when whole chunks are aligned,
    nontemporal accesses for vectors that cannot stay in the caches, one
    column per wavefront (64 lanes per column)."""
    m = 1
    while m * lanes_per_column < nz:
        m *= 2
    vec = nz % m == 0 and (m * elem) % 16 == 0 and (nz * elem) % 16 == 0
    nt = n * nrhs * elem >= STREAM_BYTES and m * elem == 16
    t = "double" if elem == 8 else "float"
    b = lambda v: str(v).lower()
    sym = "k_%s<%s, %d, %s, %s, %s, %s" % (kernel, t, m, b(vec), b(stretched), b(nt),
                                           b(lanes_per_column == 64))
    if kernel == "fused_prec":   # z stored cached (nontemporal instances only)
        sym += ", %s" % b(nt and n * nrhs * elem <= CACHE_Z_BYTES)
    return sym + ">"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources the fused kernels A and B are built from: a traffic
    summary taken with other sources does not describe them."""
    h = hashlib.sha256()
    for f in ("kernels.h", "kernels_f64.hip", "kernels_f32.hip", "column.h", "device_common.h",
              "internal.h"):
        with open(os.path.join(ROOT, "paper_1302_7193_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload_tag: str, symbol: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source and launch shape (else
    None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload_tag))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    # a first-launch kernel's name carries more template arguments (its step,
    # and kernel B's cache policy for z, which follows the general kernel's)
    stored = kv.get("kernel", "")
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or not (
            stored == symbol or (kernel.endswith("_first") and stored.startswith(symbol[:-1] + ","))):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def solve_mean_traffic(kernel, iterations, symbol):
    """HBM bytes per launch of kernel A or B averaged over its launches in a
    solve of `iterations` iterations, as the event timings are: the first
    launch (its own kernel) and the others (A: k - 1 of them, B: k), each
    from its committed counter summary; None unless both are current."""
    args = symbol[symbol.index("<") + 1:-1].split(", ")
    head, cz = args[:6], args[6:]      # kernel B: its z cache policy last
    first = measured_traffic(kernel + "_first", "512x512x128",
                             "k_%s_first<%s>" % (kernel, ", ".join(head)))
    if first is not None and cz:
        path = os.path.join(ROOT, "profiles", "traffic_%s_first_512x512x128.txt" % kernel)
        stored = [ln.split("=", 1)[1].strip() for ln in open(path) if ln.startswith("kernel =")]
        if not stored or not stored[0].endswith(", %s>" % cz[0]):
            first = None
    rest = measured_traffic(kernel, "512x512x128", symbol)
    if first is None or rest is None:
        return None
    others = iterations - 1 if kernel == "fused_apply" else iterations
    return (first + others * rest) / (1 + others)


def run_main(pcg, si, torch, steps, warmup):
    nx, ny, nz = 512, 512, 128
    desc = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, 1e5, pcg.PCG_BC_PERIODIC)
    P = pcg.Problem(desc)
    n = P.n
    b = torch.from_numpy(si.rhs_uniform(nx, ny, nz, 1)).cuda()
    x = torch.empty_like(b)
    # the timed solves carry event nodes around kernel A only (the dominant
    # kernel of the roofline); kernel B is timed in a profiled pass after them
    opts = pcg.pcg_default_opts(rtol=1e-8, profile=2, x0_zero=1, graph_chunk=-1)
    tuning = pcg.pcg_get_tuning(P, pcg.PCG_F64).as_dict()
    ws = pcg.workspace(P, opts)
    for _ in range(warmup):
        st, r = pcg.pcg_solve(P, b, x, ws, opts)
        assert st == pcg.PCG_OK, r
    torch.cuda.synchronize()
    iters = launches = 0
    ms = {"fused_apply": 0.0, "fused_prec": 0.0}
    cnt = {"fused_apply": 0, "fused_prec": 0}
    t0 = time.perf_counter()
    for _ in range(steps):
        st, r = pcg.pcg_solve(P, b, x, ws, opts)
        iters += r["iterations"]
        launches += r["launches"]
        ms["fused_apply"] += r["ms_apply_kernel"]
        ms["fused_prec"] += r["ms_precond_kernel"]
        cnt["fused_apply"] += r["n_apply_kernel"]
        cnt["fused_prec"] += r["n_precond_kernel"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert st == pcg.PCG_OK, r
    # kernel B: the same solves with events around both kernels, untimed,
    # scaled to the timed solves' launch count
    ob = pcg.pcg_default_opts(rtol=1e-8, profile=1, x0_zero=1, graph_chunk=-1)
    reps = min(steps, 5)
    mb = nb = 0
    for _ in range(reps):
        _, rb = pcg.pcg_solve(P, b, x, ws, ob)
        mb += rb["ms_precond_kernel"]
        nb += rb["n_precond_kernel"]
    cnt["fused_prec"] = nb * steps // reps
    ms["fused_prec"] = mb / max(nb, 1) * cnt["fused_prec"]
    return dict(P=P, b=b, x=x, n=n, nz=nz, steps=steps, iters=iters, elapsed=elapsed, ms=ms,
                cnt=cnt, launches=launches, last=r, tuning=tuning)


def cuda_time(torch, fn, reps):
    """Mean ms per call of fn() with events on the current stream."""
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cold_time(torch, fn, n, dtype, reps, k=3):
    """Mean ms per call of fn(x, y) cycling over k input/output vector pairs
    of n values, so that each call reads vectors the previous calls did not
    touch (k pairs of the main workload's size exceed the 256 MB Infinity
    Cache)."""
    xs = [torch.rand(n, dtype=dtype, device="cuda") for _ in range(k)]
    ys = [torch.empty_like(xs[0]) for _ in range(k)]
    for i in range(k):
        fn(xs[i], ys[i])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        fn(xs[i % k], ys[i % k])
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def hbm_probe(pcg, torch, n=1 << 25, reps=10):
    """The library's streaming kernel (pcg_stream_probe) with the access mixes
    of kernel A (4 vectors in / 3 out), kernel B (2 / 2) and a copy (1 / 1),
    on vectors of the main workload's size (n FP64 values): the best over
    workgroup counts and the probe's nontemporal patterns (none, every
    access, all but the first vector's reads -- kernel A's -- and all but the
    last vector's writes -- kernel B's).  The practical ceiling beside the
    8 TB/s peak."""
    vecs = [torch.full((n,), 1.0 + k, dtype=torch.float64, device="cuda") for k in range(7)]
    out = {}
    for name, nr, nw in (("copy", 1, 1), ("kernel_b_mix", 2, 2), ("kernel_a_mix", 4, 3)):
        best = None
        for nt in (0, 1, 2, 3):
            for blocks in (4096, 16384, 65536):
                ms = cuda_time(torch, lambda: pcg.pcg_stream_probe(vecs[:nr], vecs[nr:nr + nw],
                                                                   nt, blocks), reps)
                gbps = (nr + nw) * n * 8 / (ms * 1e-3) / 1e9
                if best is None or gbps > best["GBps"]:
                    best = dict(GBps=gbps, nontemporal=nt, blocks=blocks, vectors_in=nr,
                                vectors_out=nw, bytes_per_vector=n * 8)
        out[name] = best
        log("probe %s: %.0f GB/s" % (name, best["GBps"]))
    del vecs
    return out


def timed_solves(pcg, torch, P, b, x, ws, opts, reps):
    st, r = pcg.pcg_solve(P, b, x, ws, opts)          # warm (graph capture, chunk length)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for _ in range(reps):
        st, r = pcg.pcg_solve(P, b, x, ws, opts)
        its += r["iterations"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt / reps * 1e3, its / reps, st, r


class OracleSolve(threading.Thread):
    """The oracle's FP64 solve of the 1024 x 1024 x 128 workload (smooth field
    + 1 % noise, seed 2) to relative residual 1e-12, on a host thread while
    the GPU extras run (the C oracle releases the interpreter lock): the
    reference the mixed-precision and FP64 GPU solutions are compared with."""

    def __init__(self):
        super().__init__(daemon=True)
        self.result, self.error, self.seconds = None, None, 0.0

    def run(self):
        try:
            import oracle
            import synth_inputs as si
            t0 = time.perf_counter()
            g = oracle.grid_from_ratio(1024, 1024, 128, 1e4, q=1.05)
            b = si.rhs_smooth_noise(1024, 1024, 128, 2)
            A = oracle.assemble(g)
            ref = oracle.pcg(A, oracle.line_blocks(A, 128), b, rtol=1e-12)
            del A
            self.result = dict(x=ref["x"], iterations=ref["iterations"],
                               rel_res_true=ref["rel_res_true"])
            self.seconds = time.perf_counter() - t0
        except Exception as e:  # reported in the extras
            self.error = repr(e)


def extras(pcg, si, torch, main):
    out = {}
    P, b, x, n = main["P"], main["b"], main["x"], main["n"]
    ref3 = OracleSolve()
    ref3.start()

    # production path: HIP graph chunks, no per-kernel events
    o = pcg.pcg_default_opts(x0_zero=1, graph_chunk=-1)
    ws = pcg.workspace(P, o)
    ms, its, st, r = timed_solves(pcg, torch, P, b, x, ws, o, 20)
    out["fused_fp64_graph"] = dict(ms_per_solve=ms, iterations=its,
                                   unknowns_iter_per_s=n * its / (ms * 1e-3),
                                   algorithmic_GBps=BYTES["iteration"] * n * its / (ms * 1e-3) / 1e9)
    log("graph path: %.3f ms/solve, %.1f it" % (ms, its))

    # unfused standard PCG (separate operator / preconditioner / BLAS-1 sweeps)
    o = pcg.pcg_default_opts(x0_zero=1, fused=0, graph_chunk=-1)
    ms, its, st, r = timed_solves(pcg, torch, P, b, x, ws, o, 10)
    out["unfused_fp64"] = dict(ms_per_solve=ms, iterations=its,
                               unknowns_iter_per_s=n * its / (ms * 1e-3),
                               algorithmic_GBps=BYTES["unfused_iteration"] * n * its / (ms * 1e-3) / 1e9)
    out["fused_over_unfused_time_per_iteration"] = (
        (out["fused_fp64_graph"]["ms_per_solve"] / out["fused_fp64_graph"]["iterations"]) /
        (ms / its))
    log("unfused: %.3f ms/solve" % ms)

    # operator alone: matrix-free vs assembled CSR; line preconditioner alone
    # (inputs cycled so that no call finds its vector in the caches)
    f64 = torch.float64
    t_mf = cold_time(torch, lambda xv, yv: pcg.pcg_apply(P, pcg.PCG_F64, xv, yv), n, f64, 60)
    t_pc = cold_time(torch, lambda xv, yv: pcg.pcg_precond(P, pcg.PCG_F64, xv, yv), n, f64, 60)
    csr = torch.empty(pcg.pcg_csr_bytes(P, pcg.PCG_F64), dtype=torch.uint8, device="cuda")
    pcg.pcg_csr_build(P, pcg.PCG_F64, csr)
    t_csr = cold_time(torch, lambda xv, yv: pcg.pcg_csr_apply(P, pcg.PCG_F64, csr, xv, yv), n,
                      f64, 30)
    nnz_bytes = csr.numel() - 4 * (n + 1)           # values + column indices (+ padding)
    csr_bytes = nnz_bytes + 4 * (n + 1) + 16 * n    # + row offsets + x + y
    out["operator_fp64"] = dict(
        matrix_free_us=t_mf * 1e3, matrix_free_GBps=BYTES["apply"] * n / (t_mf * 1e-3) / 1e9,
        csr_us=t_csr * 1e3, csr_GBps=csr_bytes / (t_csr * 1e-3) / 1e9,
        csr_bytes_per_unknown=csr_bytes / n, csr_over_matrix_free_time=t_csr / t_mf,
        csr_over_matrix_free_bytes=csr_bytes / (BYTES["apply"] * n),
        line_precond_us=t_pc * 1e3, line_precond_GBps=BYTES["precond"] * n / (t_pc * 1e-3) / 1e9)
    del csr
    log("operator: MF %.1f us, CSR %.1f us, precond %.1f us" % (t_mf * 1e3, t_csr * 1e3, t_pc * 1e3))
    del ws

    # small Dirichlet problem: latency-bound (fits in cache)
    d1 = pcg.pcg_desc_from_ratio(64, 64, 32, 1.05, 1e4, pcg.PCG_BC_DIRICHLET)
    P1 = pcg.Problem(d1)
    b1 = torch.from_numpy(si.rhs_uniform(64, 64, 32, 0)).cuda()
    x1 = torch.empty_like(b1)
    o = pcg.pcg_default_opts(x0_zero=1, graph_chunk=-1)
    ws1 = pcg.workspace(P1, o)
    ms, its, st, r = timed_solves(pcg, torch, P1, b1, x1, ws1, o, 50)
    out["small_64x64x32_fp64"] = dict(ms_per_solve=ms, iterations=its,
                                      us_per_iteration=ms * 1e3 / max(its, 1),
                                      unknowns_iter_per_s=P1.n * its / (ms * 1e-3))
    log("64x64x32: %.3f ms/solve, %.1f it" % (ms, its))
    del P1, b1, x1, ws1

    # mixed precision vs plain FP64 on 1024 x 1024 x 128
    d3 = pcg.pcg_desc_from_ratio(1024, 1024, 128, 1.05, 1e4, pcg.PCG_BC_DIRICHLET)
    P3 = pcg.Problem(d3)
    b3 = si.rhs_smooth_noise_torch(1024, 1024, 128, 2)
    x3 = torch.empty_like(b3)
    res3, sol3 = {}, {}
    for name, o in (("fp64", pcg.pcg_default_opts(x0_zero=1, true_residual=1)),
                    ("mixed", pcg.pcg_default_opts(x0_zero=1, precision=pcg.PCG_PREC_MIXED))):
        ws3 = pcg.workspace(P3, o)
        ms, its, st, r = timed_solves(pcg, torch, P3, b3, x3, ws3, o, 5)
        res3[name] = dict(ms_per_solve=ms, iterations=its, outer=r["outer_iterations"],
                          status=pcg.STATUS_NAMES[st], rel_res_true=r["rel_res_true"])
        nb = (fp64_solve_bytes(r["iterations"], P3.n) if name == "fp64" else
              mixed_solve_bytes(r["iterations"], r["outer_iterations"], P3.n))
        res3[name]["roofline"] = solve_roofline(nb, ms)
        sol3[name] = x3.cpu().numpy()
        del ws3
        log("1024x1024x128 %s: %.3f ms/solve" % (name, ms))
    res3["mixed_speedup_over_fp64"] = res3["fp64"]["ms_per_solve"] / res3["mixed"]["ms_per_solve"]
    res3["unknowns"] = P3.n
    out["mixed_1024x1024x128"] = res3
    del P3, b3, x3

    out["end_to_end_512x512x128_fp64"] = end_to_end(pcg, si, torch)
    out["stretched_512x512x128_fp64"] = stretched(pcg, si, torch, out["fused_fp64_graph"])
    out["preconditioners_512x512x128"] = multigrid(pcg, si, torch)
    out["batched_256x256x64x64"] = batched(pcg, si, torch)
    out["serving_512_requests"] = serving(pcg, si, torch)
    out["serving_512_requests_auto_preconditioner"] = serving(
        pcg, si, torch, preconditioner=pcg.PCG_PRECOND_AUTO)
    out["serving_512_requests_batched"] = serving(pcg, si, torch, max_active=16, batched=True)
    out["serving_2048_small_requests"] = serving_small(pcg, si, torch)

    # error of the 1024 x 1024 x 128 solutions against the oracle's FP64 solve
    log("waiting for the oracle's 1024x1024x128 FP64 solve")
    ref3.join()
    if ref3.result is not None:
        import numpy as np
        xr = ref3.result["x"]
        nr = np.linalg.norm(xr)
        for name in ("fp64", "mixed"):
            res3[name]["rel_error_vs_fp64_oracle"] = float(np.linalg.norm(sol3[name] - xr) / nr)
        res3["fp64_oracle"] = dict(rtol=1e-12, iterations=ref3.result["iterations"],
                                   rel_res_true=ref3.result["rel_res_true"],
                                   host_seconds=ref3.seconds)
        log("1024x1024x128 error vs FP64 oracle: fp64 %.2e, mixed %.2e"
            % (res3["fp64"]["rel_error_vs_fp64_oracle"], res3["mixed"]["rel_error_vs_fp64_oracle"]))
    else:
        res3["fp64_oracle_error"] = ref3.error
    del sol3, ref3

    # plain copy kernel: attainable HBM bandwidth
    a = torch.empty(1 << 29, dtype=torch.float64, device="cuda")   # 4 GiB
    c = torch.empty_like(a)
    t_cp = cuda_time(torch, lambda: c.copy_(a), 10)
    out["hbm_copy_probe_GBps"] = 2 * a.numel() * 8 / (t_cp * 1e-3) / 1e9
    del a, c
    return out


def end_to_end(pcg, si, torch, reps=5):
    """Whole solve as a host program sees it: problem set-up (geometry tables,
    tuning lookup), workspace, right-hand side host -> device, the solve (its
    first call on a new problem builds the graph chunks), solution device ->
    host.  Pinned host buffers; median over reps fresh problems."""
    nx, ny, nz = 512, 512, 128
    desc = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, 1e5, pcg.PCG_BC_PERIODIC)
    n = nx * ny * nz
    b_host = torch.from_numpy(si.rhs_uniform(nx, ny, nz, 1)).pin_memory()
    x_host = torch.empty(n, dtype=torch.float64, pin_memory=True)
    o = pcg.pcg_default_opts(x0_zero=1, graph_chunk=-1)
    rows = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = pcg.Problem(desc)
        ws = pcg.workspace(P, o)
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        x = torch.empty_like(b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b.copy_(b_host, non_blocking=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st, r = pcg.pcg_solve(P, b, x, ws, o)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        x_host.copy_(x, non_blocking=True)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        assert st == pcg.PCG_OK, r
        rows.append((t1 - t0, t2 - t1, t3 - t2, t4 - t3, t4 - t0, r["iterations"]))
        del P, ws, b, x
    rows.sort(key=lambda t: t[4])
    setup, h2d, solve, d2h, total, its = rows[len(rows) // 2]
    out = dict(setup_ms=setup * 1e3, h2d_ms=h2d * 1e3, first_solve_ms=solve * 1e3, d2h_ms=d2h * 1e3,
               total_ms=total * 1e3, iterations=its, h2d_GBps=8 * n / h2d / 1e9,
               unknowns_iter_per_s_incl_setup_and_transfers=n * its / total)
    log("end to end: %.2f ms (set-up %.2f, H2D %.2f, solve %.2f, D2H %.2f)"
        % (total * 1e3, setup * 1e3, h2d * 1e3, solve * 1e3, d2h * 1e3))
    return out


def stretched(pcg, si, torch, uniform):
    """The main workload's operator on a stretched horizontal grid (widths
    proportional to 1 + a sin(2 pi (i + 1/2) / n), a = 0.5 in x and 0.25 in
    y, so neighbouring columns differ and the widest cell is 3x the
    narrowest): |T| and alpha_{T,T'} rebuilt per column from the widths and
    every column block factorised in the kernel.  FP64 fused solve, and the
    operator and preconditioner alone."""
    nx, ny, nz = 512, 512, 128
    d = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, 1e5, pcg.PCG_BC_PERIODIC)
    P = pcg.Problem(d, si.widths_sine(nx, 0.5), si.widths_sine(ny, 0.25))
    n = P.n
    b = torch.from_numpy(si.rhs_uniform(nx, ny, nz, 1)).cuda()
    x = torch.empty_like(b)
    o = pcg.pcg_default_opts(x0_zero=1, graph_chunk=-1, true_residual=1)
    ws = pcg.workspace(P, o)
    ms, its, st, r = timed_solves(pcg, torch, P, b, x, ws, o, 10)
    f64 = torch.float64
    t_mf = cold_time(torch, lambda xv, yv: pcg.pcg_apply(P, pcg.PCG_F64, xv, yv), n, f64, 30)
    t_pc = cold_time(torch, lambda xv, yv: pcg.pcg_precond(P, pcg.PCG_F64, xv, yv), n, f64, 30)
    out = dict(ms_per_solve=ms, iterations=its, status=pcg.STATUS_NAMES[st],
               rel_res_true=r["rel_res_true"], unknowns_iter_per_s=n * its / (ms * 1e-3),
               algorithmic_GBps=BYTES["iteration"] * n * its / (ms * 1e-3) / 1e9,
               time_per_iteration_over_uniform=(ms / its) / (uniform["ms_per_solve"] /
                                                             uniform["iterations"]),
               apply_us=t_mf * 1e3, apply_GBps=BYTES["apply"] * n / (t_mf * 1e-3) / 1e9,
               precond_us=t_pc * 1e3, precond_GBps=BYTES["precond"] * n / (t_pc * 1e-3) / 1e9,
               tuning=pcg.pcg_get_tuning(P, pcg.PCG_F64).as_dict())
    log("stretched 512x512x128: %.3f ms/solve, %.1f it" % (ms, its))
    return out


def multigrid(pcg, si, torch):
    """Tensor-product multigrid and red-black block Gauss-Seidel
    preconditioners vs vertical line relaxation on
    512 x 512 x 128 Dirichlet with weak anisotropy (1e2: line relaxation
    alone needs many iterations) and on the main workload's operator
    (anisotropy 1e5, periodic): FP64 fused solves on the graph path, mixed
    precision on the weak case, and the V-cycle's share of an iteration from
    per-phase events."""
    out = {}
    for tag, g2, bc in (("anisotropy_1e2_dirichlet", 1e2, pcg.PCG_BC_DIRICHLET),
                        ("anisotropy_1e5_periodic", 1e5, pcg.PCG_BC_PERIODIC)):
        d = pcg.pcg_desc_from_ratio(512, 512, 128, 1.05, g2, bc)
        P = pcg.Problem(d)
        b = torch.from_numpy(si.rhs_uniform(512, 512, 128, 1)).cuda()
        x = torch.empty_like(b)
        res = dict(levels=pcg.pcg_mg_levels(P))
        for name, kw in (("line_fp64", dict()), ("mg_fp64", dict(preconditioner=pcg.PCG_PRECOND_MG)),
                         ("rbgs_fp64", dict(preconditioner=pcg.PCG_PRECOND_RBGS)),
                         ("line_mixed", dict(precision=pcg.PCG_PREC_MIXED)),
                         ("mg_mixed", dict(precision=pcg.PCG_PREC_MIXED,
                                           preconditioner=pcg.PCG_PRECOND_MG))):
            if "mixed" in name and g2 > 1e4:
                continue
            o = pcg.pcg_default_opts(x0_zero=1, graph_chunk=-1, true_residual=1, **kw)
            ws = pcg.workspace(P, o)
            ms, its, st, r = timed_solves(pcg, torch, P, b, x, ws, o, 3)
            res[name] = dict(ms_per_solve=ms, iterations=its, outer=r["outer_iterations"],
                             status=pcg.STATUS_NAMES[st], rel_res_true=r["rel_res_true"],
                             ms_per_iteration=ms / max(its, 1))
            if name.endswith("fp64"):
                op = pcg.pcg_default_opts(x0_zero=1, profile=1, **kw)
                st, rp = pcg.pcg_solve(P, b, x, ws, op)
                res[name]["kernel_a_ms_per_launch"] = rp["ms_apply_kernel"] / max(rp["n_apply_kernel"], 1)
                res[name]["kernel_b_phase_ms_per_launch"] = (rp["ms_precond_kernel"] /
                                                             max(rp["n_precond_kernel"], 1))
            del ws
            log("multigrid %s %s: %.2f ms, %.1f it" % (tag, name, ms, its))
        res["mg_speedup_fp64"] = res["line_fp64"]["ms_per_solve"] / res["mg_fp64"]["ms_per_solve"]
        res["rbgs_speedup_fp64"] = (res["line_fp64"]["ms_per_solve"] /
                                    res["rbgs_fp64"]["ms_per_solve"])
        out[tag] = res
        del P, b, x
    return out


def batched(pcg, si, torch, nrhs=64):
    """64 right-hand sides (seeds 100..163) on one 256 x 256 x 64 Dirichlet
    operator (anisotropy 1e3): mixed precision, every kernel launched once for
    all right-hand sides, launch parameters from the autotuner."""
    d = pcg.pcg_desc_from_ratio(256, 256, 64, 1.05, 1e3, pcg.PCG_BC_DIRICHLET)
    P = pcg.Problem(d)
    n = P.n
    B = torch.empty(nrhs * n, dtype=torch.float64, device="cuda")
    for s_ in range(nrhs):
        si.rhs_uniform_torch(256, 256, 64, 100 + s_, out=B[s_ * n:(s_ + 1) * n])
    X = torch.empty_like(B)
    t32 = pcg.pcg_autotune(P, pcg.PCG_F32, nrhs).as_dict()
    t64 = pcg.pcg_autotune(P, pcg.PCG_F64, nrhs).as_dict()
    out = {"nrhs": nrhs, "unknowns_per_rhs": n, "tuning_fp32": t32, "tuning_fp64": t64}
    for name, o in (("mixed", pcg.pcg_default_opts(x0_zero=1, precision=pcg.PCG_PREC_MIXED)),
                    ("fp64", pcg.pcg_default_opts(x0_zero=1, true_residual=1))):
        ws = pcg.workspace(P, o, nrhs)
        pcg.pcg_solve_batched(P, nrhs, B, X, ws, o)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            st, res = pcg.pcg_solve_batched(P, nrhs, B, X, ws, o)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        its = [r["iterations"] for r in res]
        nb = sum(mixed_solve_bytes(r["iterations"], r["outer_iterations"], n) if name == "mixed"
                 else fp64_solve_bytes(r["iterations"], n) for r in res)
        out[name] = dict(ms_per_batched_solve=ms, status=pcg.STATUS_NAMES[st],
                         roofline=solve_roofline(nb, ms),
                         all_ok=all(r["status"] == 0 for r in res),
                         iterations_mean=sum(its) / nrhs, iterations_max=max(its),
                         outer_max=max(r["outer_iterations"] for r in res),
                         max_rel_res_true=max(r["rel_res_true"] for r in res),
                         rhs_unknowns_iter_per_s=n * sum(its) / (ms * 1e-3),
                         algorithmic_GBps=(44 if name == "mixed" else 88) * n * sum(its) / (ms * 1e-3) / 1e9)
        del ws
        log("batched %s: %.2f ms, %.1f it/rhs" % (name, ms, sum(its) / nrhs))
    out["mixed_speedup_over_fp64"] = out["fp64"]["ms_per_batched_solve"] / out["mixed"]["ms_per_batched_solve"]
    return out


def serving(pcg, si, torch, n_requests=512, max_active=4, preconditioner=0, batched=False,
            rate=200.0, sizes=(64, 128, 256, 512), levels=(32, 64, 128)):
    """Poisson arrivals (mean `rate`/s, seed 5) of mixed-precision solves with
    n x n x n_z grids, n in `sizes` ({64,128,256,512}), n_z in `levels`
    ({32,64,128}), anisotropy log-uniform in [1e2,1e5], U[-1,1) right-hand
    sides (seed 1000 + id), device-resident; admitted by a 200 GB HBM budget.
    The trace is replayed once to warm the per-shape state, then timed.
    batched: one scheduler advances up to max_active requests with shared
    multi-request launches (line preconditioner) instead of one worker per
    request."""
    import numpy as np
    trace = si.serving_trace(n_requests, rate, seed=5, sizes=sizes, levels=levels)
    opts = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, preconditioner=preconditioner)
    descs, bs, xs = [], [], []
    for r in trace:
        descs.append(pcg.pcg_desc_from_ratio(r["nx"], r["ny"], r["nz"], 1.05, r["gamma2"],
                                             pcg.PCG_BC_DIRICHLET))
        bs.append(si.rhs_uniform_torch(r["nx"], r["ny"], r["nz"], r["seed"]))
        xs.append(torch.empty_like(bs[-1]))
    need = max(pcg.pcg_request_bytes(d, opts) for d in descs)
    arena = torch.empty(max_active * need + (64 << 20), dtype=torch.uint8, device="cuda")
    srv = pcg.Server(arena, 200 * 10**9, max_active, batched=batched)
    torch.cuda.synchronize()

    def replay():
        t0 = time.perf_counter()
        tickets, pending, lat, done_at, stats = [None] * n_requests, set(), [0.0] * n_requests, 0.0, []
        nxt = 0
        while nxt < n_requests or pending:
            now = time.perf_counter() - t0
            while nxt < n_requests and trace[nxt]["arrival"] <= now:
                tickets[nxt] = pcg.pcg_submit_device(srv, descs[nxt], bs[nxt], xs[nxt], opts)
                pending.add(nxt)
                nxt += 1
            for i in list(pending):
                st, r = pcg.pcg_poll(srv, tickets[i])
                if st != pcg.PCG_E_AGAIN:
                    pending.discard(i)
                    lat[i] = r["elapsed_ms"]
                    stats.append((st, r["rel_res_true"], r["iterations"]))
                    done_at = time.perf_counter() - t0
            time.sleep(0.0002)
        return lat, done_at, stats

    log("serving: warm-up replay")
    replay()
    log("serving: timed replay")
    lat, span, stats = replay()
    q = pcg.pcg_server_query(srv)
    srv.close()
    lat = np.array(lat)
    ok = sum(1 for st, _, _ in stats if st == 0)
    nunk = np.array([d.nx * d.ny * d.nz for d in descs], dtype=np.float64)
    return dict(requests=n_requests, completed_ok=ok, solves_per_s=n_requests / span,
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                max_rel_res_true=float(max(r for _, r, _ in stats)),
                mean_inner_iterations=float(np.mean([it for _, _, it in stats])),
                trace_span_s=trace[-1]["arrival"], makespan_s=span,
                mean_unknowns=float(nunk.mean()), max_active=max_active,
                peak_bytes_in_use=q["peak_bytes_in_use"], budget_bytes=200 * 10**9,
                peak_active=q["peak_active"],
                mode="batched (shared multi-request launches)" if batched else
                "one worker and stream per admitted request",
                input="device-resident right-hand sides (pcg_submit_device)")


def serving_small(pcg, si, torch):
    """Many small requests at a rate no single-request path keeps up with:
    2048 mixed-precision solves on 32 x 32 or 64 x 64 grids with 32 or 64
    levels, Poisson arrivals at 20000/s, served by per-request workers (8)
    and in batched mode (64 requests per launch)."""
    kw = dict(n_requests=2048, rate=20000.0, sizes=(32, 64), levels=(32, 64))
    return dict(workers=serving(pcg, si, torch, max_active=8, **kw),
                batched=serving(pcg, si, torch, max_active=64, batched=True, **kw))


def profile_run(pcg, si, torch, steps, mixed_1024):
    """Timed solves of one configuration alone, for profiler runs: the
    1024 x 1024 x 128 mixed-precision workload, or the 64 right-hand sides on
    256 x 256 x 64 (mixed precision, launch parameters from the committed
    tuning table, no autotuning)."""
    if mixed_1024:
        nx, ny, nz, g2, nrhs = 1024, 1024, 128, 1e4, 1
    else:
        nx, ny, nz, g2, nrhs = 256, 256, 64, 1e3, 64
    d = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, g2, pcg.PCG_BC_DIRICHLET)
    P = pcg.Problem(d)
    n = P.n
    if mixed_1024:
        B = si.rhs_smooth_noise_torch(nx, ny, nz, 2)
    else:
        B = torch.empty(nrhs * n, dtype=torch.float64, device="cuda")
        for s_ in range(nrhs):
            si.rhs_uniform_torch(nx, ny, nz, 100 + s_, out=B[s_ * n:(s_ + 1) * n])
    X = torch.empty_like(B)
    o = pcg.pcg_default_opts(x0_zero=1, precision=pcg.PCG_PREC_MIXED)
    ws = pcg.workspace(P, o, nrhs)
    pcg.pcg_solve_batched(P, nrhs, B, X, ws, o)     # warm: graph chunks, chunk length
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, res = pcg.pcg_solve_batched(P, nrhs, B, X, ws, o)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    nb = sum(mixed_solve_bytes(r["iterations"], r["outer_iterations"], n) for r in res)
    return dict(workload="%dx%dx%d x %d right-hand sides, mixed precision" % (nx, ny, nz, nrhs),
                ms_per_solve=ms, inner_iterations=[r["iterations"] for r in res][:4],
                outer=[r["outer_iterations"] for r in res][:4], status=pcg.STATUS_NAMES[st],
                roofline=solve_roofline(nb, ms))


def cpu_baseline(n_iter=10):
    """Oracle (plain C, FP64, one thread) on the same 512 x 512 x 128 problem:
    assembly, then a fixed number of PCG iterations."""
    import oracle
    import synth_inputs as si
    g = oracle.grid_from_ratio(512, 512, 128, 1e5, q=1.05, periodic=True)
    b = si.rhs_uniform(512, 512, 128, 1)
    t0 = time.perf_counter()
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, g.nz)
    t1 = time.perf_counter()
    res = oracle.pcg(A, M, b, rtol=0.0, max_iter=n_iter)
    t2 = time.perf_counter()
    return dict(value=g.n * res["iterations"] / (t2 - t1), unit="unknowns·iter/s", cores=1,
                kind="oracle",
                sample="512x512x128 periodic FP64: CSR assembly (%.1f s, not in value) then %d PCG "
                       "iterations incl. start-up residual/preconditioner (%.1f s)"
                       % (t1 - t0, res["iterations"], t2 - t1))


def copy_probe(gib=1, reps=5):
    """Plain device copy of a known size (for calibrating HBM byte counters)."""
    import torch
    torch.cuda.set_device(0)
    a = torch.ones((gib << 30) // 8, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": a.numel() * 8,
                      "reps": reps}))


def _csv_rows(directory, suffix):
    import csv
    import glob
    for path in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(path) as f:
            yield path, list(csv.DictReader(f))


def _working(values, frac=0.1):
    """Dispatches that did work: an early-exit launch (the solve had already
    stopped) takes a few microseconds and moves almost nothing."""
    top = max(values) if values else 0.0
    return [v for v in values if v >= frac * top]


def summarize_rocprof(directory, kernel_filter="k_fused|k_init|k_fixup|k_finalize|k_mg|k_rb|copy|elementwise"):
    """Condense rocprofv3 CSV output under `directory` into a few lines:
    the per-kernel stats table, per-dispatch durations from the kernel trace
    (all dispatches and the ones that did work), and counter means."""
    import re
    lines = []
    for path, rows in _csv_rows(directory, "kernel_stats.csv"):
        lines.append("# kernel stats: %s" % os.path.relpath(path, directory))
        lines.append("name | calls | total_ms | avg_us | min_us | max_us | pct")
        for row in rows:
            lines.append("%s | %s | %.3f | %.2f | %.2f | %.2f | %s" % (
                row["Name"], row["Calls"], float(row["TotalDurationNs"]) / 1e6,
                float(row["AverageNs"]) / 1e3, float(row["MinNs"]) / 1e3,
                float(row["MaxNs"]) / 1e3, row.get("Percentage", "")))
    for path, rows in _csv_rows(directory, "kernel_trace.csv"):
        per = {}
        for row in rows:
            name = row["Kernel_Name"]
            if re.search(kernel_filter, name):
                per.setdefault(name, []).append(
                    (float(row["End_Timestamp"]) - float(row["Start_Timestamp"])) / 1e3)
        lines.append("# kernel trace: %s" % os.path.relpath(path, directory))
        lines.append("name | dispatches | avg_us | working_dispatches | working_avg_us")
        for name, d in sorted(per.items()):
            w = _working(d)
            lines.append("%s | %d | %.2f | %d | %.2f" % (name, len(d), sum(d) / len(d), len(w),
                                                        sum(w) / len(w)))
    for path, rows in _csv_rows(directory, "counter_collection.csv"):
        per = {}
        for row in rows:
            name = row["Kernel_Name"]
            if re.search(kernel_filter, name):
                per.setdefault((name, row["Counter_Name"]), []).append(float(row["Counter_Value"]))
        lines.append("# counters: %s" % os.path.relpath(path, directory))
        lines.append("kernel | counter | dispatches | mean | working_dispatches | working_mean")
        for (name, cn), v in sorted(per.items()):
            w = _working(v)
            lines.append("%s | %s | %d | %.1f | %d | %.1f" % (name, cn, len(v), sum(v) / len(v),
                                                              len(w), sum(w) / len(w)))
    print("\n".join(lines))


BOUNDARY = re.compile(r"k_fixup|k_residual64|k_update64|k_init|k_true_residual")


def launch_position(name):
    """Position classes of a launch of a fused kernel within one (inner) solve."""
    if "k_fused_apply" in name:
        return ("first", "second", "steady")
    if "k_fused_prec" in name:
        return ("first", "steady")
    return ("all",)


def classify_launches(rows, value_key):
    """rows: dicts with Kernel_Name, an order key and `value_key`, in dispatch
    order.  Each launch of a fused kernel that did work (at least a tenth of
    that kernel's largest value: the early-exit launches past convergence do
    not) gets its position since the last start-up, exit-correction or
    refinement kernel: kernel A's first, second and steady-state launches,
    kernel B's first and steady-state ones."""
    top = {}
    for r in rows:
        top[r["Kernel_Name"]] = max(top.get(r["Kernel_Name"], 0.0), r[value_key])
    pos, out = {}, []
    for r in rows:
        name = r["Kernel_Name"]
        if r[value_key] < 0.1 * top[name]:
            continue              # returned at once (an exit correction included)
        if BOUNDARY.search(name):
            pos = {}
        classes = launch_position(name)
        i = pos.get(name, 0)
        pos[name] = i + 1
        out.append((name, classes[min(i, len(classes) - 1)], r[value_key]))
    return out


def summarize_launches(directory, kernel_filter=r"pcg::.*k_\w+|copyBuffer"):
    """Per kernel and launch position (first / second / steady state within
    each solve): dispatches that did work and their mean duration (kernel
    trace) or mean counter value (counter runs)."""
    lines = []
    for path, rows in _csv_rows(directory, "kernel_trace.csv"):
        rs = [dict(Kernel_Name=r["Kernel_Name"], t=float(r["Start_Timestamp"]),
                   us=(float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3)
              for r in rows if re.search(kernel_filter, r["Kernel_Name"])]
        rs.sort(key=lambda r: r["t"])
        agg = {}
        for name, cls, v in classify_launches(rs, "us"):
            agg.setdefault((name, cls), []).append(v)
        lines.append("# launches by position: %s" % os.path.relpath(path, directory))
        lines.append("name | position | working_dispatches | avg_us | min_us | max_us")
        for (name, cls), v in sorted(agg.items()):
            lines.append("%s | %s | %d | %.2f | %.2f | %.2f" % (name, cls, len(v), sum(v) / len(v),
                                                              min(v), max(v)))
        # kernels A and B over all their working launches, the first-launch
        # kernel included (what the bench's HIP events time)
        fam = {}
        for (name, cls), v in agg.items():
            m = re.search(r"k_fused_(apply|prec)(_first)?<(double|float)", name)
            if m:
                fam.setdefault(("A" if m.group(1) == "apply" else "B", m.group(3)), []).extend(v)
        if fam:
            lines.append("# kernels A and B, all working launches (first-launch kernel included)")
            lines.append("kernel | precision | working_dispatches | avg_us")
            for (k, t), v in sorted(fam.items()):
                lines.append("%s | %s | %d | %.2f" % (k, t, len(v), sum(v) / len(v)))
    for path, rows in _csv_rows(directory, "counter_collection.csv"):
        per = {}
        for r in rows:
            if re.search(kernel_filter, r["Kernel_Name"]):
                per.setdefault(r["Counter_Name"], []).append(
                    dict(Kernel_Name=r["Kernel_Name"], t=int(r["Dispatch_Id"]),
                         v=float(r["Counter_Value"])))
        lines.append("# counters by position: %s" % os.path.relpath(path, directory))
        lines.append("name | position | counter | working_dispatches | mean")
        for cn, rs in sorted(per.items()):
            rs.sort(key=lambda r: r["t"])
            agg = {}
            for name, cls, v in classify_launches(rs, "v"):
                agg.setdefault((name, cls), []).append(v)
            for (name, cls), v in sorted(agg.items()):
                lines.append("%s | %s | %s | %d | %.1f" % (name, cls, cn, len(v), sum(v) / len(v)))
    print("\n".join(lines))


def traffic_by_position(fetch_dir, write_dir, cfetch_dir, cwrite_dir,
                        kernel_filter=r"pcg::.*k_\w+"):
    """HBM bytes per working dispatch of every kernel by launch position, from
    FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch), each scaled by the
    same counter's reading for a plain 1 GiB device copy (--copy-probe)."""
    def means(directory, counter, pattern):
        vals = []
        for _, rows in _csv_rows(directory, "counter_collection.csv"):
            vals += [float(r["Counter_Value"]) for r in rows
                     if r["Counter_Name"] == counter and re.search(pattern, r["Kernel_Name"])]
        w = _working(vals)
        return sum(w) / len(w)

    def by_pos(directory, counter):
        rs = []
        for _, rows in _csv_rows(directory, "counter_collection.csv"):
            rs += [dict(Kernel_Name=r["Kernel_Name"], t=int(r["Dispatch_Id"]),
                        v=float(r["Counter_Value"])) for r in rows
                   if r["Counter_Name"] == counter and re.search(kernel_filter, r["Kernel_Name"])]
        rs.sort(key=lambda r: r["t"])
        agg = {}
        for name, cls, v in classify_launches(rs, "v"):
            agg.setdefault((name, cls), []).append(v)
        return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}

    gib_kib = float(1 << 20)
    ff = gib_kib / means(cfetch_dir, "FETCH_SIZE", "copyBuffer")
    fw = gib_kib / means(cwrite_dir, "WRITE_SIZE", "copyBuffer")
    f, w = by_pos(fetch_dir, "FETCH_SIZE"), by_pos(write_dir, "WRITE_SIZE")
    lines = ["# scale factors from a 1 GiB copy: fetch x %.4f, write x %.4f" % (ff, fw),
             "name | position | fetch_kib | write_kib | dispatches | hbm_bytes_per_launch"]
    for key in sorted(set(f) & set(w)):
        (fv, nf), (wv, nw) = f[key], w[key]
        lines.append("%s | %s | %.1f | %.1f | %d | %.0f" % (key[0], key[1], fv, wv, min(nf, nw),
                                                          (fv * ff + wv * fw) * 1024))
    print("\n".join(lines))


def traffic_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, kernel, command):
    """HBM bytes per working dispatch of `kernel` from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled by the same counter's reading for a plain
    1 GiB device copy (bench.py --copy-probe)."""
    import re

    def means(directory, counter, pattern):
        vals = []
        for _, rows in _csv_rows(directory, "counter_collection.csv"):
            vals += [float(r["Counter_Value"]) for r in rows
                     if r["Counter_Name"] == counter and re.search(pattern, r["Kernel_Name"])]
        w = _working(vals)
        return sum(w) / len(w), len(w)

    gib_kib = float(1 << 20)
    cf, _ = means(cfetch_dir, "FETCH_SIZE", "copyBuffer")
    cw, _ = means(cwrite_dir, "WRITE_SIZE", "copyBuffer")
    ff, fw = gib_kib / cf, gib_kib / cw
    sym = KERNEL_PATTERN[kernel]
    names = set()
    for _, rows in _csv_rows(fetch_dir, "counter_collection.csv"):
        names |= {re.search(sym, r["Kernel_Name"]).group(0) for r in rows
                  if re.search(sym, r["Kernel_Name"])}
    if len(names) != 1:
        raise SystemExit("expected one instance of %s in the counters, found %s" % (kernel, names))
    f, nf = means(fetch_dir, "FETCH_SIZE", sym)
    w, nw = means(write_dir, "WRITE_SIZE", sym)
    out = [
        "# HBM traffic of %s on 512x512x128 (FP64, tuning in use), per dispatch" % kernel,
        "# commands: %s" % command,
        "kernel = %s" % names.pop(),
        "kernel_source_sha256_16 = %s" % kernel_source_hash(),
        "copy_probe_fetch_kib_per_gib = %.1f" % cf,
        "copy_probe_write_kib_per_gib = %.1f" % cw,
        "fetch_scale = %.4f" % ff,
        "write_scale = %.4f" % fw,
        "fetch_kib_per_dispatch = %.1f  (mean over %d working dispatches)" % (f, nf),
        "write_kib_per_dispatch = %.1f  (mean over %d working dispatches)" % (w, nw),
        "hbm_fetch_bytes_per_launch = %.0f" % (f * ff * 1024),
        "hbm_write_bytes_per_launch = %.0f" % (w * fw * 1024),
        "hbm_bytes_per_launch = %.0f" % ((f * ff + w * fw) * 1024),
    ]
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rbgs-only", action="store_true",
                    help="only FP64 block-Gauss-Seidel-preconditioned solves of 512x512x128 "
                         "Dirichlet with anisotropy 1e2 (for profiler runs of its kernels)")
    ap.add_argument("--mg-only", action="store_true",
                    help="only FP64 multigrid-preconditioned solves of 512x512x128 Dirichlet "
                         "with anisotropy 1e2 (for profiler runs of the V-cycle kernels)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only mixed-precision solves of 1024x1024x128 (for profiler runs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only mixed-precision batched solves of 64 right-hand sides on "
                         "256x256x64 with the committed tuning (for profiler runs)")
    ap.add_argument("--ops-only", action="store_true",
                    help="only the operator and the line preconditioner alone on 512x512x128 "
                         "(FP64 and FP32), --steps launches each (for profiler runs)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving replays (per-request workers and batched mode)")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed loop (for profiler runs): no extras, no CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration)")
    ap.add_argument("--summarize-rocprof", metavar="DIR",
                    help="print a text summary of rocprofv3 CSV output under DIR and exit")
    ap.add_argument("--summarize-launches", metavar="DIR",
                    help="print per-position (first / second / steady-state launch) kernel "
                         "durations and counter means from rocprofv3 CSV output under DIR")
    ap.add_argument("--traffic-by-position", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="print HBM bytes per launch of every kernel by launch position from "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE runs and exit")
    ap.add_argument("--traffic-summary", nargs=5,
                    metavar=("KERNEL", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="print the HBM traffic summary of a fused kernel (fused_apply or "
                         "fused_prec, or fused_apply_first / fused_prec_first: the first launches) from "
                         "rocprofv3 counter runs and exit")
    ap.add_argument("--traffic-command", default="",
                    help="the profiling commands, recorded in the traffic summary")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize_rocprof(args.summarize_rocprof)
        return
    if args.traffic_by_position:
        traffic_by_position(*args.traffic_by_position)
        return
    if args.summarize_launches:
        summarize_launches(args.summarize_launches)
        return
    if args.traffic_summary:
        k, fd, wd, cfd, cwd = args.traffic_summary
        traffic_summary(fd, wd, cfd, cwd, k, args.traffic_command)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(sharded, each GPU would own a block of whole columns and exchange one "
              "ring of neighbour columns per iteration)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1302_7193_amd as pcg
    import synth_inputs as si
    torch.cuda.set_device(0)

    if args.ops_only:
        d = pcg.pcg_desc_from_ratio(512, 512, 128, 1.05, 1e5, pcg.PCG_BC_PERIODIC)
        P = pcg.Problem(d)
        out = {}
        for dt, td in ((pcg.PCG_F64, torch.float64), (pcg.PCG_F32, torch.float32)):
            ms_a = cold_time(torch, lambda xv, yv: pcg.pcg_apply(P, dt, xv, yv), P.n, td, args.steps)
            ms_p = cold_time(torch, lambda xv, yv: pcg.pcg_precond(P, dt, xv, yv), P.n, td,
                             args.steps)
            csr = torch.empty(pcg.pcg_csr_bytes(P, dt), dtype=torch.uint8, device="cuda")
            pcg.pcg_csr_build(P, dt, csr)
            ms_c = cold_time(torch, lambda xv, yv: pcg.pcg_csr_apply(P, dt, csr, xv, yv), P.n, td,
                             args.steps)
            e = torch.empty(0, dtype=td).element_size()
            csr_bytes = csr.numel() + 2 * e * P.n
            del csr
            out["fp64" if dt == pcg.PCG_F64 else "fp32"] = dict(
                apply_us=ms_a * 1e3, apply_GBps=2 * e * P.n / (ms_a * 1e-3) / 1e9,
                precond_us=ms_p * 1e3, precond_GBps=2 * e * P.n / (ms_p * 1e-3) / 1e9,
                csr_us=ms_c * 1e3, csr_GBps=csr_bytes / (ms_c * 1e-3) / 1e9,
                csr_over_matrix_free=ms_c / ms_a)
        print(json.dumps(out))
        return

    if args.mixed_only or args.batched_only:
        print(json.dumps(profile_run(pcg, si, torch, args.steps, args.mixed_only)))
        return

    if args.serving_only:
        print(json.dumps(dict(workers=serving(pcg, si, torch),
                              batched=serving(pcg, si, torch, max_active=16, batched=True),
                              small=serving_small(pcg, si, torch))))
        return

    if args.mg_only or args.rbgs_only:
        d = pcg.pcg_desc_from_ratio(512, 512, 128, 1.05, 1e2, pcg.PCG_BC_DIRICHLET)
        P = pcg.Problem(d)
        b = torch.from_numpy(si.rhs_uniform(512, 512, 128, 1)).cuda()
        x = torch.empty_like(b)
        prec = pcg.PCG_PRECOND_MG if args.mg_only else pcg.PCG_PRECOND_RBGS
        o = pcg.pcg_default_opts(x0_zero=1, preconditioner=prec, graph_chunk=-1)
        ws = pcg.workspace(P, o)
        ms, its, st, r = timed_solves(pcg, torch, P, b, x, ws, o, args.steps)
        name = "MG" if args.mg_only else "RBGS"
        print(json.dumps(dict(workload="512x512x128 Dirichlet anisotropy 1e2, FP64 %s-PCG" % name,
                              ms_per_solve=ms, iterations=its, status=pcg.STATUS_NAMES[st],
                              levels=pcg.pcg_mg_levels(P) if args.mg_only else 1)))
        return

    log("main loop: %d warm-up + %d timed solves of 512x512x128" % (args.warmup, args.steps))
    m = run_main(pcg, si, torch, args.steps, args.warmup)
    n, iters, el = m["n"], m["iters"], m["elapsed"]
    value = n * iters / el
    kern = {}
    its_per_solve = iters // args.steps
    for k in ("fused_apply", "fused_prec"):
        avg = m["ms"][k] / max(m["cnt"][k], 1)
        per_launch = solve_kernel_bytes(k, its_per_solve, n) * args.steps / max(m["cnt"][k], 1)
        achieved = per_launch / (avg * 1e-3) / 1e9
        kern[k] = dict(avg_ms=avg, launches=m["cnt"][k], achieved_GBps=achieved,
                       algorithmic_bytes_per_launch=per_launch,
                       total_ms=m["ms"][k],
                       symbol=kernel_symbol(k, m["tuning"]["lanes_per_column_prec" if k == "fused_prec"
                                                             else "lanes_per_column"], n, m["nz"]))
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    for k in kern:
        kern[k]["traffic"] = solve_mean_traffic(k, its_per_solve, kern[k]["symbol"])
    traffic = kern[dom]["traffic"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns·iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "512x512x128 periodic, anisotropy 1e5, grading 1.05, "
                               "U[-1,1) seed 1, FP64 fused PCG to rel. residual 1e-8",
                   "nx": 512, "ny": 512, "nz": 128, "unknowns": n,
                   "iterations_per_solve": iters / args.steps},
        "roofline": {"bound": "hbm", "kernel": kern[dom]["symbol"],
                     "achieved": kern[dom]["achieved_GBps"], "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": kern[dom]["achieved_GBps"] / PEAK_HBM_GBPS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": kern[dom]["algorithmic_bytes_per_launch"],
                     "avg_launch_ms": kern[dom]["avg_ms"],
                     # HBM bytes the counters measured, at this run's launch time
                     "measured_GBps": (traffic / (kern[dom]["avg_ms"] * 1e-3) / 1e9
                                       if traffic else None),
                     "traffic_over_algorithmic": (traffic / kern[dom]["algorithmic_bytes_per_launch"]
                                                  if traffic else None)},
        "kernels": kern,
        "algorithmic_GBps_per_iteration": BYTES["iteration"] * n * iters / el / 1e9,
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    if not args.main_only:
        probe = hbm_probe(pcg, torch)
        mix = probe["kernel_a_mix" if dom == "fused_apply" else "kernel_b_mix"]["GBps"]
        line["roofline"]["probe_GBps"] = mix
        line["roofline"]["frac_of_probe"] = kern[dom]["achieved_GBps"] / mix
        line["hbm_probe"] = probe
        try:
            line["extras"] = extras(pcg, si, torch, m)
        except Exception as e:  # report, keep the main line
            line["extras_error"] = repr(e)
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle)")
            line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
