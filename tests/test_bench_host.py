"""Host-only checks of bench.py's bookkeeping: the algorithmic bytes it
divides by (counted vector by vector from what each kernel launch reads and
writes), the kernel instance it names for the launch shape, the guard that
ties committed traffic summaries to the kernel sources, the one-GPU rule
and the rocprofv3 summary on a synthetic trace."""
import contextlib
import csv
import io
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N = 512 * 512 * 128


def test_algorithmic_bytes_per_solve():
    # kernel A, 5 launches: z in / q out (16 B), then p, q, z in / u, p, q
    # out (48 B: u is zero and not read), then 4 in / 3 out (56 B) x 3
    assert bench.solve_kernel_bytes("fused_apply", 5, N) == N * (2 + 6 + 7 * 3) * 8
    # kernel B, 6 launches: b in / z out (16 B), then r, q in / r, z out x 5
    assert bench.solve_kernel_bytes("fused_prec", 5, N) == N * (2 + 4 * 5) * 8
    assert bench.solve_kernel_bytes("fused_apply", 1, N) == N * 2 * 8
    assert bench.BYTES["iteration"] == bench.BYTES["fused_apply"] + bench.BYTES["fused_prec"]


def test_kernel_symbol_for_launch_shapes():
    assert (bench.kernel_symbol("fused_apply", 64, N, 128)
            == "k_fused_apply<double, 2, true, false, true, true>")
    # FP32 at 32 lanes: 4 levels per lane = 16 bytes, streamed
    assert (bench.kernel_symbol("fused_prec", 32, 1024 * 1024 * 128, 128, elem=4)
            == "k_fused_prec<float, 4, true, false, true, false, false>")
    # kernel B stores z cached when the z vector takes at most 384 MiB
    assert (bench.kernel_symbol("fused_prec", 64, N, 128)
            == "k_fused_prec<double, 2, true, false, true, true, true>")
    # small vectors stay in the caches; a ragged column has no vector path
    assert (bench.kernel_symbol("fused_apply", 8, 64 * 64 * 33, 33)
            == "k_fused_apply<double, 8, false, false, false, false>")


def test_traffic_summaries_tied_to_sources():
    sym = "k_fused_apply<double, 2, true, false, true, true>"
    t = bench.measured_traffic("fused_apply", "512x512x128", sym)
    path = os.path.join(ROOT, "profiles", "traffic_fused_apply_512x512x128.txt")
    recorded = [ln.split("=")[1].strip() for ln in open(path)
                if ln.startswith("kernel_source_sha256_16")][0]
    if recorded == bench.kernel_source_hash():
        assert t is not None and t > 0
    else:
        assert t is None
    assert bench.measured_traffic("fused_apply", "512x512x128", sym.replace("2,", "4,")) is None


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_rocprof_summary_of_a_synthetic_trace(tmp_path):
    d = tmp_path / "prof"
    d.mkdir()
    name = "void pcg::k_fused_apply<double, 2, true, false, true, true>(pcg::ColArgs)"
    with open(d / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for start, dur in ((0, 300000), (1000000, 310000), (2000000, 5000)):
            w.writerow({"Kernel_Name": name, "Start_Timestamp": start,
                        "End_Timestamp": start + dur})
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        bench.summarize_rocprof(str(d), kernel_filter="k_fused")
    out = buf.getvalue()
    row = [ln for ln in out.splitlines() if ln.startswith(name)][0].split(" | ")
    # 3 dispatches averaging 205 us; the 5 us early-exit one is not working
    assert row[1] == "3" and abs(float(row[2]) - 205.0) < 1e-6
    assert row[3] == "2" and abs(float(row[4]) - 305.0) < 1e-6


def test_whole_solve_bytes_by_enumeration():
    """The whole-solve byte counts against a launch-by-launch enumeration
    (bytes per unknown of each vector each launch reads or writes)."""
    n = 1000

    def inner(k, e, fixup=True):   # a zero-start solve of k iterations, e bytes per value
        b = [2 * e] + [4 * e] * k                       # kernel B: b -> z, then r, q -> r, z
        a = [2 * e] + ([6 * e] if k >= 2 else []) + [7 * e] * max(k - 2, 0)
        fix = 3 * e if k >= 2 else 2 * e                # u += alpha p (u unset after one)
        return sum(b) + sum(a) + (fix if fixup else 0)

    for k in (1, 2, 5, 9):
        assert bench.fp64_solve_bytes(k, n) == n * inner(k, 8)
    for ks in ((11,), (7, 4), (9, 2, 3)):
        s = len(ks)
        residuals = (8 + 4) + (8 + 8 + 4) * s           # b [, x] in, r32 out; s + 1 of them
        updates = (4 + 4 + 8) + (8 + 4 + 4 + 8) * (s - 1)   # u32, p32 [, x] in, x out
        want = sum(inner(k, 4, fixup=False) for k in ks) + residuals + updates
        assert bench.mixed_solve_bytes(sum(ks), s, n) == n * want, ks


def test_launch_positions_of_a_synthetic_trace():
    """Kernel A's and B's launches are labelled by their position within
    each solve (reset at the exit correction and the refinement kernels);
    early-exit launches are left out."""
    A = "void pcg::k_fused_apply<float, 4, true, false, true, false>(pcg::ColArgs)"
    B = "void pcg::k_fused_prec<float, 4, true, false, true, false>(pcg::ColArgs)"
    F = "void pcg::k_fixup<float, 4, true, true>(pcg::ColArgs)"
    R = "void pcg::k_residual64<4, true, false>(pcg::ColArgs)"
    seq = [(R, 100), (B, 60), (A, 50), (B, 90), (A, 80), (B, 90), (A, 100), (B, 90),
           (A, 2), (B, 1), (F, 40), (R, 100), (B, 61), (A, 51), (B, 91), (A, 2), (F, 30)]
    rows = [dict(Kernel_Name=n, us=float(v)) for n, v in seq]
    got = bench.classify_launches(rows, "us")
    labels = [(n[:20], c, v) for n, c, v in got if n in (A, B)]
    assert labels == [(B[:20], "first", 60), (A[:20], "first", 50), (B[:20], "steady", 90),
                      (A[:20], "second", 80), (B[:20], "steady", 90), (A[:20], "steady", 100),
                      (B[:20], "steady", 90), (B[:20], "first", 61), (A[:20], "first", 51),
                      (B[:20], "steady", 91)]
