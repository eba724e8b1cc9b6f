"""Serving runtime on the GPU, through the C ABI, with per-request workers and
in batched mode (shared multi-request launches): results identical alone and
in a concurrent mix of different grids (line, multigrid, block Gauss-Seidel
and automatically chosen preconditioners; and identical to a direct solve),
admission by HBM budget, rejection of requests that can never fit,
cancellation of queued requests.  Accuracy of every served result is checked
with the oracle's assembled matrix."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1302_7193_amd as pcg  # noqa: E402
import synth_inputs as si  # noqa: E402

SHAPES = [(32, 32, 32, 1e2), (48, 40, 64, 1e4), (16, 16, 128, 1e5), (64, 64, 32, 3e3),
          (24, 20, 100, 1e3), (40, 40, 16, 1e2), (20, 36, 64, 5e4), (32, 32, 32, 1e2)]


def requests(precision=pcg.PCG_PREC_MIXED, preconditioner=pcg.PCG_PRECOND_LINE):
    out = []
    for rid, (nx, ny, nz, g2) in enumerate(SHAPES):
        d = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, g2, pcg.PCG_BC_DIRICHLET)
        b = si.rhs_uniform(nx, ny, nz, 1000 + rid)
        out.append((d, b))
    return out, pcg.pcg_default_opts(precision=precision, preconditioner=preconditioner)


def serve(reqs, opts, max_active, budget=None, one_at_a_time=False, batched=False):
    need = max(pcg.pcg_request_bytes(d, opts) for d, _ in reqs)
    arena = torch.empty(sum(pcg.pcg_request_bytes(d, opts) for d, _ in reqs) + (1 << 20),
                        dtype=torch.uint8, device="cuda")
    srv = pcg.Server(arena, budget or arena.numel(), max_active, batched=batched)
    xs, res = [None] * len(reqs), [None] * len(reqs)
    try:
        if one_at_a_time:
            for i, (d, b) in enumerate(reqs):
                xs[i] = np.zeros_like(b)
                t = pcg.pcg_submit(srv, d, b, xs[i], opts)
                st, res[i] = pcg.pcg_wait(srv, t)
                assert st == pcg.PCG_OK, res[i]
        else:
            tickets = []
            for i, (d, b) in enumerate(reqs):
                xs[i] = np.zeros_like(b)
                tickets.append(pcg.pcg_submit(srv, d, b, xs[i], opts))
            pending = set(range(len(reqs)))
            deadline = time.time() + 120
            while pending and time.time() < deadline:
                for i in list(pending):
                    st, r = pcg.pcg_poll(srv, tickets[i])
                    if st != pcg.PCG_E_AGAIN:
                        assert st == pcg.PCG_OK, r
                        res[i] = r
                        pending.discard(i)
                time.sleep(0.001)
            assert not pending
        stats = pcg.pcg_server_query(srv)
    finally:
        srv.close()
    return xs, res, stats, need


@pytest.mark.parametrize("precision,preconditioner", [
    (pcg.PCG_PREC_MIXED, pcg.PCG_PRECOND_LINE), (pcg.PCG_PREC_FP64, pcg.PCG_PRECOND_LINE),
    (pcg.PCG_PREC_FP64, pcg.PCG_PRECOND_MG), (pcg.PCG_PREC_MIXED, pcg.PCG_PRECOND_RBGS),
    (pcg.PCG_PREC_FP64, pcg.PCG_PRECOND_AUTO)])
def test_results_identical_alone_and_in_the_mix(precision, preconditioner):
    reqs, opts = requests(precision, preconditioner)
    alone, ra, _, _ = serve(reqs, opts, max_active=1, one_at_a_time=True)
    mixed, rm, stats, _ = serve(reqs, opts, max_active=4)
    assert stats["completed"] == len(reqs) and stats["peak_bytes_in_use"] > 0
    print("peak requests on the device at once: %d" % stats["peak_active"])
    for i, (d, b) in enumerate(reqs):
        np.testing.assert_array_equal(alone[i], mixed[i])
        assert ra[i]["iterations"] == rm[i]["iterations"]
        g = oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                        False, False)
        A = oracle.assemble(g)
        true = oracle.residual_norm(A, b, mixed[i]) / np.linalg.norm(b)
        assert true < 1.05e-8, (i, true)
        assert rm[i]["elapsed_ms"] > 0


def test_served_result_equals_direct_solve():
    reqs, opts = requests()
    d, b = reqs[1]
    xs, _, _, _ = serve([reqs[1]], opts, max_active=2)
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, x0_zero=1)
    bt = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bt)
    st, r = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert st == pcg.PCG_OK
    np.testing.assert_array_equal(x.cpu().numpy(), xs[0])


def test_admission_by_budget():
    reqs, opts = requests()
    need = max(pcg.pcg_request_bytes(d, opts) for d, _ in reqs)
    xs, res, stats, _ = serve(reqs, opts, max_active=4, budget=need)
    assert stats["completed"] == len(reqs)
    assert stats["peak_bytes_in_use"] <= need        # at most what fits in the budget at once


def test_oversize_request_rejected_and_cancel_queued():
    reqs, opts = requests()
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    small = min(pcg.pcg_request_bytes(d, opts) for d, _ in reqs)
    srv = pcg.Server(arena, small, max_active=1)
    try:
        big = pcg.pcg_desc_from_ratio(256, 256, 64, 1.05, 1e3, pcg.PCG_BC_DIRICHLET)
        bb = np.zeros(256 * 256 * 64)
        with pytest.raises(pcg.PCGError) as e:
            pcg.pcg_submit(srv, big, bb, np.zeros_like(bb), opts)
        assert e.value.status == pcg.PCG_E_NOMEM
        # one worker: the second of two requests queues behind the first
        d0, b0 = min(reqs, key=lambda r: pcg.pcg_request_bytes(r[0], opts))
        x0, x1 = np.zeros_like(b0), np.zeros_like(b0)
        t0 = pcg.pcg_submit(srv, d0, b0, x0, opts)
        t1 = pcg.pcg_submit(srv, d0, b0, x1, opts)
        c = pcg.pcg_cancel(srv, t1)
        assert c in (pcg.PCG_OK, pcg.PCG_E_AGAIN)
        st, r = pcg.pcg_wait(srv, t0)
        assert st == pcg.PCG_OK
        st1, _ = pcg.pcg_wait(srv, t1)
        assert st1 == (pcg.PCG_E_CANCELLED if c == pcg.PCG_OK else pcg.PCG_OK)
        stats = pcg.pcg_server_query(srv)
        assert stats["rejected"] == 1 and stats["queued"] == 0 and stats["active"] == 0
    finally:
        srv.close()


def test_device_resident_requests_equal_host_requests():
    reqs, opts = requests()
    host, _, _, _ = serve(reqs[:4], opts, max_active=3)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    srv = pcg.Server(arena, arena.numel(), 3)
    try:
        outs, tickets = [], []
        for d, b in reqs[:4]:
            bt = torch.from_numpy(b).cuda()
            xt = torch.full_like(bt, float("nan"))
            outs.append(xt)
            tickets.append(pcg.pcg_submit_device(srv, d, bt, xt, opts))
        for t in tickets:
            st, r = pcg.pcg_wait(srv, t)
            assert st == pcg.PCG_OK
        for i in range(4):
            np.testing.assert_array_equal(outs[i].cpu().numpy(), host[i])
    finally:
        srv.close()


def test_device_generator_matches_host_generator():
    for seed, n, start in ((1, 1 << 20, 0), (1000 + 17, 33333, 777), (2**40 + 3, 4096, 1 << 33)):
        a = si.uniform_pm1(seed, n, start)
        b = si.uniform_pm1_torch(seed, n, start, device="cuda").cpu().numpy()
        np.testing.assert_array_equal(a, b)
    a = si.rhs_smooth_noise(17, 9, 33, 2)
    b = si.rhs_smooth_noise_torch(17, 9, 33, 2).cpu().numpy()
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_requests_overlap_on_the_device():
    """Requests submitted together run concurrently: the server's count of
    requests running at once reaches the number of workers, and each result
    is still the one the request gets alone."""
    reqs = []
    for rid in range(4):
        d = pcg.pcg_desc_from_ratio(128, 128, 64, 1.05, 1e2, pcg.PCG_BC_DIRICHLET)
        reqs.append((d, si.rhs_uniform(128, 128, 64, 1000 + rid)))
    opts = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED)
    mixed, rm, stats, _ = serve(reqs, opts, max_active=4)
    print("peak requests on the device at once: %d" % stats["peak_active"])
    assert stats["peak_active"] >= 2, stats
    alone, ra, _, _ = serve(reqs[:1], opts, max_active=1, one_at_a_time=True)
    np.testing.assert_array_equal(alone[0], mixed[0])


def test_zero_right_hand_side_served_as_zero():
    """A served request with b = 0 (done at its first residual) returns
    x = 0, also when the host buffer held garbage."""
    reqs, opts = requests()
    d, b = reqs[0]
    z = np.zeros_like(b)
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    srv = pcg.Server(arena, arena.numel(), 2)
    try:
        x = np.full_like(b, np.nan)
        st, r = pcg.pcg_wait(srv, pcg.pcg_submit(srv, d, z, x, opts))
        assert st == pcg.PCG_OK and r["iterations"] == 0
        assert np.array_equal(x, z)
        bt = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        xt = torch.full_like(bt, float("nan"))
        st, r = pcg.pcg_wait(srv, pcg.pcg_submit_device(srv, d, bt, xt, opts))
        assert st == pcg.PCG_OK and not xt.cpu().numpy().any()
    finally:
        srv.close()


# ------------------------------------------------------------ batched mode --

BATCH_SHAPES = [(32, 32, 32, 1e2), (48, 40, 64, 1e4), (16, 16, 128, 1e5), (64, 64, 32, 3e3),
                (24, 20, 128, 1e3), (40, 40, 16, 1e2), (20, 36, 64, 5e4), (32, 32, 32, 1e2),
                (96, 64, 64, 2e2), (8, 8, 8, 1e3)]


def batch_requests(precision):
    out = []
    for rid, (nx, ny, nz, g2) in enumerate(BATCH_SHAPES):
        d = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, g2, pcg.PCG_BC_DIRICHLET)
        out.append((d, si.rhs_uniform(nx, ny, nz, 1000 + rid)))
    return out, pcg.pcg_default_opts(precision=precision)


@pytest.mark.parametrize("precision", [pcg.PCG_PREC_MIXED, pcg.PCG_PREC_FP64])
def test_batched_results_identical_alone_and_in_the_mix(precision):
    """Batched mode: every request's result is bitwise the same served alone
    and sharing launches with nine others (different grids and
    anisotropies, requests joining and leaving between ticks), and within
    the tolerance by the oracle's assembled matrix."""
    reqs, opts = batch_requests(precision)
    print("batched", precision, flush=True)
    alone, ra, _, _ = serve(reqs, opts, max_active=1, one_at_a_time=True, batched=True)
    mixed, rm, stats, _ = serve(reqs, opts, max_active=8, batched=True)
    print("batched: peak requests sharing launches %d" % stats["peak_active"])
    assert stats["completed"] == len(reqs) and stats["peak_active"] >= 2
    for i, (d, b) in enumerate(reqs):
        np.testing.assert_array_equal(alone[i], mixed[i])
        assert ra[i]["iterations"] == rm[i]["iterations"]
        g = oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                        False, False)
        A = oracle.assemble(g)
        true = oracle.residual_norm(A, b, mixed[i]) / np.linalg.norm(b)
        assert true < 1.05e-8, (i, true)


def test_batched_device_io_zero_rhs_and_rejections():
    """Batched mode with device-resident b and x equals host requests; a
    zero right-hand side gives x = 0; grids and preconditioners the
    multi-request kernels do not cover are rejected at submission."""
    reqs, opts = batch_requests(pcg.PCG_PREC_MIXED)
    host, _, _, _ = serve(reqs[:4], opts, max_active=4, batched=True)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    srv = pcg.Server(arena, arena.numel(), 4, batched=True)
    try:
        outs, tickets = [], []
        for d, b in reqs[:4]:
            bt = torch.from_numpy(b).cuda()
            xt = torch.full_like(bt, float("nan"))
            outs.append(xt)
            tickets.append(pcg.pcg_submit_device(srv, d, bt, xt, opts))
        z = torch.zeros(reqs[0][1].size, dtype=torch.float64, device="cuda")
        xz = torch.full_like(z, float("nan"))
        tickets.append(pcg.pcg_submit_device(srv, reqs[0][0], z, xz, opts))
        for t in tickets:
            st, r = pcg.pcg_wait(srv, t)
            assert st == pcg.PCG_OK, r
        for i in range(4):
            np.testing.assert_array_equal(outs[i].cpu().numpy(), host[i])
        assert not xz.cpu().numpy().any()
        bad = pcg.pcg_desc_from_ratio(16, 16, 100, 1.05, 1e3, pcg.PCG_BC_DIRICHLET)
        bb = np.zeros(16 * 16 * 100)
        with pytest.raises(pcg.PCGError) as e:
            pcg.pcg_submit(srv, bad, bb, np.zeros_like(bb), opts)
        assert e.value.status == pcg.PCG_E_INVALID
        mg = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, preconditioner=pcg.PCG_PRECOND_MG)
        d0, b0 = reqs[0]
        with pytest.raises(pcg.PCGError):
            pcg.pcg_submit(srv, d0, b0, np.zeros_like(b0), mg)
    finally:
        srv.close()
