"""Serving form (tsvd_submit / tsvd_poll): problems submitted together are
admitted by their HBM footprint into a running batch that they join and
leave between iterations; every result must equal the same problem solved
alone (single-problem call), to the precision form's tolerance."""

import time

import numpy as np
import pytest

import paper_1407_1785_amd as lib
import workloads
from tests.gpu_util import announce, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

ITERS = 15


def _mix(torch):
    rng = np.random.default_rng(2024)
    probs, alone = [], []
    for k in range(10):
        n1, n2, n3 = int(rng.integers(8, 60)), int(rng.integers(8, 60)), int(rng.integers(2, 20))
        fp32 = k % 3 == 0
        dt = torch.float32 if fp32 else torch.float64
        prec = lib.PREC_FP32 if fp32 else lib.PREC_FP64
        if k % 4 == 3:
            r = workloads.trpca_problem(k, shape=(n1, n2, n3), rank=2)
            x = to_gpu(torch, r["M"], dt)
            probs.append(lib.trpca_problem(x, r["lam"], 1e-3, 0.0, max_iter=ITERS))
            L, S, _ = lib.trpca(x, r["lam"], 1e-3, 0.0, max_iter=ITERS, precision=prec)
            alone.append([L.cpu().numpy(), S.cpu().numpy()])
        else:
            _, _, xt = workloads.lowrank(rng, n1, n2, n3, 2)
            mask = (rng.random((n1, n2, n3)) < 0.5).astype(np.uint8)
            y = to_gpu(torch, xt * mask, dt)
            m = to_gpu(torch, mask)
            probs.append(lib.complete_problem(y, m, 1e-2, 0.0, max_iter=ITERS))
            xs, _ = lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=ITERS, precision=prec)
            alone.append([xs.cpu().numpy()])
    return probs, alone


def _wait(tickets, handle, limit_s=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = lib.poll(t, handle)
                if r is not None:
                    done[t] = r
        assert time.time() - t0 < limit_s, "serving did not finish in time"
        time.sleep(0.001)
    return done


def test_served_results_equal_alone():
    torch = torch_cuda()
    probs, alone = _mix(torch)
    # a budget that holds only a few problems at once: the rest wait for space
    handle = lib.Handle(0, hbm_budget_bytes=24 << 20)
    try:
        announce("serve mix", len(probs))
        tickets = [lib.submit(p, handle) for p in probs]
        done = _wait(tickets, handle)
        stats = lib.serve_stats(handle)
    finally:
        handle.close()
    for t, p, want in zip(tickets, probs, alone):
        st, info = done[t]
        assert st == 0 and info.iters == ITERS
        bar = 1e-5 if p.x.dtype == torch.float32 else 1e-12
        got = [p.out.cpu().numpy()] + ([p.out_s.cpu().numpy()] if p.out_s is not None else [])
        for g, w in zip(got, want):
            assert rel_fro(g, w) <= bar
    assert stats["submitted"] == stats["finished"] == len(probs)
    assert stats["peak_running"] >= 2            # work overlapped on the device
    assert stats["arena_bytes"] == 24 << 20


def test_poll_unknown_ticket_and_late_submissions():
    torch = torch_cuda()
    handle = lib.Handle(0, hbm_budget_bytes=16 << 20)
    try:
        with pytest.raises(lib.TsvdError):
            lib.poll(12345, handle)
        rng = np.random.default_rng(5)
        tickets, probs = [], []
        for k in range(4):   # arrivals while earlier problems run
            _, _, xt = workloads.lowrank(rng, 20, 24, 6, 2)
            mask = (rng.random((20, 24, 6)) < 0.5).astype(np.uint8)
            p = lib.complete_problem(to_gpu(torch, xt * mask), to_gpu(torch, mask), 1e-2, 0.0, max_iter=30)
            probs.append(p)
            tickets.append(lib.submit(p, handle))
            time.sleep(0.002)
        done = _wait(tickets, handle)
        assert all(done[t][0] == 0 and done[t][1].iters == 30 for t in tickets)
        assert lib.poll(tickets[0], handle)[0] == 0   # a finished ticket can be polled again
    finally:
        handle.close()


def test_problem_larger_than_arena_is_refused():
    torch = torch_cuda()
    handle = lib.Handle(0, hbm_budget_bytes=1 << 20)
    try:
        x = torch.zeros((64, 64, 32), dtype=torch.float64, device="cuda")
        m = torch.ones((64, 64, 32), dtype=torch.uint8, device="cuda")
        with pytest.raises(lib.TsvdError) as e:
            lib.submit(lib.complete_problem(x, m), handle)
        assert e.value.status == -3
    finally:
        handle.close()


def _small_problem(torch, seed, iters=400, shape=(40, 44, 12), **kw):
    rng = np.random.default_rng(seed)
    _, _, xt = workloads.lowrank(rng, *shape, 2)
    mask = (rng.random(shape) < 0.5).astype(np.uint8)
    return lib.complete_problem(to_gpu(torch, xt * mask), to_gpu(torch, mask), 1e-2, 0.0, max_iter=iters, **kw)


def test_cancel_queued_and_running(monkeypatch):
    """A running request cancelled from the host leaves the batch at the next
    period boundary with TSVD_E_CANCELLED; a queued one never starts; the
    others finish normally, and cancelling a finished ticket changes
    nothing."""
    torch = torch_cuda()
    probs = [_small_problem(torch, 60 + k) for k in range(3)]
    # admission stops at 7 running Fourier slices, one problem's worth: the
    # second and third wait in the queue
    monkeypatch.setenv("TSVD_SERVE_SLICES", "7")
    handle = lib.Handle(0, hbm_budget_bytes=64 << 20)
    try:
        announce("serve cancel")
        tickets = [lib.submit(p, handle) for p in probs]
        lib.cancel(tickets[2], handle)           # queued
        time.sleep(0.05)
        lib.cancel(tickets[0], handle)           # running (400 iterations take longer)
        done = _wait(tickets, handle)
        assert done[tickets[0]][0] == lib.E_CANCELLED
        assert done[tickets[2]][0] == lib.E_CANCELLED
        assert done[tickets[1]][0] == 0 and done[tickets[1]][1].iters == 400
        lib.cancel(tickets[1], handle)
        assert lib.poll(tickets[1], handle)[0] == 0
        with pytest.raises(lib.TsvdError):
            lib.cancel(987654, handle)
        t0 = time.time()
        while lib.serve_stats(handle)["running"] and time.time() - t0 < 5.0:
            time.sleep(0.01)
        stats = lib.serve_stats(handle)
        assert stats["finished"] == 3 and stats["running"] == 0 and stats["queued"] == 0
    finally:
        handle.close()


def test_deadline_stops_a_request():
    """A request whose deadline passes stops with TSVD_E_TIMEOUT (the worker
    checks deadlines between periods); one without a deadline beside it
    finishes."""
    torch = torch_cuda()
    late = _small_problem(torch, 70, iters=100000, deadline_s=0.2)
    ok = _small_problem(torch, 71, iters=20)
    handle = lib.Handle(0, hbm_budget_bytes=64 << 20)
    try:
        announce("serve deadline")
        t_late = lib.submit(late, handle)
        t_ok = lib.submit(ok, handle)
        done = _wait([t_late, t_ok], handle)
        assert done[t_ok][0] == 0 and done[t_ok][1].iters == 20
        st, info = done[t_late]
        assert st == lib.E_TIMEOUT and info.seconds >= 0.2
    finally:
        handle.close()
