"""Batched form (tsvd_batch_run): completion and tensor-RPCA problems of
uneven shapes solved together with problem-table launches, against the FP64
oracle and against the single-problem calls; HIP-graph replay against eager
launches."""

import os

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import admm
import workloads
from tests.gpu_util import announce, assert_close_fp32, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

ITERS = 12
FP64_BAR = 1e-10
FP32_BAR = 1e-4


def _completion(shape, seed, p=0.5, rank=2):
    rng = np.random.default_rng(seed)
    if len(shape) == 3:
        _, _, x = workloads.lowrank(rng, *shape, rank)
    else:
        x = rng.normal(size=shape)
    mask = (rng.random(shape) < p).astype(np.uint8)
    return x * mask, mask


def _cases():
    """(name, kind, data, mask, dtype, extra) -- shapes cover one and several
    Jacobi blocks, n1 < n2, 4-D, n3 = 1, two columns, odd and even tubes."""
    out = []
    for name, shape in [("c32", (32, 32, 16)), ("c_ragged", (24, 17, 9)), ("c_trans", (13, 40, 6)),
                        ("c_4d", (15, 26, 4, 3)), ("c_blocks", (70, 45, 5)), ("c_matrix", (30, 20, 1)),
                        ("c_two_cols", (8, 2, 5))]:
        y, m = _completion(shape, len(out) + 3)
        out.append((name, "complete", y, m, np.float64, {}))
    y, m = _completion((40, 50, 12), 99)
    out.append(("c_fp32", "complete", y.astype(np.float32), m, np.float32, {}))
    r = workloads.trpca_problem(0, shape=(20, 24, 10), rank=2)
    out.append(("r_l1", "trpca", r["M"], None, np.float64, dict(lam=r["lam"], shrink="l1")))
    t = workloads.tube_corruption(0, shape=(20, 24, 10), rank=2)
    out.append(("r_l112", "trpca", t["M"], None, np.float64, dict(lam=t["lam"], shrink="l112")))
    return out


def _problem(torch, case, iters=ITERS, tol=0.0):
    name, kind, x, mask, dt, extra = case
    tdt = torch.float32 if dt == np.float32 else torch.float64
    xg = to_gpu(torch, x, tdt)
    if kind == "complete":
        return lib.complete_problem(xg, to_gpu(torch, mask), rho=1e-2, tol=tol, max_iter=iters)
    shrink = lib.SHRINK_L1 if extra["shrink"] == "l1" else lib.SHRINK_L112
    return lib.trpca_problem(xg, extra["lam"], mu=1e-3, tol=tol, shrink=shrink, max_iter=iters)


def _oracle(case, iters=ITERS):
    name, kind, x, mask, dt, extra = case
    x64 = np.asarray(x, dtype=np.float64)
    if kind == "complete":
        return [admm.complete(x64, mask, 1e-2, 1.1, 1e3, max_iter=iters, tol=0.0)["X"]]
    r = admm.trpca(x64, extra["lam"], 1e-3, 1.2, 1e10, max_iter=iters, tol=0.0, shrink=extra["shrink"])
    return [r["L"], r["S"]]


def _outputs(p):
    return [p.out.cpu().numpy()] + ([p.out_s.cpu().numpy()] if p.out_s is not None else [])


@pytest.fixture(scope="module")
def batch_result():
    torch = torch_cuda()
    cases = _cases()
    probs = [_problem(torch, c) for c in cases]
    announce("batch run", len(probs), "problems")
    res = lib.batch_run(probs)
    return cases, probs, res


def test_batch_matches_oracle(batch_result):
    cases, probs, res = batch_result
    for case, p, (st, info) in zip(cases, probs, res):
        assert st == 0, case[0]
        assert info.iters == ITERS and info.converged == 0, case[0]
        assert info.sweeps_total >= ITERS and info.sweeps_last >= 1, case[0]
        for got, want in zip(_outputs(p), _oracle(case)):
            if case[4] == np.float32:
                assert_close_fp32(got, want, FP32_BAR, case[0])
            else:
                err = rel_fro(got, want)
                assert err <= FP64_BAR, (case[0], err)


def test_batch_matches_single_calls(batch_result):
    torch = torch_cuda()
    cases, probs, res = batch_result
    for case, p in zip(cases, probs):
        name, kind, x, mask, dt, extra = case
        tdt = torch.float32 if dt == np.float32 else torch.float64
        xg = to_gpu(torch, x, tdt)
        prec = lib.PREC_FP32 if dt == np.float32 else lib.PREC_FP64
        announce("single call", name)
        if kind == "complete":
            xs, _ = lib.tsvd_complete(xg, to_gpu(torch, mask), 1e-2, 0.0, max_iter=ITERS, precision=prec)
            single = [xs.cpu().numpy()]
        else:
            shrink = lib.SHRINK_L1 if extra["shrink"] == "l1" else lib.SHRINK_L112
            L, S, _ = lib.trpca(xg, extra["lam"], 1e-3, 0.0, shrink=shrink, max_iter=ITERS, precision=prec)
            single = [L.cpu().numpy(), S.cpu().numpy()]
        bar = 1e-5 if dt == np.float32 else 1e-12
        for got, want in zip(_outputs(p), single):
            assert rel_fro(got, want) <= bar, name


def test_observed_entries_kept_exactly(batch_result):
    cases, probs, res = batch_result
    for case, p in zip(cases, probs):
        if case[1] != "complete":
            continue
        omega = case[3].astype(bool)
        got = p.out.cpu().numpy()
        np.testing.assert_array_equal(got[omega], np.asarray(case[2])[omega])


def test_graph_replay_equals_eager():
    """Every replay of the captured two-iteration period must give the eager
    result bit for bit (20 iterations = 10 replays, with host reads of the
    control blocks between them).  The mix holds both Jacobi schedules (one
    workgroup per slice, and one per block pair with the blocks exchanged
    inside the launch), so every running set is captured."""
    torch = torch_cuda()
    cases = _cases()[:5] + _cases()[-2:] + [("big", "complete", *_completion((150, 140, 4), 7, p=0.4, rank=3),
                                            np.float64, {})]
    outs = {}
    for mode in ("1", "0"):
        os.environ["TSVD_GRAPH"] = mode
        try:
            probs = [_problem(torch, c, iters=20) for c in cases]
            announce("graph mode", mode)
            res = lib.batch_run(probs)
        finally:
            os.environ.pop("TSVD_GRAPH", None)
        assert all(st == 0 for st, _ in res)
        outs[mode] = [_outputs(p) for p in probs]
    for a, b in zip(outs["1"], outs["0"]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_problems_stop_at_their_own_iteration():
    """With tol > 0 problems converge at different iterations; each stops
    where its single call stops and keeps its output from then on."""
    torch = torch_cuda()
    w = workloads.completion_small(0)
    cases = [("c_small", "complete", w["M_obs"], w["mask"], np.float64, {})] + _cases()[1:4]
    probs = [_problem(torch, c, iters=300, tol=1e-6) for c in cases]
    announce("batch convergence")
    res = lib.batch_run(probs)
    for case, p, (st, info) in zip(cases, probs, res):
        name, kind, x, mask, dt, extra = case
        xs, si = lib.tsvd_complete(to_gpu(torch, x), to_gpu(torch, mask), 1e-2, 1e-6, max_iter=300)
        assert st == 0
        assert info.converged == si.converged, name
        assert abs(info.iters - si.iters) <= 1, (name, info.iters, si.iters)
        if info.iters == si.iters:
            assert rel_fro(p.out.cpu().numpy(), xs.cpu().numpy()) <= 1e-10, name


def test_batch_rejects_bad_records():
    torch = torch_cuda()
    y, m = _completion((10, 10, 4), 1)
    p = lib.complete_problem(to_gpu(torch, y), to_gpu(torch, m))
    p.record.penalty = -1.0
    with pytest.raises(lib.TsvdError) as e:
        lib.batch_run([p])
    assert e.value.status == -1
    q = lib.complete_problem(to_gpu(torch, y), to_gpu(torch, m))
    q.record.shape.ndim = 5
    with pytest.raises(lib.TsvdError) as e:
        lib.batch_run([q])
    assert e.value.status == -2


def test_pairs_schedule_equals_slice_schedule():
    """The pairs-parallel Jacobi schedule (one workgroup per block pair, the
    blocks exchanged between rounds inside one launch) performs the same
    rotations in the same order as the one-workgroup-per-slice kernel:
    outputs agree bit for bit."""
    torch = torch_cuda()
    cases = _cases() + [("big", "complete", *_completion((150, 140, 4), 7, p=0.4, rank=3), np.float64, {})]
    outs = {}
    for mode in ("1", "100000"):
        os.environ["TSVD_PAIRS_MIN"] = mode
        try:
            probs = [_problem(torch, c) for c in cases]
            announce("pairs-schedule threshold", mode)
            res = lib.batch_run(probs)
        finally:
            os.environ.pop("TSVD_PAIRS_MIN", None)
        assert all(st == 0 for st, _ in res)
        outs[mode] = [_outputs(p) for p in probs]
    for a, b in zip(outs["1"], outs["100000"]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def _tune_lines(err, what):
    return [ln.split() for ln in err.splitlines() if ln.startswith(f"[tsvd tune] {what} m=101 n=93 ")]


def test_tuner_cache_file(tmp_path, monkeypatch, capfd):
    """TSVD_AUTOTUNE_CACHE: a schedule the tuner times is appended to the file
    as "arch cus elem_bytes rpt ncls slices bw pairs"; a file naming another
    admissible schedule for the same key is read and used without timing;
    both runs meet the oracle bar."""
    torch = torch_cuda()
    case = ("tune", "complete", *_completion((101, 93, 7), 31), np.float64, {})
    want = _oracle(case)[0]
    monkeypatch.setenv("TSVD_TUNE_LOG", "1")
    monkeypatch.delenv("TSVD_TUNE", raising=False)
    monkeypatch.delenv("TSVD_BATCH_BW", raising=False)
    monkeypatch.delenv("TSVD_PAIRS_MIN", raising=False)
    first = tmp_path / "tune_first.txt"
    monkeypatch.setenv("TSVD_AUTOTUNE_CACHE", str(first))
    capfd.readouterr()
    p = _problem(torch, case)
    announce("tuner cache: timed run")
    assert lib.batch_run([p])[0][0] == 0
    chose = _tune_lines(capfd.readouterr().err, "chose")
    assert len(chose) == 1, "the 101 x 93 slices were tuned before this test"
    bw, pairs = int(chose[0][-2].split("=")[1]), int(chose[0][-1].split("=")[1])
    lines = [ln.split() for ln in first.read_text().splitlines()]
    assert lines and all(len(ln) == 8 for ln in lines)
    assert [int(lines[-1][6]), int(lines[-1][7])] == [bw, pairs]
    assert int(lines[-1][2]) == 8 and int(lines[-1][5]) == 4   # FP64, 4 Fourier slices
    assert rel_fro(p.out.cpu().numpy(), want) <= FP64_BAR

    alt = (8, 1) if (bw, pairs) != (8, 1) else (16, 0)
    second = tmp_path / "tune_second.txt"
    second.write_text(" ".join(lines[-1][:6] + [str(alt[0]), str(alt[1])]) + "\n")
    monkeypatch.setenv("TSVD_AUTOTUNE_CACHE", str(second))
    q = _problem(torch, case)
    announce("tuner cache: cached run", alt)
    assert lib.batch_run([q])[0][0] == 0
    err = capfd.readouterr().err
    assert not _tune_lines(err, "chose")
    cached = _tune_lines(err, "cached")
    assert cached and cached[0][-2:] == [f"bw={alt[0]}", f"pairs={alt[1]}"]
    assert rel_fro(q.out.cpu().numpy(), want) <= FP64_BAR


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_large_slices_against_oracle(dt):
    """Slices with many column blocks (150 x 140, several block pairs per
    round) next to small ones, in one batch."""
    torch = torch_cuda()
    big = ("big", "complete", *_completion((150, 140, 4), 7, p=0.4, rank=3), dt, {})
    big = (big[0], big[1], np.asarray(big[2], dtype=dt), big[3], dt, {})
    small = _cases()[0]
    cases = [big, small]
    probs = [_problem(torch, c, iters=8) for c in cases]
    announce("large slices", dt.__name__)
    res = lib.batch_run(probs)
    bar = FP32_BAR if dt == np.float32 else FP64_BAR
    for case, p, (st, info) in zip(cases, probs, res):
        assert st == 0
        for got, want in zip(_outputs(p), _oracle(case, iters=8)):
            if dt == np.float32:
                assert_close_fp32(got, want, bar, case[0])
            else:
                assert rel_fro(got, want) <= bar, case[0]


WIDE_ITERS = 6


@pytest.fixture(scope="module")
def widest():
    """The widest Jacobi classes the 64-problem batch can draw: 320 x 300
    slices (tube length 37, a prime) and 288 x 320 slices (tube length 128),
    20 and 19 rows per lane in the one-workgroup-per-slice and round-mode
    kernels, next to a small problem; the oracle's first WIDE_ITERS
    iterations of each."""
    specs = [dict(n1=320, n2=300, n3=37, rank=9, p=0.3), dict(n1=288, n2=320, n3=128, rank=6, p=0.45),
             dict(n1=48, n2=50, n3=8, rank=2, p=0.5)]
    data = [workloads.batch_problem(sp, 900 + i, iters=WIDE_ITERS) for i, sp in enumerate(specs)]
    refs = [admm.complete(d["M_obs"], d["mask"], d["rho"], d["growth"], d["rho_max"], max_iter=WIDE_ITERS,
                          tol=0.0)["X"] for d in data]
    return data, refs


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_widest_classes_against_oracle(widest, dt):
    torch = torch_cuda()
    data, refs = widest
    tdt = torch.float32 if dt == np.float32 else torch.float64
    probs = [lib.complete_problem(to_gpu(torch, d["M_obs"], tdt), to_gpu(torch, d["mask"]), d["rho"], 0.0,
                                  d["growth"], d["rho_max"], WIDE_ITERS) for d in data]
    announce("widest classes", dt.__name__, [d["M_obs"].shape for d in data])
    res = lib.batch_run(probs)
    for d, p, ref, (st, info) in zip(data, probs, refs, res):
        assert st == 0 and info.iters == WIDE_ITERS
        got = p.out.cpu().numpy()
        if dt == np.float32:
            assert_close_fp32(got, ref, FP32_BAR, str(d["M_obs"].shape))
        else:
            assert rel_fro(got, ref) <= FP64_BAR, d["M_obs"].shape
