"""Pins of the oracle's completion ADMM (Sec. 4) and tensor-RPCA ADMM
(Sec. 5): optimality certificates that hold at every iteration, the
constraint, exact recovery of planted low-tubal-rank tensors and limit cases
(CPU only)."""

import numpy as np
import pytest

from oracle import admm, metrics, tensor as T
from oracle.tsvt import tsvt
import workloads


def nuclear_subgradient_gap(g_hat, z_hat, svtol=1e-9):
    """For G in d||.||_* at Zhat: G = U1 V1^H + R with ||R||_2 <= 1,
    U1^H R = 0 and R V1 = 0.  Returns (max |U1^H G V1 - I|, max ||R||_2,
    max |U1^H R|, max |R V1|) over the slices."""
    n_sl = z_hat.shape[2]
    worst = [0.0, 0.0, 0.0, 0.0]
    for k in range(n_sl):
        u, s, vh = np.linalg.svd(z_hat[:, :, k], full_matrices=False)
        r = int(np.count_nonzero(s > svtol * max(s.max(), 1.0)))
        u1, v1 = u[:, :r], np.conj(vh[:r].T)
        g = g_hat[:, :, k]
        core = np.conj(u1.T) @ g @ v1
        rem = g - u1 @ np.conj(v1.T)
        worst[0] = max(worst[0], np.abs(core - np.eye(r)).max() if r else 0.0)
        worst[1] = max(worst[1], np.linalg.norm(rem, 2))
        worst[2] = max(worst[2], np.abs(np.conj(u1.T) @ rem).max() if r else 0.0)
        worst[3] = max(worst[3], np.abs(rem @ v1).max() if r else 0.0)
    return worst


@pytest.fixture(scope="module")
def small():
    return workloads.completion_small(0)


def test_completion_constraint_exact_and_projection(small):
    w = small
    omega = w["mask"].astype(bool)
    r5 = admm.complete(w["M_obs"], w["mask"], max_iter=5, tol=0.0)
    r6 = admm.complete(w["M_obs"], w["mask"], max_iter=6, tol=0.0)
    np.testing.assert_array_equal(r6["X"][omega], w["X"][omega])
    # X is the closest point of the constraint set to Z - Q (Sec. 4 X-update):
    # moving it off the mask only increases the distance.
    target = r5["Z"] - r5["Q"]
    d0 = np.linalg.norm(r6["X"] - target)
    g = np.random.default_rng(0)
    for _ in range(20):
        e = g.normal(size=target.shape) * (~omega)
        assert np.linalg.norm(r6["X"] + 1e-3 * e - target) >= d0
    # values of the observation off the mask are ignored
    junk = w["M_obs"] + 100.0 * (~omega)
    r6j = admm.complete(junk, w["mask"], max_iter=6, tol=0.0)
    np.testing.assert_array_equal(r6j["X"], r6["X"])


@pytest.mark.parametrize("iters", [1, 7, 40])
def test_completion_dual_certificate_every_iteration(small, iters):
    """The Z-update is the prox of (1/rho) sum_k ||.||_* at Xhat + Qhat, so
    rho * (Q + X - Z') is a nuclear-norm subgradient at Zhat' slice by slice;
    after the rescale that is rho_next * Q.  Pins the dual sign, the
    threshold 1/rho and the rescale by rho_k / rho_{k+1}."""
    w = small
    r = admm.complete(w["M_obs"], w["mask"], max_iter=iters, tol=0.0)
    rho_next = min(1.1 * r["rho"], 1e3)
    gap = nuclear_subgradient_gap(T.fourier(rho_next * r["Q"]), T.fourier(r["Z"]))
    assert gap[0] < 1e-8 and gap[1] <= 1 + 1e-9 and gap[2] < 1e-8 and gap[3] < 1e-8, gap


def test_completion_exact_recovery_small(small):
    w = small
    r = admm.complete(w["M_obs"], w["mask"], w["rho"], w["growth"], w["rho_max"], w["max_iter"],
                      w["tol"], history=True)
    assert r["converged"] and r["iters"] < 300
    assert metrics.rse(r["X"], w["X"]) <= 1e-6
    np.testing.assert_array_equal(r["multirank"], np.full(9, 2))
    # KKT at the solution: off the mask the dual is Z_k - Z_{k+1}, bounded by
    # the last change residual
    omega = w["mask"].astype(bool)
    assert np.linalg.norm(r["Q"][~omega]) <= r["history"][-1][1] * (1 + 1e-9)
    assert np.linalg.norm(r["Q"][omega]) > 1e3 * np.linalg.norm(r["Q"][~omega])
    # stopping rule: the last residual pair is under tol * ||P_Omega M||
    assert max(r["history"][-1]) <= w["tol"] * np.linalg.norm(w["M_obs"])
    assert max(r["history"][-2]) > w["tol"] * np.linalg.norm(w["M_obs"])


def test_completion_full_mask_returns_data():
    w = workloads.completion_small(1, shape=(8, 6, 5), rank=2, p=1.0)
    r = admm.complete(w["M_obs"], w["mask"], max_iter=3, tol=0.0)
    np.testing.assert_array_equal(r["X"], w["X"])


def test_completion_n3_one_is_matrix_completion():
    """n3 = 1: matrix nuclear-norm completion; a rank-2 matrix from 60% of
    its entries is recovered."""
    g = np.random.default_rng(3)
    x = (g.normal(size=(60, 2)) @ g.normal(size=(2, 50)))[:, :, None]
    mask = (g.random(x.shape) < 0.6).astype(np.uint8)
    r = admm.complete(x * mask, mask, max_iter=400, tol=1e-10)
    assert metrics.rse(r["X"], x) < 1e-7
    assert r["multirank"][0] == 2


@pytest.fixture(scope="module")
def rpca_small():
    return workloads.trpca_problem(0, shape=(48, 48, 16), rank=3)


@pytest.mark.parametrize("iters", [22, 30, 45])
def test_trpca_sparse_certificate_every_iteration(rpca_small, iters):
    """The S-update is the prox of (lam/mu)||.||_1 at M - W - L', so
    -mu * W~ is in lam d||S'||_1; after the rescale -mu_next W is.
    Pins the dual sign, the threshold lam/mu and the rescale."""
    p = rpca_small
    r = admm.trpca(p["M"], p["lam"], max_iter=iters, tol=0.0)
    mu_next = min(1.2 * r["mu"], 1e10)
    g = -mu_next * r["W"]
    supp = r["S"] != 0
    assert supp.any()
    np.testing.assert_allclose(g[supp], p["lam"] * np.sign(r["S"][supp]), rtol=1e-9, atol=1e-12)
    assert np.abs(g[~supp]).max() <= p["lam"] * (1 + 1e-9)


def test_trpca_tube_certificate_every_iteration():
    """l1,1,2 (eq. sparse2): -mu_next W(i,j,:) = lam S(i,j,:)/||S(i,j,:)|| on
    non-zero tubes and ||mu_next W(i,j,:)|| <= lam elsewhere."""
    p = workloads.tube_corruption(0, shape=(20, 24, 10), rank=2)
    r = admm.trpca(p["M"], p["lam"], max_iter=12, tol=0.0, shrink="l112")
    mu_next = min(1.2 * r["mu"], 1e10)
    g = -mu_next * r["W"]
    norms = np.linalg.norm(r["S"], axis=2)
    on = norms > 0
    assert on.any() and (~on).any()
    np.testing.assert_allclose(g[on], p["lam"] * r["S"][on] / norms[on][:, None], rtol=1e-8,
                               atol=1e-12)
    assert np.linalg.norm(g[~on], axis=1).max() <= p["lam"] * (1 + 1e-9)


def test_trpca_exact_recovery_and_low_rank_certificate(rpca_small):
    p = rpca_small
    r = admm.trpca(p["M"], p["lam"], p["mu"], p["growth"], p["mu_max"], p["max_iter"], p["tol"])
    assert r["converged"]
    assert metrics.rse(r["L"], p["L"]) <= 1e-5
    assert metrics.support_f1(r["S"], p["S"], p["M"]) >= 0.99
    assert np.linalg.norm(r["L"] + r["S"] - p["M"]) <= 1e-6 * np.linalg.norm(p["M"])
    np.testing.assert_array_equal(r["multirank"], np.full(9, 3))
    # L-update optimality at the fixed point: -mu W in d sum_k ||Lhat_k||_*
    # (a converged run returns W before the rescale, so mu is the last one used)
    gap = nuclear_subgradient_gap(T.fourier(-r["mu"] * r["W"]), T.fourier(r["L"]))
    assert gap[0] < 1e-3 and gap[1] <= 1 + 1e-3, gap


def test_trpca_huge_lambda_gives_no_sparse_part(rpca_small):
    p = rpca_small
    r = admm.trpca(p["M"], 1e12, max_iter=200, tol=1e-9)
    assert np.abs(r["S"]).max() == 0.0
    assert metrics.rse(r["L"], p["M"]) < 1e-8


def test_trpca_l112_detects_corrupted_tubes():
    """Sec. 5 setting, synthetic: tube-sparse noise, lam = 1/sqrt(max(n1,n2))."""
    p = workloads.tube_corruption(0, shape=(30, 36, 20), rank=2, frac=0.05, block=10, amp=1.0)
    r = admm.trpca(p["M"], p["lam"], max_iter=500, tol=1e-8, shrink="l112")
    assert r["converged"]
    truth = np.linalg.norm(p["S"], axis=2) > 0
    found = np.linalg.norm(r["S"], axis=2) > 1e-3
    assert (truth & found).sum() == truth.sum()
    assert (found & ~truth).sum() == 0
    assert metrics.rse(r["L"], p["L"]) < 1e-2


@pytest.mark.parametrize("k", [20, 30, 45])
def test_trpca_l112_low_rank_certificate_every_iteration(k):
    """The L-update of iteration k + 1 is the prox of (1/mu) times the tubal
    nuclear norm at M - S_k - W_k, so mu (M - S_k - W_k - L_{k+1}) has every
    Fourier slice in the nuclear-norm subdifferential at L_{k+1}'s slice
    (U1 V1^H + R, ||R||_2 <= 1).  Runs of k and k + 1 iterations share their
    first k; pins the L-update's input, its threshold and the dual rescale
    under the tube shrink."""
    p = workloads.tube_corruption(0, shape=(20, 24, 10), rank=2)
    a = admm.trpca(p["M"], p["lam"], max_iter=k, tol=0.0, shrink="l112")
    b = admm.trpca(p["M"], p["lam"], max_iter=k + 1, tol=0.0, shrink="l112")
    mu = min(1.2 * a["mu"], 1e10)
    assert b["mu"] == mu
    assert b["multirank"].min() >= 1 and np.abs(a["S"]).max() > 0   # the check is not vacuous
    g = mu * (p["M"] - a["S"] - a["W"] - b["L"])
    gap = nuclear_subgradient_gap(T.fourier(g), T.fourier(b["L"]), svtol=1e-9)
    assert gap[0] < 1e-9 and gap[1] <= 1 + 1e-9 and gap[2] < 1e-9 and gap[3] < 1e-9, gap


def _tube_objective(lo, sp, lam, n3_weight):
    """sum_k ||Lhat_k||_* / n3_weight + lam * sum_ij ||S(i,j,:)||_2."""
    nuc = sum(np.linalg.svd(T.fourier(lo)[:, :, k], compute_uv=False).sum() for k in range(lo.shape[2]))
    return nuc / n3_weight + lam * np.linalg.norm(sp, axis=2).sum()


def test_trpca_l112_objective_reading():
    """The objective the tube-shrink ADMM minimises.  With the threshold 1/mu
    applied to the singular values of unnormalised DFT slices, the L-update
    is the prox of (1/mu) sum_k ||Lhat_k||_* / n3 in the Frobenius norm of
    the tensor (Parseval), so the fixed point minimises
    sum_k ||Lhat_k||_* / n3 + lam ||S||_{1,1,2} over L + S = M: no feasible
    perturbation (L + E, S - E) lowers it.  Read with the weight 1 on the
    Fourier-domain sum (Sec. 5's objective with this lam taken literally),
    the same point is not optimal: a perturbation along -L lowers it."""
    p = workloads.tube_corruption(0, shape=(16, 18, 8), rank=2, frac=0.05, block=4, amp=1.0)
    n3 = p["M"].shape[2]
    r = admm.trpca(p["M"], p["lam"], max_iter=2000, tol=1e-11, shrink="l112")
    assert r["converged"]
    lo, sp = r["L"], r["S"]
    f0 = _tube_objective(lo, sp, p["lam"], n3)
    g = np.random.default_rng(3)
    scale = 1e-4 * np.linalg.norm(p["M"])
    for _ in range(30):
        e = g.normal(size=lo.shape)
        e *= scale / np.linalg.norm(e)
        assert _tube_objective(lo + e, sp - e, p["lam"], n3) >= f0 * (1 - 1e-9)
    e = -1e-3 * lo
    assert _tube_objective(lo + e, sp - e, p["lam"], 1) < _tube_objective(lo, sp, p["lam"], 1)


def test_shrinks_closed_form():
    d = np.array([[[3.0, -0.5, 0.2, -2.0]]])
    np.testing.assert_allclose(admm.shrink_l1(d, 1.0), [[[2.0, 0.0, 0.0, -1.0]]])
    t = np.array([[[3.0, 4.0]], [[0.0, 0.0]]])
    np.testing.assert_allclose(admm.shrink_tube(t, 2.5), [[[1.5, 2.0]], [[0.0, 0.0]]])
    np.testing.assert_allclose(admm.shrink_tube(t, 6.0), np.zeros_like(t))


def test_metrics_closed_forms():
    """The recovery metrics against hand-computed values: an error of a tenth
    of the reference's norm is -20 dB, of a hundredth -40 dB; F1 from
    counted true and false positives."""
    x = np.zeros((4, 5, 3))
    x[0, 0, 0] = 3.0
    x[1, 2, 1] = 4.0                       # ||x|| = 5
    e = np.zeros_like(x)
    e[2, 2, 2] = 0.5                       # ||e|| = 0.5 = ||x|| / 10
    assert metrics.rse(x + e, x) == pytest.approx(0.1, rel=1e-15)
    assert metrics.rse_db(x + e, x) == pytest.approx(-20.0, rel=1e-14)
    assert metrics.rse_db(x + e / 10, x) == pytest.approx(-40.0, rel=1e-14)
    m = np.full((2, 2, 2), 10.0)           # threshold 1e-3 * 10 = 0.01
    s_true = np.zeros((2, 2, 2))
    s_true[0, 0, 0] = s_true[1, 1, 1] = 1.0
    s_hat = np.zeros((2, 2, 2))
    s_hat[0, 0, 0] = 0.5                   # true positive
    s_hat[0, 1, 0] = 0.02                  # false positive (above 0.01)
    s_hat[1, 0, 0] = 0.005                 # below the threshold: not predicted
    # tp = 1, fp = 1, fn = 1 -> F1 = 2 / (2 + 1 + 1)
    assert metrics.support_f1(s_hat, s_true, m) == pytest.approx(0.5, rel=1e-15)
    assert metrics.support_f1(np.zeros_like(s_hat), s_true, m) == 0.0
