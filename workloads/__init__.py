"""Seeded synthetic workloads shared by the tests, the benchmark and smoke().

This module only draws inputs.  It holds none of the solver arithmetic: no
transform of the hot path, no thresholding, no ADMM step.  The one piece of
tensor algebra here is the t-product used to *plant* a low-tubal-rank tensor
(X = A * B, Sec. 2.1 of arXiv:1407.1785); ``tests/test_oracle_tensor.py``
pins it against the oracle's direct circular-convolution t-product.

Every generator takes a ``trial`` number and draws from
``SeedSequence([14071785, workload_id, trial])`` with one child stream per
ingredient (factors, mask, sparse part, texture, arrivals), so changing one
ingredient's size never shifts another's random numbers.

Workloads (ids):
  0  plain completion, tubal rank 2, 32x32x16, Bernoulli(0.5) mask
  1  video-shaped completion, 128x160x64 smoothed translated texture, 20% seen
  2  tensor RPCA, 256x256x64 rank-5 plus 10% sparse U[-1,1] corruption
  3  batch of 64 uneven completion problems
  4  serving mix (Poisson arrivals, completion / RPCA / 4-D colour video)
  5  tube-block corruption for the l1,1,2 RPCA (same pixels within blocks of frames)
  6  sampling-rate sweep (3-D and 4-D synthetic videos, masks 10%..90%)
  7  tube-block video RPCA (Sec. 5 experiment shape 72x128x80, synthetic)
"""

from __future__ import annotations

import math

import numpy as np

SEED_BASE = 14071785


def streams(workload: int, trial: int, count: int = 5):
    """Independent generators for one (workload, trial) pair."""
    ss = np.random.SeedSequence([SEED_BASE, int(workload), int(trial)])
    return [np.random.default_rng(s) for s in ss.spawn(count)]


def plant_tprod(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """X = A * B for planting a low-tubal-rank tensor (third-order only)."""
    ah = np.fft.rfft(a, axis=2)
    bh = np.fft.rfft(b, axis=2)
    ch = np.einsum("ikt,kjt->ijt", ah, bh)
    return np.fft.irfft(ch, n=a.shape[2], axis=2)


def lowrank(rng, n1, n2, n3, r, std=1.0):
    """A (n1 x r x n3), B (r x n2 x n3) i.i.d. N(0, std^2) and X = A * B."""
    a = rng.normal(0.0, std, size=(n1, r, n3))
    b = rng.normal(0.0, std, size=(r, n2, n3))
    return a, b, plant_tprod(a, b)


def bernoulli_mask(rng, shape, p):
    return (rng.random(shape) < p).astype(np.uint8)


def exact_mask(rng, shape, frac):
    """Exactly round(frac * size) entries observed, uniformly without
    replacement."""
    size = int(np.prod(shape))
    k = int(round(frac * size))
    mask = np.zeros(size, dtype=np.uint8)
    mask[rng.choice(size, size=k, replace=False)] = 1
    return mask.reshape(shape)


# ------------------------------------------------------------ workload 0

def completion_small(trial=0, shape=(32, 32, 16), rank=2, p=0.5):
    """Plain completion: X = A * B with A n1 x r x n3 and B r x n2 x n3
    i.i.d. N(0, 1); Bernoulli(p) mask.  Solver settings: rho0 = 1e-2 grown
    by 1.1 up to 1e3, at most 300 iterations, tol 1e-8."""
    n1, n2, n3 = shape
    g_fac, g_mask = streams(0, trial, 2)
    _, _, x = lowrank(g_fac, n1, n2, n3, rank)
    mask = bernoulli_mask(g_mask, shape, p)
    return dict(X=x, mask=mask, M_obs=x * mask, rho=1e-2, growth=1.1, rho_max=1e3,
                max_iter=300, tol=1e-8)


# ------------------------------------------------------------ workload 1

def texture(rng, rows, cols, sigma=4.0):
    """U[0,1) noise smoothed by a Gaussian (sigma px, reflect, truncate 4),
    min-max scaled to [0, 1]."""
    from scipy import ndimage

    t = ndimage.gaussian_filter(rng.random((rows, cols)), sigma=sigma, mode="reflect",
                                truncate=4.0)
    t -= t.min()
    t /= t.max()
    return t


def translate(tex, n1, n2, frames, vy=0.4, vx=0.7, margin=2.0):
    """Frame t at pixel (i, j) samples the texture bilinearly at
    (margin + i + vy t, margin + j + vx t): rows (mode 1) drift vy px per
    frame, columns (mode 2) vx px per frame."""
    out = np.empty((n1, n2, frames))
    ii = np.arange(n1, dtype=np.float64)[:, None]
    jj = np.arange(n2, dtype=np.float64)[None, :]
    for t in range(frames):
        y = margin + ii + vy * t
        x = margin + jj + vx * t
        y0 = np.floor(y).astype(np.int64)
        x0 = np.floor(x).astype(np.int64)
        fy = y - y0
        fx = x - x0
        out[:, :, t] = ((1 - fy) * (1 - fx) * tex[y0, x0] + (1 - fy) * fx * tex[y0, x0 + 1]
                        + fy * (1 - fx) * tex[y0 + 1, x0] + fy * fx * tex[y0 + 1, x0 + 1])
    return out


def video(rng, n1, n2, frames, vy=0.4, vx=0.7, sigma=4.0):
    """Grayscale video-shaped tensor in [0, 1] (float32 values)."""
    rows = n1 + int(math.ceil(vy * (frames - 1))) + 6
    cols = n2 + int(math.ceil(vx * (frames - 1))) + 6
    tex = texture(rng, rows, cols, sigma)
    return translate(tex, n1, n2, frames, vy, vx).astype(np.float32)


def video_completion(trial=0, shape=(128, 160, 64), frac=0.2, iters=200):
    """Video-shaped completion: smoothed texture (sigma = 4 px) translated by
    (0.4, 0.7) px per frame, float32 in [0, 1]; exactly frac of the entries
    observed; a fixed number of ADMM iterations (tol = 0) with the rho
    schedule of workload 0."""
    n1, n2, n3 = shape
    g_tex, g_mask = streams(1, trial, 2)
    x = video(g_tex, n1, n2, n3)
    mask = exact_mask(g_mask, shape, frac)
    return dict(X=x, mask=mask, M_obs=x * mask, rho=1e-2, growth=1.1, rho_max=1e3,
                max_iter=iters, tol=0.0)


def color_video(rng, n1=96, n2=128, channels=3, frames=48):
    """4-D colour video (n1, n2, channels, frames): one independent smoothed
    texture per channel, all translated the same way."""
    out = np.empty((n1, n2, channels, frames), dtype=np.float32)
    for c in range(channels):
        out[:, :, c, :] = video(rng, n1, n2, frames)
    return out


def sampling_sweep(trial=0, rates=(0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9)):
    """Sampling-rate sweep inputs (the Sec. 6 completion experiment, synthetic):
    the grayscale video 128 x 160 x 64 and the colour video 96 x 128 x 3 x 48
    (smoothed textures translated by (0.4, 0.7) px per frame), and for each
    rate an exactly-sized uniform mask of each."""
    g_v3, g_v4, g_mask = streams(6, trial, 3)
    v3 = video(g_v3, 128, 160, 64)
    v4 = color_video(g_v4)
    masks = {p: (exact_mask(g_mask, v3.shape, p), exact_mask(g_mask, v4.shape, p)) for p in rates}
    return dict(video3=v3, video4=v4, masks=masks, rho=1e-2, growth=1.1, rho_max=1e3)


# ------------------------------------------------------------ workload 2

def trpca_problem(trial=0, n=256, n3=64, rank=5, frac=0.1, shape=None):
    """Tensor RPCA: L = A * B with A n1 x r x n3, B r x n2 x n3 i.i.d.
    N(0, 1/n1); S on exactly frac of the entries with values U[-1, 1];
    M = L + S; lam = 1/sqrt(max(n1, n2) n3); mu0 = 1e-3 grown by 1.2 up to
    1e10; tol 1e-7; at most 500 iterations; entrywise l1 shrink."""
    if shape is None:
        shape = (n, n, n3)
    n1, n2, n3 = shape
    g_fac, g_sp = streams(2, trial, 2)
    _, _, lo = lowrank(g_fac, n1, n2, n3, rank, std=1.0 / math.sqrt(n1))
    supp = exact_mask(g_sp, shape, frac).astype(bool)
    sp = np.zeros(shape)
    sp[supp] = g_sp.uniform(-1.0, 1.0, size=int(supp.sum()))
    lam = 1.0 / math.sqrt(max(n1, n2) * n3)
    return dict(L=lo, S=sp, M=lo + sp, lam=lam, mu=1e-3, growth=1.2, mu_max=1e10,
                max_iter=500, tol=1e-7, shrink="l1")


def tube_corruption(trial=0, shape=(36, 64, 40), rank=3, frac=0.05, block=10, amp=1.0):
    """Tube-sparse corruption (the Sec. 5 experiment shape, synthetic): a
    random fraction of pixel tubes gets Gaussian noise, the corrupted pixels
    being the same within every block of ``block`` frames."""
    n1, n2, n3 = shape
    g_fac, g_sp = streams(5, trial, 2)
    _, _, lo = lowrank(g_fac, n1, n2, n3, rank, std=1.0 / math.sqrt(n1))
    sp = np.zeros(shape)
    for t0 in range(0, n3, block):
        pix = g_sp.random((n1, n2)) < frac
        t1 = min(n3, t0 + block)
        sp[pix, t0:t1] = g_sp.normal(0.0, amp, size=(int(pix.sum()), t1 - t0))
    lam = 1.0 / math.sqrt(max(n1, n2))
    return dict(L=lo, S=sp, M=lo + sp, lam=lam)


def tube_block_video(trial=0, shape=(72, 128, 80), frac=0.02, block=10, amp=0.5):
    """The Sec. 5 RPCA experiment, synthetic: a smoothed translated-texture
    video (values in [0, 1]) as the low-rank part; in every block of `block`
    frames a random fraction `frac` of the pixels gets i.i.d. N(0, amp^2)
    noise on every frame of the block (the same pixels within a block).
    lam_tensor = 1/sqrt(max(n1, n2)) (the paper's choice for tensor RPCA with
    the tube shrink), lam_matrix = 1/sqrt(max(n1 n2, n3)) for matrix RPCA on
    the n1 n2 x n3 unfolding; mu0 = 1e-3 grown by 1.2 up to 1e10, tol 1e-7,
    at most 500 iterations."""
    n1, n2, n3 = shape
    g_v, g_sp = streams(7, trial, 2)
    lo = video(g_v, n1, n2, n3).astype(np.float64)
    sp = np.zeros(shape)
    for t0 in range(0, n3, block):
        pix = g_sp.random((n1, n2)) < frac
        t1 = min(n3, t0 + block)
        sp[pix, t0:t1] = g_sp.normal(0.0, amp, size=(int(pix.sum()), t1 - t0))
    return dict(L=lo, S=sp, M=lo + sp, lam_tensor=1.0 / math.sqrt(max(n1, n2)),
                lam_matrix=1.0 / math.sqrt(max(n1 * n2, n3)), mu=1e-3, growth=1.2, mu_max=1e10,
                tol=1e-7, max_iter=500)


# ------------------------------------------------------------ workload 3

def batch_specs(trial=0, count=64, n_lo=48, n_hi=320, n3_lo=8, n3_hi=128):
    """Shapes and settings of the uneven batch: n1, n2 ~ U{48..320},
    n3 ~ U{8..128}, tubal rank ~ U{2..10}, sampling ratio ~ U[0.2, 0.6]."""
    (g,) = streams(3, trial, 1)
    specs = []
    for _ in range(count):
        specs.append(dict(n1=int(g.integers(n_lo, n_hi + 1)), n2=int(g.integers(n_lo, n_hi + 1)),
                          n3=int(g.integers(n3_lo, n3_hi + 1)), rank=int(g.integers(2, 11)),
                          p=float(g.uniform(0.2, 0.6))))
    return specs


def batch_problem(spec, index, trial=0, iters=150):
    """One member of the batch: N(0, 1) factors, Bernoulli(p) mask, a fixed
    iteration count with the rho schedule of workload 0."""
    g_fac, g_mask = streams(3, 1000 * (trial + 1) + index, 2)
    shape = (spec["n1"], spec["n2"], spec["n3"])
    _, _, x = lowrank(g_fac, *shape, spec["rank"])
    mask = bernoulli_mask(g_mask, shape, spec["p"])
    return dict(X=x, mask=mask, M_obs=x * mask, rho=1e-2, growth=1.1, rho_max=1e3,
                max_iter=iters, tol=0.0)


# ------------------------------------------------------------ workload 4

def arrivals(trial=0, rate=50.0, seconds=60.0):
    """Poisson arrival times (s) and request kinds for the serving mix:
    70% completion / 30% tensor RPCA; 10% of requests are 4-D colour video
    96 x 128 x 3 x 48, the rest draw a 3-D shape as in workload 3."""
    g_arr, g_kind = streams(4, trial, 2)
    times = []
    t = g_arr.exponential(1.0 / rate)
    while t < seconds:
        times.append(t)
        t += g_arr.exponential(1.0 / rate)
    reqs = []
    for i, ta in enumerate(times):
        kind = "complete" if g_kind.random() < 0.7 else "trpca"
        color = bool(g_kind.random() < 0.1)
        reqs.append(dict(id=i, t=float(ta), kind=kind, color=color))
    return reqs


def serve_request(req, trial=0, iters=150, tol=1e-7):
    """Data of one request of the serving mix (``arrivals``).

    Shape: the 4-D colour video 96 x 128 x 3 x 48 when ``req["color"]``,
    else n1, n2 ~ U{48..320}, n3 ~ U{8..128} as in workload 3.
    Completion requests: tubal rank ~ U{2..10} with N(0, 1) factors (colour
    requests: the video itself), Bernoulli(p) mask with p ~ U[0.2, 0.6],
    rho0 = 1e-2 grown by 1.1 up to 1e3.  RPCA requests: the low-rank part as
    in workload 2 (factors N(0, 1/n1); colour requests: the video), 10% of
    the entries replaced by U[-1, 1] corruption added on top, lam =
    1/sqrt(max(n1, n2) * L) with L the tube length, mu0 = 1e-3 grown by 1.2
    up to 1e10.  At most ``iters`` iterations, stopping tolerance ``tol``."""
    g_shape, g_fac, g_mask = streams(4, 100000 * (trial + 1) + int(req["id"]), 3)
    rpca = req["kind"] == "trpca"
    if req["color"]:
        x = color_video(g_fac).astype(np.float64)
    else:
        n1, n2 = (int(v) for v in g_shape.integers(48, 321, size=2))
        n3 = int(g_shape.integers(8, 129))
        r = int(g_shape.integers(2, 11))
        _, _, x = lowrank(g_fac, n1, n2, n3, r, std=(1.0 / math.sqrt(n1)) if rpca else 1.0)
    shape = x.shape
    if not rpca:
        p = float(g_shape.uniform(0.2, 0.6))
        mask = bernoulli_mask(g_mask, shape, p)
        return dict(kind="complete", X=x, mask=mask, M_obs=x * mask, rho=1e-2, growth=1.1, rho_max=1e3,
                    max_iter=iters, tol=tol)
    supp = exact_mask(g_mask, shape, 0.1).astype(bool)
    sp = np.zeros(shape)
    sp[supp] = g_mask.uniform(-1.0, 1.0, size=int(supp.sum()))
    tube = int(np.prod(shape[2:]))
    lam = 1.0 / math.sqrt(max(shape[0], shape[1]) * tube)
    return dict(kind="trpca", L=x, S=sp, M=x + sp, lam=lam, mu=1e-3, growth=1.2, mu_max=1e10,
                max_iter=iters, tol=tol)
