"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the method's
arithmetic, and both the GPU library's callers and the oracle's tests use it.
All draws use numpy's PCG64 generator with the seeds listed per workload.

Workloads (sizes and distributions):

* ``single``   C = A B, 256^3, A and B i.i.d. N(0, 1) (seeds 11 / 12).
* ``sweep``    4096^3, i.i.d. Laplace(b = 1) (seeds 21 / 22) or N(0, 1)
               (seeds 23 / 24); the throughput-distortion sweep of Sec. 7.
* ``scatter``  X: 2000 vectors x 10304 dims, uniform [0, 1) with the column
               means removed, float32 (seed 31); P: 10304 x 200 i.i.d. N(0, 1)
               float32 (seed 32). Stand-in for the 2D-PCA face-image scatter
               and projection GEMMs of Sec. 8.A (the face database is not
               available): X^T X and X P.
* ``mlp``      512 -> 1024 -> 1024 -> 10 perceptron, batch 4096, Xavier-uniform
               float32 weights (seed 41), inputs N(0, 1) and labels uniform on
               {0..9} in a pool of 16 batches (seed 42). Stand-in for the
               metadata-learning MLP of Sec. 8.B (the music database is not
               available).
* ``precision`` 8192^3 i.i.d. Laplace(b = 1) (seeds 51 / 52).
* ``random_range`` the generic inputs of Sec. 7: per L x L block, uniform on
               [-max_e, max_e] with max_e drawn from {4, 5, ..., 2048}.
* ``calib_uniforms`` the uniform [0, 1) draws of the representation-noise
               measurement (Sec. 4.B): (instances, L, L) for A and for B.
* ``faces``    synthetic stand-in for the 288 x 288 cropped face images of the
               2D-PCA application (Sec. 8.A; the face database is not
               available): 15 identities x 11 images (5 for training, 6 for
               testing), float32 pixel values in [0, 255]. An identity is a
               smooth random field (24 separable low-frequency cosine products,
               frequencies 0..6 per axis, amplitude 40) around 128; each image
               adds its own smooth variation (12 products, frequencies 0..3,
               amplitude 70) and N(0, 30^2) pixel noise, clipped (seed 81), so
               that FP64 2D-PCA (d = 10) recognises about 88 % of the test
               images, near the paper's accuracy on real faces.
"""
from __future__ import annotations

import numpy as np

SEEDS = {
    "single": (11, 12),
    "sweep_laplace": (21, 22),
    "sweep_gaussian": (23, 24),
    "scatter": (31, 32),
    "mlp": (41, 42),
    "precision": (51, 52),
    "random_range": (61, 62),
    "calib": (71, 72),
    "faces": (81, 82),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(shape, seed: int, dtype=np.float64) -> np.ndarray:
    return _rng(seed).standard_normal(shape).astype(dtype, copy=False)


def laplacian(shape, seed: int, b: float = 1.0, dtype=np.float64) -> np.ndarray:
    return _rng(seed).laplace(0.0, b, shape).astype(dtype, copy=False)


def single(n: int = 256):
    """256^3 single GEMM, N(0, 1) inputs."""
    sa, sb = SEEDS["single"]
    return gaussian((n, n), sa), gaussian((n, n), sb)


def sweep(dist: str = "gaussian", n: int = 4096, m: int | None = None, k: int | None = None):
    """Square (or M x K by K x N) sweep inputs, Laplace(1) or N(0, 1), float64."""
    m = n if m is None else m
    k = n if k is None else k
    if dist == "laplace":
        sa, sb = SEEDS["sweep_laplace"]
        return laplacian((m, k), sa), laplacian((k, n), sb)
    if dist == "gaussian":
        sa, sb = SEEDS["sweep_gaussian"]
        return gaussian((m, k), sa), gaussian((k, n), sb)
    if dist == "random_range":
        sa, sb = SEEDS["random_range"]
        return random_range((m, k), sa), random_range((k, n), sb)
    raise ValueError(dist)


def scatter(n_vec: int = 2000, dim: int = 10304, n_proj: int = 200):
    """Mean-removed uniform vectors X (float32) and a Gaussian projection P (float32)."""
    sx, sp = SEEDS["scatter"]
    x = _rng(sx).random((n_vec, dim))
    x = (x - x.mean(axis=0, keepdims=True)).astype(np.float32)
    p = gaussian((dim, n_proj), sp, np.float32)
    return x, p


def mlp(sizes=(512, 1024, 1024, 10), batch: int = 4096, pool: int = 16):
    """Xavier-uniform weights (in x out, float32), zero biases, and a pool of batches."""
    sw, sd = SEEDS["mlp"]
    rw = _rng(sw)
    weights, biases = [], []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = float(np.sqrt(6.0 / (fan_in + fan_out)))
        weights.append(rw.uniform(-lim, lim, (fan_in, fan_out)).astype(np.float32))
        biases.append(np.zeros(fan_out, dtype=np.float32))
    rd = _rng(sd)
    xs = rd.standard_normal((pool, batch, sizes[0])).astype(np.float32)
    ys = rd.integers(0, sizes[-1], (pool, batch)).astype(np.int64)
    return weights, biases, xs, ys


def precision(n: int = 8192):
    """8192^3 Laplace(1) inputs, float64."""
    sa, sb = SEEDS["precision"]
    return laplacian((n, n), sa), laplacian((n, n), sb)


def random_range(shape, seed: int, L: int = 64, lo: int = 4, hi: int = 2048) -> np.ndarray:
    """Per L x L block, uniform on [-max_e, max_e], max_e uniform on {lo, ..., hi}."""
    r = _rng(seed)
    out = r.uniform(-1.0, 1.0, shape)
    nb0, nb1 = -(-shape[0] // L), -(-shape[1] // L)
    scale = r.integers(lo, hi + 1, (nb0, nb1)).astype(np.float64)
    out *= np.repeat(np.repeat(scale, L, axis=0), L, axis=1)[:shape[0], :shape[1]]
    return out


def calib_uniforms(L: int, instances: int = 5):
    """Uniform [0, 1) draws for the representation-noise measurement."""
    sa, sb = SEEDS["calib"]
    return _rng(sa).random((instances, L, L)), _rng(sb).random((instances, L, L))


def faces(n_person: int = 15, n_train: int = 5, n_test: int = 6, size: int = 288):
    """(train, train_labels, test, test_labels): images (n, size, size) float32."""
    r = _rng(SEEDS["faces"][0])
    x = np.arange(size) / size

    def field(n_comp: int, fmax: int, amp: float) -> np.ndarray:
        out = np.zeros((size, size))
        for _ in range(n_comp):
            u, v = r.integers(0, fmax + 1, 2)
            pu, pv = r.uniform(0.0, 2.0 * np.pi, 2)
            a = amp * r.standard_normal()
            out += a * np.outer(np.cos(2.0 * np.pi * u * x + pu), np.cos(2.0 * np.pi * v * x + pv))
        return out

    train, test, ltr, lte = [], [], [], []
    for p in range(n_person):
        base = 128.0 + field(24, 6, 40.0)
        for k in range(n_train + n_test):
            img = base + field(12, 3, 70.0) + r.normal(0.0, 30.0, (size, size))
            img = np.clip(img, 0.0, 255.0).astype(np.float32)
            (train if k < n_train else test).append(img)
            (ltr if k < n_train else lte).append(p)
    return np.stack(train), np.array(ltr), np.stack(test), np.array(lte)
