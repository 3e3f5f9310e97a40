"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and arranges them into arrays.  It holds
none of the sampler's arithmetic (no likelihood, no move, no weight, no
resampling), so both the CPU oracle and the HIP path can take their inputs
from it without sharing any of the method's code.

The paper evaluates on MNIST and FashionMNIST (image classification, 70,000
28x28 grey images, 10 classes; Section 4).  Those datasets are not available
here, so the generators below produce synthetic stand-ins with the same
shapes, value ranges and class structure:

* ``blobs``        two 2-D Gaussian classes with means +-(1.5, 1.5) and unit
                   covariance (a tiny parity workload);
* ``templates28``  28x28 grey images: one N(0,1) template per class plus
                   pixel noise of std 0.3, clipped to [0, 1] (MNIST-shaped);
* ``textures32``   32x32x3 class-conditional Gaussian textures (a
                   CIFAR-shaped workload for the convolutional model);
* ``linreg``       Gaussian linear-regression data for the exact Bayesian
                   linear-regression posterior check.

Noise that the sampler draws (momenta, resampling uniforms, prior draws) can
also be produced here so that the CPU oracle and the GPU path can be fed the
same random numbers in parity tests.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "blobs",
    "templates28",
    "textures32",
    "linreg",
    "annealing_permutation",
    "momenta",
    "uniforms",
    "prior_draw",
]


def _balanced_labels(rng: np.random.Generator, n: int, n_cls: int) -> np.ndarray:
    """n labels with each class appearing floor(n/n_cls) or +1 times, shuffled."""
    y = np.arange(n, dtype=np.int64) % n_cls
    rng.shuffle(y)
    return y.astype(np.int32)


def blobs(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Two-class 2-D Gaussian blobs: class 0 around (-1.5,-1.5), class 1 around (+1.5,+1.5).

    Returns (X float32 [n x 2], y int32 [n]); the classes are balanced.
    """
    rng = np.random.default_rng(seed)
    y = _balanced_labels(rng, n, 2)
    mu = np.where(y[:, None] == 1, 1.5, -1.5).astype(np.float64)
    X = mu + rng.standard_normal((n, 2))
    return X.astype(np.float32), y


def templates28(n: int, seed: int, template_seed: int = 0, n_cls: int = 10,
                noise_std: float = 0.3) -> tuple[np.ndarray, np.ndarray]:
    """MNIST-shaped images: x = clip(T_c + noise_std * eps, 0, 1), flattened to 784.

    The class templates T_c ~ N(0, I_784) depend only on ``template_seed`` so that
    train and test sets drawn with different ``seed`` share the same classes.
    Returns (X float32 [n x 784], y int32 [n]).
    """
    trng = np.random.default_rng(template_seed)
    T = trng.standard_normal((n_cls, 784)).astype(np.float32)
    rng = np.random.default_rng(seed)
    y = _balanced_labels(rng, n, n_cls)
    X = np.empty((n, 784), dtype=np.float32)
    step = 8192
    for s in range(0, n, step):
        e = min(n, s + step)
        eps = rng.standard_normal((e - s, 784), dtype=np.float32)
        X[s:e] = np.clip(T[y[s:e]] + np.float32(noise_std) * eps, 0.0, 1.0)
    return X, y


def textures32(n: int, seed: int, template_seed: int = 0, n_cls: int = 10, size: int = 32) -> tuple[np.ndarray, np.ndarray]:
    """CIFAR-shaped class-conditional textures, NHWC float32 [n x size x size x 3] (size 32 by default).

    Class c has a mean colour m_c ~ N(0, 0.5) per channel and a 3x3 kernel k_c ~
    N(0, 1/9) per channel; an image is m_c + (k_c convolved with white noise),
    with circular boundary handling.
    """
    trng = np.random.default_rng(template_seed)
    mean = trng.normal(0.0, np.sqrt(0.5), size=(n_cls, 3))
    kern = trng.normal(0.0, 1.0 / 3.0, size=(n_cls, 3, 3, 3))  # [class, dy, dx, channel]
    rng = np.random.default_rng(seed)
    y = _balanced_labels(rng, n, n_cls)
    X = np.empty((n, size, size, 3), dtype=np.float32)
    step = 4096
    for s in range(0, n, step):
        e = min(n, s + step)
        eps = rng.standard_normal((e - s, size, size, 3))
        k = kern[y[s:e]]
        acc = np.zeros((e - s, size, size, 3))
        for dy in range(3):
            for dx in range(3):
                acc += k[:, dy, dx, :][:, None, None, :] * np.roll(eps, (1 - dy, 1 - dx), axis=(1, 2))
        X[s:e] = (acc + mean[y[s:e]][:, None, None, :]).astype(np.float32)
    return X, y


def linreg(n: int, d: int, seed: int, noise_std: float = 0.5) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Gaussian linear-regression data y = X w + b + noise_std * eps.

    Returns (X float32 [n x d], y float32 [n], true parameters float64 [d+1]).
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(d + 1)
    X = rng.standard_normal((n, d))
    y = X @ w[:d] + w[d] + noise_std * rng.standard_normal(n)
    return X.astype(np.float32), y.astype(np.float32), w


def annealing_permutation(n: int, seed: int) -> np.ndarray:
    """One without-replacement ordering of the n data points (int64 [n])."""
    return np.random.default_rng(seed).permutation(n)


def momenta(seed: int, shape) -> np.ndarray:
    """Standard-normal float32 draws (momenta or other Gaussian move noise)."""
    return np.random.default_rng(seed).standard_normal(shape, dtype=np.float32)


def uniforms(seed: int, n: int) -> np.ndarray:
    """Uniform float64 draws in [0, 1) (e.g. the systematic-resampling offset)."""
    return np.random.default_rng(seed).random(n)


def prior_draw(seed: int, n_particles: int, dim: int, prior_std: float) -> np.ndarray:
    """Initial particles from the N(0, prior_std^2 I) prior, float32 [J x D]."""
    rng = np.random.default_rng(seed)
    return (prior_std * rng.standard_normal((n_particles, dim))).astype(np.float32)
