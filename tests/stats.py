"""Small statistics helpers for the Monte Carlo tests (no method arithmetic)."""
import numpy as np


def batch_mean_se(x, nbatch=20):
    """Mean and batch-means standard error of a correlated series."""
    x = np.asarray(x, dtype=np.float64)
    nb = len(x) // nbatch
    if nb < 1:
        raise ValueError("series too short")
    b = x[: nb * nbatch].reshape(nbatch, nb).mean(axis=1)
    return float(x.mean()), float(b.std(ddof=1) / np.sqrt(nbatch))


def langevin(x):
    return 1.0 / np.tanh(x) - 1.0 / x


def langevin_prime(x):
    return 1.0 / x ** 2 - 1.0 / np.sinh(x) ** 2
