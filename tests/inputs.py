"""Seeded synthetic inputs shared by the CPU reference and the GPU library.

This module holds no arithmetic of the method: it only draws parameter sets
and spin configurations from numpy's seeded generator, in the lexicographic
(site id = x + nx*(y + ny*z)) AoS layout that both sides accept.
"""
import numpy as np


def random_unit_spins(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def tilted_spins(n, seed, spread=0.3, axis=(0.0, 0.0, 1.0)):
    """Spins scattered around `axis` (an ordered but not aligned state)."""
    rng = np.random.default_rng(seed)
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    v = a[None, :] + spread * rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def random_params(seed):
    """A parameter set with every term of the Hamiltonian switched on."""
    rng = np.random.default_rng(seed)
    eu = rng.normal(size=3)
    eu /= np.linalg.norm(eu)
    return dict(J=float(rng.uniform(0.5, 1.5)), Ku=float(rng.uniform(-0.2, 0.3)), eu=tuple(eu),
                Kc=float(rng.uniform(-0.2, 0.2)), h=tuple(rng.normal(scale=0.2, size=3)))
