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


def random_bond_masks(shape, p_cut, seed):
    """Symmetric per-site bond masks (bits x-, x+, y-, y+, z-, z+): every bond
    of the periodic lattice is cut with probability p_cut, at both ends."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    mask = np.full((nz, ny, nx), 0x3F, dtype=np.uint8)
    for axis, (lo, hi) in zip((2, 1, 0), ((0, 1), (2, 3), (4, 5))):
        cut = rng.uniform(size=mask.shape) < p_cut        # bond from each site to its + neighbour
        mask[cut] &= np.uint8(~(1 << hi) & 0xFF)
        nb_cut = np.roll(cut, 1, axis=axis)               # the same bond seen from the + neighbour
        mask[nb_cut] &= np.uint8(~(1 << lo) & 0xFF)
    return mask.reshape(-1)
