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


def grain_bond_masks(shape, diameter, seed):
    """Bond masks of a granular film: columnar grains from the nearest of
    nx*ny/(pi d^2/4) seeds placed uniformly in the periodic plane, every
    in-plane bond between two grains cut at both ends (z bonds stay).
    Returns (masks in site order, number of grains)."""
    from scipy.spatial import cKDTree
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    ng = max(1, int(round(nx * ny / (np.pi * diameter ** 2 / 4.0))))
    seeds = rng.uniform(0.0, 1.0, size=(ng, 2)) * np.array([nx, ny])
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    _, grain = cKDTree(seeds, boxsize=[nx, ny]).query(np.stack([xx.ravel(), yy.ravel()], axis=1))
    grain = grain.reshape(ny, nx)
    plane = np.full((ny, nx), 0x3F, dtype=np.uint8)
    cut_x = grain != np.roll(grain, -1, axis=1)          # bond to the x+ neighbour
    plane[cut_x] &= np.uint8(~(1 << 1) & 0xFF)
    plane[np.roll(cut_x, 1, axis=1)] &= np.uint8(~(1 << 0) & 0xFF)
    cut_y = grain != np.roll(grain, -1, axis=0)          # bond to the y+ neighbour
    plane[cut_y] &= np.uint8(~(1 << 3) & 0xFF)
    plane[np.roll(cut_y, 1, axis=0)] &= np.uint8(~(1 << 2) & 0xFF)
    return np.broadcast_to(plane, (nz, ny, nx)).reshape(-1).copy(), len(np.unique(grain))


def wall_spins(shape, width, seed, noise=0.05):
    """A wall across z: S = (sech u, 0, tanh u) with u = pi (z - nz/2)/width,
    plus seeded noise, normalised; site order x fastest."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    u = np.pi * (np.arange(nz) + 0.5 - nz / 2.0) / width
    prof = np.stack([1.0 / np.cosh(u), np.zeros(nz), np.tanh(u)], axis=1)
    v = np.repeat(prof, nx * ny, axis=0) + noise * rng.normal(size=(nx * ny * nz, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v
