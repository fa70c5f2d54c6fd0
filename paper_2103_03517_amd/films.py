"""Granular thin films (Sec. 4): columnar Voronoi grains with no exchange
between grains, and the weighted multi-Bloch fit of m(T) (Eq. 8).

A film is nx x ny x nz with periodic x and y and an open z boundary.  Grain
seeds are placed uniformly in the periodic nx x ny plane; every column of
sites belongs to the grain of the nearest seed (periodic distance), so the
grains run through the thickness.  A bond between two sites of different
grains is cut (its bit cleared at both ends), which sets the intergrain
exchange to zero.
"""
import math

import numpy as np


def voronoi_grains(nx, ny, mean_diameter, seed):
    """Grain index of every (y, x) column: nearest of n_g seeds, with
    n_g = nx ny / (pi d^2 / 4) for the mean grain diameter d (lattice
    sites).  Returns (grain map of shape (ny, nx), number of grains)."""
    from scipy.spatial import cKDTree
    ng = max(1, int(round(nx * ny / (math.pi * mean_diameter ** 2 / 4.0))))
    rng = np.random.default_rng(seed)
    sx = rng.uniform(0, nx, ng)
    sy = rng.uniform(0, ny, ng)
    # nearest seed of every column centre on the periodic nx x ny torus (a
    # k-d tree with periodic box: 1024^2 columns and 2 10^4 seeds in about a
    # second)
    tree = cKDTree(np.stack([sx, sy], axis=1), boxsize=(float(nx), float(ny)))
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    _, idx = tree.query(np.stack([xx.ravel(), yy.ravel()], axis=1))
    return idx.reshape(ny, nx).astype(np.int64), ng


def grain_bond_masks(grain, nz):
    """Bond masks (bits x-, x+, y-, y+, z-, z+ = bond active) of an nz-thick
    film whose columns carry the grain map: in-plane bonds between different
    grains are cut; bonds along z stay (columnar grains); the bonds across
    the open z boundary are left set, they do not exist."""
    ny, nx = grain.shape
    same_xp = grain == np.roll(grain, -1, axis=1)    # site and its x+ neighbour
    same_xm = grain == np.roll(grain, 1, axis=1)
    same_yp = grain == np.roll(grain, -1, axis=0)
    same_ym = grain == np.roll(grain, 1, axis=0)
    plane = (same_xm.astype(np.uint8) | (same_xp.astype(np.uint8) << 1) | (same_ym.astype(np.uint8) << 2)
             | (same_yp.astype(np.uint8) << 3) | np.uint8(16) | np.uint8(32))
    return np.broadcast_to(plane, (nz, ny, nx)).reshape(-1).copy()


def grain_areas(grain):
    _, counts = np.unique(grain, return_counts=True)
    return counts


def bloch(T, Tc, beta):
    """Bloch law of Eq. 3: (1 - T/Tc)^beta below Tc, 0 above."""
    T = np.asarray(T, dtype=float)
    return np.where(T < Tc, np.clip(1.0 - T / Tc, 0.0, None) ** beta, 0.0)


def multi_bloch(T, w, Tc, beta):
    """Eq. 8: sum_i w_i (1 - T/Tc_i)^beta_i."""
    return sum(wi * bloch(T, ti, bi) for wi, ti, bi in zip(w, Tc, beta))


def fit_multi_bloch(T, m, n_terms, seed=0, tc_range=(0.05, 2.5), beta_range=(0.2, 0.6)):
    """Least-squares fit of Eq. 8 with n_terms Bloch terms (weights >= 0
    summing to one, through a softmax); returns (w, Tc, beta, mean Tc =
    sum w_i Tc_i, rms residual).  Several starts; the best is kept."""
    from scipy.optimize import least_squares
    T = np.asarray(T, dtype=float)
    m = np.asarray(m, dtype=float)
    rng = np.random.default_rng(seed)
    t_lo, t_hi = tc_range
    b_lo, b_hi = beta_range

    def unpack(p):
        a = p[:n_terms]
        w = np.exp(a - a.max())
        w /= w.sum()
        return w, p[n_terms:2 * n_terms], p[2 * n_terms:]

    def resid(p):
        w, tc, b = unpack(p)
        return multi_bloch(T, w, tc, b) - m

    lo = np.concatenate([np.full(n_terms, -20.0), np.full(n_terms, t_lo), np.full(n_terms, b_lo)])
    hi = np.concatenate([np.full(n_terms, 20.0), np.full(n_terms, t_hi), np.full(n_terms, b_hi)])
    best = None
    tmax = float(T.max())
    for start in range(8):
        tc0 = np.sort(rng.uniform(max(t_lo, 0.3 * tmax), min(t_hi, 1.2 * tmax), n_terms))
        p0 = np.concatenate([np.zeros(n_terms), tc0, np.full(n_terms, 0.35)])
        r = least_squares(resid, np.clip(p0, lo + 1e-9, hi - 1e-9), bounds=(lo, hi))
        if best is None or r.cost < best.cost:
            best = r
    w, tc, b = unpack(best.x)
    rms = float(np.sqrt(np.mean(resid(best.x) ** 2)))
    return w, tc, b, float(np.dot(w, tc)), rms
