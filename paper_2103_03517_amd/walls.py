"""Domain-wall width and exchange stiffness (Sec. 3, Eq. 5).

A lattice that is anti-periodic along z holds exactly one domain wall across
z in its ordered state: continuing the profile past the box flips its sign,
f(z + nz) = -f(z), so the easy-axis component must cross zero an odd number
of times.  The profile of the easy-axis magnetisation, averaged over each
z plane (nx*ny sites), follows m tanh(-pi (z - z0)/Delta) (Eq. 5's wall
width Delta = pi sqrt(A/K)), so A(T) = K(T) Delta(T)^2 / pi^2 once K(T) is
known from uniform-state runs.

Without dipolar coupling a wall whose normal is z and one whose normal is x
are related by a lattice rotation, so the wall along z with the easy axis
along z has the width of the paper's wall along x.
"""
import math

import numpy as np


def extended_profile(f):
    """The twisted profile continued over two box lengths: index t in
    [0, 2 nz) holds f(t mod nz) times (-1)^(t // nz)."""
    f = np.asarray(f, dtype=float)
    return np.concatenate([f, -f])


def wall_centre(f):
    """Centre of the wall: the shift z0 in [0, nz) that maximises the overlap
    of the twisted profile with a step from +1 to -1 at z0 (a matched
    filter, robust to thermal noise)."""
    f = np.asarray(f, dtype=float)
    nz = len(f)
    e = extended_profile(f)
    half = nz // 2
    best, z0 = -math.inf, 0.0
    for c in range(nz):
        # window [c - half, c + half) in the extended profile (period 2 nz)
        idx = (np.arange(c - half, c + half) + 2 * nz) % (2 * nz)
        w = e[idx]
        score = w[:half].sum() - w[half:].sum()
        score = max(score, -score)
        if score > best:
            best, z0 = score, c - 0.5
    return z0 % nz


def window(f, z0):
    """Positions t (relative to z0, in [-nz/2, nz/2)) and the twisted
    profile at those planes, so that the wall sits at t = 0."""
    f = np.asarray(f, dtype=float)
    nz = len(f)
    e = extended_profile(f)
    c = int(math.floor(z0 + 0.5))
    zs = np.arange(c - nz // 2, c + nz // 2)
    vals = e[(zs + 2 * nz) % (2 * nz)]
    return zs - z0, vals


def fit_wall(f, delta_guess=10.0):
    """Least-squares fit of m tanh(-pi (t - t0)/Delta) to one profile.
    Returns (m, z0, Delta); m > 0 by convention (the sign of the wall is
    absorbed in the direction of t)."""
    from scipy.optimize import curve_fit
    z0 = wall_centre(f)
    t, v = window(f, z0)
    sgn = 1.0 if v[: len(v) // 2].mean() >= v[len(v) // 2:].mean() else -1.0
    v = sgn * v

    def model(tt, m, t0, d):
        return m * np.tanh(-math.pi * (tt - t0) / d)

    m0 = max(float(np.abs(v).max()), 1e-3)
    p, _ = curve_fit(model, t, v, p0=(m0, 0.0, delta_guess),
                     bounds=([0.0, -len(f) / 4, 0.5], [1.5, len(f) / 4, float(len(f))]))
    return float(p[0]), float((z0 + p[1]) % len(f)), float(p[2])


def exchange_stiffness(K, delta):
    """A = K Delta^2 / pi^2 (Eq. 5)."""
    return K * delta ** 2 / math.pi ** 2


def zero_temperature_width(J, Ku):
    """Delta(0) = pi sqrt(A/K) with the continuum stiffness A = J/2 of the
    simple-cubic lattice (E = -J sum_bonds S_i.S_j, unit spacing) and
    K = Ku."""
    return math.pi * math.sqrt(J / (2.0 * Ku))


def initial_wall(nx, ny, nz, width=None):
    """One wall centred between planes nz/2 - 1 and nz/2 and none at the
    anti-periodic boundary: spins +z below, -z above.  width=None gives a
    sharp wall; otherwise the T = 0 profile of that width, S = (sech u, 0,
    -tanh u) with u = pi (z - z0)/width.  Site order x fastest, then y, z."""
    n = nx * ny * nz
    z = np.repeat(np.arange(nz), nx * ny).astype(float)
    S = np.zeros((n, 3))
    if width is None:
        S[:, 2] = np.where(z < nz // 2, 1.0, -1.0)
    else:
        u = math.pi * (z - (nz / 2.0 - 0.5)) / width
        S[:, 0] = 1.0 / np.cosh(u)
        S[:, 2] = -np.tanh(u)
    return S
