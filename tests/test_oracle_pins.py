"""Pins of the CPU reference against facts fixed outside of it.

Each test names what it checks the reference against: an installed library
(rocRAND), a closed form of the mathematics, a limit of the physics, or an
independent sampler.  None of these tests calls the GPU library.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats as sps

from tests import inputs
from tests.stats import batch_mean_se, langevin, langevin_prime

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host program")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "golden", "philox_rocrand.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(oracle_mod, rocrand_philox):
    """Philox4x32-10 of the reference equals rocRAND's engine bit for bit."""
    rng = np.random.default_rng(11)
    rows = [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0), (0, 0, 0, 0, 1, 0), (0, 1, 2, 3, 4, 5),
            (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(300):
        c = rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF  # rocRAND's offset argument holds counter word 1 times four
        rows.append(tuple(int(v) for v in c))
    text = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_philox], input=text, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        expect = [int(v) for v in line.split()]
        assert oracle_mod.philox(r[:4], r[4:]) == expect, r


def test_fmix32_avalanche(oracle_mod):
    """The round function mixes: one flipped input bit flips ~16 output bits."""
    rng = np.random.default_rng(3)
    flips = []
    for _ in range(2000):
        x = int(rng.integers(0, 2 ** 32))
        b = int(rng.integers(0, 32))
        flips.append(bin(oracle_mod.fmix32(x) ^ oracle_mod.fmix32(x ^ (1 << b))).count("1"))
    assert abs(np.mean(flips) - 16.0) < 0.4
    assert oracle_mod.fmix32(0) == 0  # every step of the finaliser maps 0 to 0


@pytest.mark.parametrize("n", list(range(1, 300)) + [1023, 1024, 1025, 4096, 4100, 65536])
def test_feistel_is_a_permutation(oracle_mod, n):
    key = (0x12345678, 0x9ABCDEF0, 0x0F1E2D3C, 0x4B5A6978)
    img = [oracle_mod.feistel(x, n, key) for x in range(n)]
    assert sorted(img) == list(range(n))


def test_feistel_depends_on_key_and_mixes(oracle_mod):
    n = 4096
    ka = (1, 2, 3, 4)
    kb = (1, 2, 3, 5)
    pa = np.array([oracle_mod.feistel(x, n, ka) for x in range(n)])
    pb = np.array([oracle_mod.feistel(x, n, kb) for x in range(n)])
    assert np.mean(pa == pb) < 0.01
    # a uniform random permutation has ~1 fixed point and |pi(x)-x| averaging n/3
    assert np.sum(pa == np.arange(n)) < 8
    assert abs(np.mean(np.abs(pa - np.arange(n))) / n - 1.0 / 3.0) < 0.03
    # consecutive outputs (which form the pairs) are not correlated
    assert abs(np.corrcoef(pa[0::2], pa[1::2])[0, 1]) < 0.06


# --------------------------------------------------------------------------
# Cone proposal (Table A1: a uniform draw in a cone about the spin)
# --------------------------------------------------------------------------

def test_onb_is_orthonormal_right_handed(oracle_mod):
    vs = list(inputs.random_unit_spins(500, 5))
    vs += [np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, -1.0]),
           np.array([1e-9, 0.0, -1.0]) / np.linalg.norm([1e-9, 0.0, -1.0]),
           np.array([1.0, 0.0, 0.0])]
    for n in vs:
        b1, b2 = oracle_mod.onb(n)
        M = np.stack([b1, b2, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(b1, b2), n, atol=1e-12)


def test_cone_move_closed_form(oracle_mod):
    """S.S' = 1 - u0 (1 - cos theta) and the azimuth in (b1, b2) is 2 pi u1."""
    rng = np.random.default_rng(7)
    spins = inputs.random_unit_spins(300, 8)
    for S in spins:
        th = int(rng.integers(1, 181))
        u0, u1 = rng.uniform(size=2)
        Sn = oracle_mod.cone_move(S, u0, u1, th)
        c1 = 1.0 - np.cos(np.radians(th))
        assert abs(np.linalg.norm(Sn) - 1.0) < 1e-14
        assert abs(S @ Sn - (1.0 - u0 * c1)) < 1e-12
        b1, b2 = oracle_mod.onb(S)
        phi = np.arctan2(Sn @ b2, Sn @ b1) % (2 * np.pi)
        if u0 * c1 > 1e-10:
            d = abs(phi - 2 * np.pi * u1)
            assert min(d, 2 * np.pi - d) < 1e-6


def test_cone_move_is_uniform_on_the_cap(oracle_mod):
    """cos(alpha) ~ U(cos theta, 1) and azimuth ~ U(0, 2 pi) for uniform u0, u1."""
    rng = np.random.default_rng(9)
    S = np.array([0.3, -0.4, 0.866])
    S /= np.linalg.norm(S)
    th = 40
    b1, b2 = oracle_mod.onb(S)
    ca, ph = [], []
    for u0, u1 in rng.uniform(size=(4000, 2)):
        Sn = oracle_mod.cone_move(S, u0, u1, th)
        ca.append(S @ Sn)
        ph.append(np.arctan2(Sn @ b2, Sn @ b1) % (2 * np.pi))
    lo = np.cos(np.radians(th))
    assert min(ca) >= lo - 1e-12 and max(ca) <= 1.0 + 1e-12
    assert sps.kstest(ca, sps.uniform(loc=lo, scale=1 - lo).cdf).pvalue > 1e-3
    assert sps.kstest(ph, sps.uniform(loc=0, scale=2 * np.pi).cdf).pvalue > 1e-3
    # theta = 180 covers the whole sphere uniformly: z ~ U(-1, 1)
    z = [oracle_mod.cone_move(S, u0, u1, 180) @ S for u0, u1 in rng.uniform(size=(3000, 2))]
    assert sps.kstest(z, sps.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3


def test_random_start_is_uniform_on_the_sphere(oracle_mod):
    """The random initial state is uniform on S^2 (the paper's increasing-T
    sweeps start from a disordered state).  Archimedes' hat-box theorem: a
    point is uniform on the unit sphere exactly when its projection on ANY
    fixed axis is U(-1, 1) and its azimuth about that axis is U(0, 2 pi),
    independent of the projection.  Checked on 64 x 64 x 32 = 131072 sites
    for the z axis and for two oblique axes, with unit length to 1e-15, zero
    mean and the isotropic second moment <S S^T> = I/3."""
    o = oracle_mod.OracleLattice(64, 64, 32, seed=12345, instance=3, init="random")
    S = o.spins()
    n = len(S)
    assert np.max(np.abs(np.linalg.norm(S, axis=1) - 1.0)) < 1e-15
    for axis in ((0.0, 0.0, 1.0), (1.0, 1.0, 1.0), (0.2, -0.9, 0.4)):
        a = np.asarray(axis) / np.linalg.norm(axis)
        b1 = np.cross(a, (1.0, 0.0, 0.0) if abs(a[0]) < 0.9 else (0.0, 1.0, 0.0))
        b1 /= np.linalg.norm(b1)
        b2 = np.cross(a, b1)
        proj = S @ a
        phi = np.arctan2(S @ b2, S @ b1) % (2 * np.pi)
        assert sps.kstest(proj, sps.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3, axis
        assert sps.kstest(phi, sps.uniform(loc=0, scale=2 * np.pi).cdf).pvalue > 1e-3, axis
        # projection and azimuth independent: no rank correlation
        assert abs(sps.spearmanr(proj, phi).statistic) < 5.0 / np.sqrt(n), axis
    # moments of the uniform distribution: <S> = 0, <S S^T> = I/3
    assert np.max(np.abs(S.mean(axis=0))) < 5.0 * np.sqrt(1.0 / 3.0 / n)
    assert np.max(np.abs(S.T @ S / n - np.eye(3) / 3.0)) < 5.0 * np.sqrt(4.0 / 45.0 / n)
    # the draw is keyed: another instance gives other spins
    o2 = oracle_mod.OracleLattice(64, 64, 32, seed=12345, instance=4, init="random")
    assert np.mean(np.abs(o2.spins() - S) > 1e-3) > 0.99


# --------------------------------------------------------------------------
# Energies (Eq. 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 4, 6), (4, 4, 4), (6, 2, 4)])
def test_local_energy_difference_equals_total_energy_difference(oracle_mod, shape):
    """dE from the local form of Eq. 2 equals the change of the bond-counted
    Hamiltonian, including lattices where the +/- neighbours coincide."""
    p = inputs.random_params(sum(shape))
    nx, ny, nz = shape
    L = oracle_mod.OracleLattice(nx, ny, nz, **p, init=None)
    n = nx * ny * nz
    S = inputs.random_unit_spins(n, 17)
    L.set_spins(S)
    rng = np.random.default_rng(4)
    for _ in range(40):
        i = int(rng.integers(0, n))
        new = inputs.random_unit_spins(1, int(rng.integers(0, 10 ** 6)))[0]
        e0 = L.total_energy()
        d_local = L.local_energy(i, new) - L.local_energy(i, S[i])
        S2 = S.copy()
        S2[i] = new
        L.set_spins(S2)
        e1 = L.total_energy()
        L.set_spins(S)
        assert abs((e1 - e0) - d_local) < 1e-12 * max(1.0, abs(e0))


def test_aligned_state_energies(oracle_mod):
    """Closed forms of the uniform state: E/N = -3J - Ku (S || e) and
    -3J + Kc f(S) - h.S in general."""
    L = oracle_mod.OracleLattice(4, 6, 8, J=1.3, Ku=0.02, Kc=0.0)
    assert abs(L.total_energy() / L.n - (-3 * 1.3 - 0.02)) < 1e-13
    d = np.array([1.0, 1.0, 1.0]) / np.sqrt(3)
    h = np.array([0.1, -0.2, 0.3])
    L = oracle_mod.OracleLattice(4, 4, 4, J=1.0, Ku=0.0, Kc=0.05, h=h, init_dir=d)
    assert abs(L.total_energy() / L.n - (-3.0 + 0.05 / 3 - h @ d)) < 1e-13


@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 4, 6), (4, 4, 4), (6, 2, 4)])
def test_antiperiodic_local_energy_difference(oracle_mod, shape):
    """The same identity on a lattice anti-periodic along z (the bond across
    the z boundary couples S_i to -S_j), including nz = 2, where both z
    neighbours of a site are the same site."""
    p = inputs.random_params(3 * sum(shape))
    nx, ny, nz = shape
    L = oracle_mod.OracleLattice(nx, ny, nz, **p, init=None, boundary_z="antiperiodic")
    n = nx * ny * nz
    S = inputs.random_unit_spins(n, 23)
    L.set_spins(S)
    rng = np.random.default_rng(5)
    for _ in range(40):
        i = int(rng.integers(0, n))
        new = inputs.random_unit_spins(1, int(rng.integers(0, 10 ** 6)))[0]
        e0 = L.total_energy()
        d_local = L.local_energy(i, new) - L.local_energy(i, S[i])
        S2 = S.copy()
        S2[i] = new
        L.set_spins(S2)
        e1 = L.total_energy()
        L.set_spins(S)
        assert abs((e1 - e0) - d_local) < 1e-12 * max(1.0, abs(e0))


def test_antiperiodic_closed_form_energies(oracle_mod):
    """Uniform state: the nx*ny bonds across the z boundary each cost 2J, so
    E = -3JN + 2J nx ny.  The uniform twist S(z) = (sin(pi z/nz), 0,
    cos(pi z/nz)) closes on itself through the boundary: every z bond has
    the angle pi/nz, so E = -J N (2 + cos(pi/nz))."""
    nx, ny, nz, J = 4, 6, 10, 1.3
    n = nx * ny * nz
    L = oracle_mod.OracleLattice(nx, ny, nz, J=J, boundary_z="antiperiodic")
    assert abs(L.total_energy() - (-3 * J * n + 2 * J * nx * ny)) < 1e-11
    z = np.repeat(np.arange(nz), nx * ny)
    S = np.stack([np.sin(np.pi * z / nz), np.zeros(n), np.cos(np.pi * z / nz)], axis=1)
    L.set_spins(S)
    assert abs(L.total_energy() - (-J * n * (2 + np.cos(np.pi / nz)))) < 1e-11
    P = oracle_mod.OracleLattice(nx, ny, nz, J=J)
    P.set_spins(S)
    # periodic: the bond from plane nz-1 back to plane 0 has the angle pi (nz-1)/nz
    ref = -J * n * 2 - J * nx * ny * ((nz - 1) * np.cos(np.pi / nz) + np.cos(np.pi * (nz - 1) / nz))
    assert abs(P.total_energy() - ref) < 1e-11


@pytest.mark.parametrize("shape,boundary", [((4, 4, 5), "open"), ((2, 4, 1), "open"), ((4, 2, 4), "periodic"),
                                            ((6, 4, 2), "antiperiodic")])
def test_masked_local_energy_difference(oracle_mod, shape, boundary):
    """The local/total identity with bond masks and an open or twisted z
    boundary (odd and unit thickness included)."""
    p = inputs.random_params(11 * sum(shape))
    nx, ny, nz = shape
    L = oracle_mod.OracleLattice(nx, ny, nz, **p, init=None, boundary_z=boundary)
    L.set_bond_masks(inputs.random_bond_masks(shape, 0.35, 8))
    n = nx * ny * nz
    S = inputs.random_unit_spins(n, 29)
    L.set_spins(S)
    rng = np.random.default_rng(6)
    for _ in range(40):
        i = int(rng.integers(0, n))
        new = inputs.random_unit_spins(1, int(rng.integers(0, 10 ** 6)))[0]
        e0 = L.total_energy()
        d_local = L.local_energy(i, new) - L.local_energy(i, S[i])
        S2 = S.copy()
        S2[i] = new
        L.set_spins(S2)
        e1 = L.total_energy()
        L.set_spins(S)
        assert abs((e1 - e0) - d_local) < 1e-12 * max(1.0, abs(e0))


def test_open_and_masked_closed_forms(oracle_mod):
    """Aligned state: an open film has 2N + nx ny (nz - 1) bonds, each worth
    -J; with masks, E = -J times the number of active bonds (counted from
    the masks); cutting every bond leaves no exchange."""
    nx, ny, nz, J = 6, 4, 5, 1.2
    n = nx * ny * nz
    L = oracle_mod.OracleLattice(nx, ny, nz, J=J, boundary_z="open")
    assert abs(L.total_energy() - (-J * (2 * n + nx * ny * (nz - 1)))) < 1e-11
    M = oracle_mod.OracleLattice(nx, ny, 4, J=J)
    mask = inputs.random_bond_masks((nx, ny, 4), 0.4, 3)
    M.set_bond_masks(mask)
    active = sum(int(b) for b in np.unpackbits(mask.reshape(-1, 1), axis=1)[:, 2:].ravel()) // 2
    assert abs(M.total_energy() - (-J * active)) < 1e-11
    M.set_bond_masks(np.zeros(nx * ny * 4, dtype=np.uint8))
    assert abs(M.total_energy()) < 1e-14
    # an odd periodic thickness is not bipartite: the sweeps refuse it
    P = oracle_mod.OracleLattice(4, 4, 3, J=J)
    assert P.sweep(1.0) == -1


# --------------------------------------------------------------------------
# Chain mechanics
# --------------------------------------------------------------------------

def test_theta_rule_all_accepted_and_all_rejected(oracle_mod):
    """With dE = 0 every move is accepted, theta climbs by 1 per sweep to 180;
    with T tiny in the ground state every move is rejected, theta falls to 1."""
    L = oracle_mod.OracleLattice(4, 4, 4, J=0.0, Ku=0.0, theta0_deg=170)
    thetas = []
    for _ in range(15):
        acc = L.sweep(1.0)
        assert acc == L.n
        thetas.append(L.counters()[0])
    assert thetas == [min(171 + k, 180) for k in range(15)]
    L = oracle_mod.OracleLattice(4, 4, 4, J=1.0, Ku=0.1, theta0_deg=5)
    for k in range(8):
        acc = L.sweep(1e-30)
        assert acc == 0
        assert L.counters() == (max(4 - k, 1), k + 1)


def test_theta_tie_goes_down(oracle_mod):
    """An acceptance rate of exactly 1/2 lowers theta (strict comparison)."""
    # A 2x2x2 lattice with J = 0 and a strong field: red sites start along the
    # field (any move raises E, nearly always rejected at tiny T), black sites
    # start against it (any move lowers E, always accepted): 4 of 8 accepted.
    L = oracle_mod.OracleLattice(2, 2, 2, J=0.0, h=(0, 0, 1.0), theta0_deg=20, init=None)
    S = np.zeros((8, 3))
    for i in range(8):
        x, y, z = i % 2, (i // 2) % 2, i // 4
        S[i, 2] = 1.0 if (x + y + z) % 2 == 0 else -1.0
    L.set_spins(S)
    assert L.sweep(1e-30) == 4
    assert L.counters()[0] == 19


# --------------------------------------------------------------------------
# Statistical physics pins
# --------------------------------------------------------------------------

def test_langevin_law_and_field_susceptibility(oracle_mod):
    """Free spins in a field: <S_z> = L(h/T) and chi_z = L'(h/T)/T."""
    T, hz = 0.5, 1.0
    L = oracle_mod.OracleLattice(8, 8, 8, J=0.0, h=(0, 0, hz), seed=21)
    L.sweep(T, 100)
    L.sweep(T, 4000, sample=True)
    mz = L.samples()[:, 3]
    mean, se = batch_mean_se(mz)
    assert abs(mean - langevin(hz / T)) < 4 * se + 1e-4, (mean, se)
    # chi_z = N var(m_z) / T (Eq. 6); its error bar from batch variances
    o = L.observables(T)
    assert abs(o["chi"][3] - L.n * np.var(mz) / T) < 1e-12
    chi_b = [L.n * np.var(b) / T for b in np.array_split(mz, 10)]
    expect = langevin_prime(hz / T) / T
    se_chi = np.std(chi_b, ddof=1) / np.sqrt(len(chi_b))
    assert abs(np.mean(chi_b) - expect) < 4 * se_chi, (np.mean(chi_b), expect, se_chi)


def test_curie_law(oracle_mod):
    """Free spins without a field: chi_x = 1/(3T)."""
    T = 0.7
    L = oracle_mod.OracleLattice(8, 8, 8, J=0.0, seed=22, init="random")
    L.sweep(T, 50)
    L.sweep(T, 2000, sample=True)
    m = L.samples()
    for a in (1, 2, 3):
        chi_b = [L.n * np.var(b) / T for b in np.array_split(m[:, a], 10)]
        se = np.std(chi_b, ddof=1) / np.sqrt(len(chi_b))
        assert abs(np.mean(chi_b) - 1.0 / (3 * T)) < 4 * se, (a, np.mean(chi_b), se)


def test_uniaxial_free_spins_quadrature(oracle_mod):
    """Free spins with uniaxial anisotropy: <S_z^2> from the Boltzmann integral."""
    T, Ku = 0.5, 1.0
    num = integrate.quad(lambda x: x * x * np.exp(Ku * x * x / T), 0, 1)[0]
    den = integrate.quad(lambda x: np.exp(Ku * x * x / T), 0, 1)[0]
    expect = num / den
    L = oracle_mod.OracleLattice(8, 8, 8, J=0.0, Ku=Ku, seed=23)
    L.sweep(T, 100)
    L.sweep(T, 2000, sample=True)
    sz2 = -L.samples()[:, 4] / Ku      # E/N = -Ku <S_z^2> for free spins
    mean, se = batch_mean_se(sz2)
    assert abs(mean - expect) < 4 * se + 1e-4, (mean, expect, se)


def test_infinite_temperature_isotropic_averages(oracle_mod):
    """At T -> infinity <(S.e)^2> = 1/3 and <f> = 1/5 (the zero of Eq. 4)."""
    L = oracle_mod.OracleLattice(8, 8, 8, J=0.0, Ku=1.0, eu=(1, 2, 2), Kc=1.0, seed=24,
                                 init="random")
    T = 1e7
    L.sweep(T, 200)
    assert L.counters()[0] == 180
    L.sweep(T, 800, sample=True)
    ean = L.samples()[:, 5]          # (E_uni + E_cub)/N = -<(S.e)^2> + <f>
    mean, se = batch_mean_se(ean)
    assert abs(mean - (-1.0 / 3.0 + 1.0 / 5.0)) < 4 * se + 1e-4


def test_low_temperature_equipartition(oracle_mod):
    """T -> 0: <E>/N = -3J - Ku + T (two quadratic transverse modes per spin)."""
    T = 0.01
    L = oracle_mod.OracleLattice(8, 8, 8, J=1.0, Ku=0.01, seed=25)
    L.sweep(T, 300)
    L.sweep(T, 1500, sample=True)
    mean, se = batch_mean_se(L.samples()[:, 4])
    assert abs(mean - (-3.0 - 0.01 + T)) < 0.05 * T + 4 * se


def test_spin_wave_magnetisation(oracle_mod):
    """T -> 0: 1 - <m_z> = (T / 2N) sum_k 1 / (J (3 - sum_a cos k_a) + Ku)."""
    Lx, Ku, T = 8, 0.1, 0.02
    k = 2 * np.pi * np.arange(Lx) / Lx
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    omega = (3 - np.cos(kx) - np.cos(ky) - np.cos(kz)) + Ku
    slope = np.sum(1.0 / omega) / (2 * Lx ** 3)
    L = oracle_mod.OracleLattice(Lx, Lx, Lx, J=1.0, Ku=Ku, seed=26)
    L.sweep(T, 300)
    L.sweep(T, 3000, sample=True)
    mean, se = batch_mean_se(1.0 - L.samples()[:, 3])
    assert abs(mean - slope * T) < 0.05 * slope * T + 4 * se, (mean, slope * T, se)


def test_paramagnet_above_tc_scales_as_inverse_sqrt_n(oracle_mod):
    """Above T_C (about 1.443 J for the simple-cubic Heisenberg model) <|m|>
    vanishes as N^-1/2: <|m|> sqrt(N) does not depend on the size."""
    T = 2.2
    res = {}
    for Lx in (8, 16):
        L = oracle_mod.OracleLattice(Lx, Lx, Lx, J=1.0, seed=27, init="random")
        L.sweep(T, 100)
        L.sweep(T, 600 if Lx == 8 else 300, sample=True)
        res[Lx] = np.mean(L.samples()[:, 0]) * np.sqrt(Lx ** 3)
    assert abs(res[8] / res[16] - 1.0) < 0.1, res
    # and below T_C the ordered moment survives at the larger size
    L = oracle_mod.OracleLattice(16, 16, 16, J=1.0, seed=28)
    L.sweep(1.0, 200, sample=True)
    assert np.mean(L.samples()[100:, 0]) > 0.5


def test_detailed_balance_against_heat_bath_2cubed(oracle_mod):
    """On 2x2x2 the Metropolis chain and an exact conditional (heat-bath)
    sampler reach the same <E> and <m_z^2>."""
    T = 1.0
    kw = dict(J=1.0, h=(0.0, 0.0, 0.3), seed=29, init="random")
    A = oracle_mod.OracleLattice(2, 2, 2, **kw)
    A.sweep(T, 500)
    A.sweep(T, 40000, sample=True)
    B = oracle_mod.OracleLattice(2, 2, 2, **dict(kw, seed=30))
    B.heatbath_sweep(T, 500)
    B.heatbath_sweep(T, 40000, sample=True)
    for col, f in ((4, lambda v: v), (3, lambda v: v * v)):
        ma, sa = batch_mean_se(f(A.samples()[:, col]), 40)
        mb, sb = batch_mean_se(f(B.samples()[:, col]), 40)
        assert abs(ma - mb) < 4 * np.hypot(sa, sb), (col, ma, mb, sa, sb)


def test_random_order_serial_matches_checkerboard(oracle_mod):
    """The serial algorithm (random site order) and the red/black order sample
    the same distribution."""
    T = 1.2
    kw = dict(J=1.0, Ku=0.05, Kc=0.03, h=(0.05, 0, 0), seed=31)
    A = oracle_mod.OracleLattice(6, 6, 6, **kw)
    A.sweep(T, 300)
    A.sweep(T, 4000, sample=True)
    B = oracle_mod.OracleLattice(6, 6, 6, **dict(kw, seed=32))
    B.serial_random_sweep(T, 300)
    B.serial_random_sweep(T, 4000, sample=True)
    for col in (0, 4):
        ma, sa = batch_mean_se(A.samples()[:, col])
        mb, sb = batch_mean_se(B.samples()[:, col])
        assert abs(ma - mb) < 4 * np.hypot(sa, sb), (col, ma, mb, sa, sb)


# --------------------------------------------------------------------------
# Constrained Monte Carlo (Table A2)
# --------------------------------------------------------------------------

def _ec(theta_deg, phi_deg):
    t, p = np.radians(theta_deg), np.radians(phi_deg)
    return np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])


def test_constrained_invariants(oracle_mod):
    """Every pair move keeps sum_i S_perp and each |S_i|."""
    eC = _ec(35, 20)
    L = oracle_mod.OracleLattice(6, 4, 4, J=1.0, Kc=0.3, Ku=0.1, eu=(1, 0, 0), seed=33,
                                 init=None)
    S = inputs.tilted_spins(L.n, 3, spread=0.5, axis=eC)
    L.set_spins(S)
    perp0 = S.sum(0) - (S.sum(0) @ eC) * eC
    acc = 0
    for _ in range(100):
        acc += L.constrained_sweep(0.9, eC)
    S1 = L.spins()
    perp1 = S1.sum(0) - (S1.sum(0) @ eC) * eC
    assert acc > 1000
    assert np.max(np.abs(perp1 - perp0)) < 1e-12 * L.n
    assert np.max(np.abs(np.linalg.norm(S1, axis=1) - 1.0)) < 1e-12
    assert S1.sum(0) @ eC > 0


@pytest.mark.parametrize("theta,phi", [(30, 0), (60, 0), (50, 45), (90, 45)])
def test_constrained_low_temperature_cubic_energy(oracle_mod, theta, phi):
    """T -> 0 with the moment held along e_C(theta, phi): the cubic energy per
    spin is Kc f(e_C), i.e. Kc sin^2 cos^2 at phi = 0 and
    Kc (sin^4/4 + sin^2 cos^2) at phi = 45 degrees."""
    Kc, T = 0.05, 0.004
    eC = _ec(theta, phi)
    t = np.radians(theta)
    expect = Kc * (np.sin(t) ** 2 * np.cos(t) ** 2 if phi == 0
                   else np.sin(t) ** 4 / 4 + np.sin(t) ** 2 * np.cos(t) ** 2)
    L = oracle_mod.OracleLattice(6, 6, 6, J=1.0, Kc=Kc, seed=34, init_dir=eC)
    L.constrained_sweep(T, eC, 100)
    L.constrained_sweep(T, eC, 300, sample=True)
    ean = L.samples()[:, 5]
    assert abs(np.mean(ean) - expect) < 2e-4
    # the moment stays along e_C
    m = L.samples()[-1, 1:4]
    assert np.linalg.norm(m - (m @ eC) * eC) < 1e-10
    # the torque matches the uniform state's: e_C x (-Kc grad f(e_C))
    x, y, z = eC
    g = -Kc * 2 * np.array([x * (y * y + z * z), y * (x * x + z * z), z * (x * x + y * y)])
    o = L.observables(T)
    assert np.allclose(o["mean_torque"], np.cross(eC, g), atol=5e-4)


def test_constrained_hard_axis_energy(oracle_mod):
    """Cubic hard axis (body diagonal) at T -> 0: E_anis / N = Kc / 3."""
    Kc, T = 0.05, 0.004
    eC = np.ones(3) / np.sqrt(3)
    L = oracle_mod.OracleLattice(6, 6, 6, J=1.0, Kc=Kc, seed=35, init_dir=eC)
    L.constrained_sweep(T, eC, 100)
    L.constrained_sweep(T, eC, 200, sample=True)
    assert abs(np.mean(L.samples()[:, 5]) - Kc / 3) < 2e-4


def test_constrained_along_easy_axis_matches_unconstrained(oracle_mod):
    """With e_C on the easy axis the constraint is inactive on average: the
    constrained and standard chains give the same <E>."""
    T = 0.8
    kw = dict(J=1.0, Ku=0.3, seed=36)
    A = oracle_mod.OracleLattice(6, 6, 6, **kw)
    A.constrained_sweep(T, (0, 0, 1), 300)
    A.constrained_sweep(T, (0, 0, 1), 4000, sample=True)
    B = oracle_mod.OracleLattice(6, 6, 6, **dict(kw, seed=37))
    B.sweep(T, 300)
    B.sweep(T, 4000, sample=True)
    ma, sa = batch_mean_se(A.samples()[:, 4])
    mb, sb = batch_mean_se(B.samples()[:, 4])
    assert abs(ma - mb) < 4 * np.hypot(sa, sb), (ma, mb, sa, sb)


def test_once_per_sweep_ml_matches_exact_serial(oracle_mod):
    """M_L taken once per sweep (the parallel scheme) samples the same <E>
    and <E_anis> as the serial scheme that updates M_L after every pair."""
    T = 0.7
    eC = _ec(45, 0)
    kw = dict(J=1.0, Kc=0.2, init_dir=eC)
    A = oracle_mod.OracleLattice(6, 6, 6, seed=38, **kw)
    A.constrained_sweep(T, eC, 300)
    A.constrained_sweep(T, eC, 4000, sample=True)
    B = oracle_mod.OracleLattice(6, 6, 6, seed=39, **kw)
    B.constrained_sweep(T, eC, 300, exact_serial=True)
    B.constrained_sweep(T, eC, 4000, sample=True, exact_serial=True)
    for col in (4, 5):
        ma, sa = batch_mean_se(A.samples()[:, col])
        mb, sb = batch_mean_se(B.samples()[:, col])
        assert abs(ma - mb) < 4 * np.hypot(sa, sb), (col, ma, mb, sa, sb)
