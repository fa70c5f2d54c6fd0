"""Host-side logic of the measurement protocols (no GPU)."""
import numpy as np

from paper_2103_03517_amd import protocols as P


def test_block_stats_from_cumulative_reads_equal_reset_blocks():
    """Blocks recovered from running sums read at the block ends equal the
    blocks of accumulators reset at each block start."""
    rng = np.random.default_rng(0)
    x = rng.normal(0.5, 0.1, (600, 4))
    e = rng.normal(-3.0, 0.1, 600)
    reads, blocks = [], []
    for b in range(6):
        ns = (b + 1) * 100
        reads.append({"samples": ns, "mean_m": x[:ns].mean(0).tolist(),
                      "var_m": x[:ns].var(0).tolist(), "mean_E": float(e[:ns].mean())})
        xb, eb = x[b * 100:ns], e[b * 100:ns]
        blocks.append({"mean_m": xb.mean(0), "var_m": xb.var(0), "mean_E": float(eb.mean())})
    r1 = P.block_stats_from_reads(reads, 1000, 0.7)
    r2 = P._block_stats(blocks, 1000, 0.7)
    assert np.allclose(r1["m"], r2["m"], rtol=1e-12)
    assert np.allclose(r1["se_m"], r2["se_m"], rtol=1e-8)
    assert np.allclose(r1["chi"], r2["chi"], rtol=1e-8)
    assert abs(r1["E"] - r2["E"]) < 1e-12
    # whole-window variance = mean within-block variance + variance of block means
    assert np.allclose(np.asarray(r1["chi"]) * 0.7 / 1000, x.var(0), rtol=1e-9)


def test_batched_workload_recipe():
    jobs = P.c4_jobs()
    assert len(jobs) == 64 and jobs == P.c4_jobs()
    edges = {e for e, _ in jobs}
    assert edges <= {48, 64, 80, 96, 128} and len(edges) == 5
    assert all(0.05 <= t < 1.7 for _, t in jobs)
    assert P.c4_jobs(seed=5) != jobs


def test_compare_precisions_units():
    def job(m, se_m, mz, se_mz, E, se_E, chi=1.0, se_chi=0.1):
        return {"edge": 8, "T": 1.0, "m": [m, 0, 0, mz], "se_m": [se_m, 0, 0, se_mz], "E": E, "se_E": se_E,
                "chi": [chi, 0, 0, 0], "se_chi": [se_chi, 0, 0, 0]}
    a = [job(0.5, 3e-4, 0.5, 4e-4, -2.0, 1e-4)]
    b = [job(0.5005, 4e-4, 0.5, 3e-4, -2.0001, 1e-4, chi=1.2)]
    r = P.compare_precisions(a, b)[0]
    assert abs(r["dm"] - 5e-4) < 1e-12
    assert abs(r["dm_over_se"] - 1.0) < 1e-9
    assert abs(r["dE_over_se"] - 1e-4 / np.hypot(1e-4, 1e-4)) < 1e-9
    assert abs(r["dchi_over_se"] - 0.2 / np.hypot(0.1, 0.1)) < 1e-9
    assert r["resolves_1e-3"] is False and r["pass"] is True    # 3 SE = 1.5e-3
    # m_z is reported, not gated
    b = [job(0.5005, 4e-4, 0.51, 3e-4, -2.0001, 1e-4)]
    r = P.compare_precisions(a, b)[0]
    assert r["dmz_over_se"] > 3 and r["pass"] is True
    # an unresolvable job (3 SE >= 1e-3) outside 1e-3 passes on the 3 SE rule
    # alone; a resolvable one outside 1e-3 fails (it is then also beyond
    # 3 SE: the 1e-3 rule adds nothing where it applies)
    r = P.compare_precisions([job(0.5, 5e-4, 0.5, 0, -2.0, 1e-4)], [job(0.5011, 1e-4, 0.5, 0, -2.0, 1e-4)])[0]
    assert r["resolves_1e-3"] is False and r["dm_over_se"] <= 3 and r["pass"] is True
    r = P.compare_precisions([job(0.5, 2e-4, 0.5, 0, -2.0, 1e-4)], [job(0.50105, 1.5e-4, 0.5, 0, -2.0, 1e-4)])[0]
    assert r["resolves_1e-3"] is True and r["dm_over_se"] > 3 and r["pass"] is False
    # energies beyond 3 SE fail
    r = P.compare_precisions([job(0.5, 2e-4, 0.5, 0, -2.0, 1e-4)], [job(0.5, 2e-4, 0.5, 0, -2.001, 1e-4)])[0]
    assert r["dE_over_se"] > 3 and r["pass"] is False


def test_serving_job_schedule_and_stream():
    from paper_2103_03517_amd import serving as S
    j = S.Job(16, 1.0, equil=30, samples=100, block=25)
    assert j.total == 130 and not j.sampling() and j.next_event() == 30
    j.done = 30
    assert j.sampling() and j.next_event() == 25
    j.done = 42
    assert j.next_event() == 13
    import pytest
    with pytest.raises(ValueError):
        S.Job(16, 1.0, samples=90, block=25)
    a = S.poisson_jobs(rate=20, seconds=10)
    b = S.poisson_jobs(rate=20, seconds=10)
    assert [(x.edge, x.T, x.arrival) for x in a] == [(x.edge, x.T, x.arrival) for x in b]
    assert 150 < len(a) < 250
    gaps = np.diff([0.0] + [x.arrival for x in a])
    assert abs(gaps.mean() - 1 / 20) < 0.015
    assert {x.instance for x in a} == set(range(len(a)))


def test_torque_integral_gives_the_cubic_energy():
    """Synthetic T = 0 torques integrate to Kc f(e_C(theta)) along both scan
    planes, and the amplitude fit recovers Kc on the 10-degree grid."""
    from paper_2103_03517_amd import anisotropy as A
    Kc = 0.05
    for phi in (0.0, 45.0, 30.0):
        th = np.arange(0.0, 90.01, 0.5)
        tau = np.array([A.cubic_torque(t, phi, Kc) for t in th])
        F = A.free_energy_from_torque(th, tau, phi)
        ref = Kc * (A.cubic_f(th, phi) - A.cubic_f(0.0, phi))
        assert np.max(np.abs(F - ref)) < 2e-5 * Kc * 10, phi
        # the torque is perpendicular to e_C; in the symmetry planes phi = 0
        # and 45 degrees (df/dphi = 0) it lies along e_phi
        for t, v in zip(th[::20], tau[::20]):
            assert abs(np.dot(v, A.e_c(t, phi))) < 1e-15
            if phi in (0.0, 45.0):
                assert np.linalg.norm(v - np.dot(v, A.e_phi(phi)) * A.e_phi(phi)) < 1e-12
    grid = list(range(0, 91, 10))
    curves = [(grid, A.free_energy_from_torque(grid, [A.cubic_torque(t, p, Kc) for t in grid], p), p)
              for p in (0.0, 45.0)]
    assert abs(A.fit_cubic_amplitude(curves) / Kc - 1) < 0.03


def test_callen_callen_exponent_recovered():
    from paper_2103_03517_amd import anisotropy as A
    m = np.array([0.95, 0.9, 0.8, 0.6])
    assert abs(A.callen_callen_exponent(0.05 * m ** 10, 0.05, m) - 10.0) < 1e-12
    assert abs(A.callen_callen_exponent(0.05 * m ** 3, 0.05, m) - 3.0) < 1e-12


def test_constrained_reference_torque_integrates_to_free_energy():
    """End to end on the CPU reference: constrained chains at T -> 0 along a
    grid of e_C; the integral of their mean torque reproduces Kc f(e_C) -
    Kc f(z).  Pins the torque sign and the integration together."""
    from oracle import oracle as O
    from paper_2103_03517_amd import anisotropy as A
    Kc, T = 0.05, 0.002
    th = list(range(0, 91, 5))
    tau = []
    for t in th:
        e = A.e_c(t, 0.0)
        o = O.OracleLattice(4, 4, 4, J=1.0, Kc=Kc, seed=3, init="aligned", init_dir=tuple(e))
        o.constrained_sweep(T, tuple(e), 40)
        o.constrained_sweep(T, tuple(e), 60, sample=True)
        tau.append(o.observables(T)["mean_torque"])
    F = A.free_energy_from_torque(th, tau, 0.0)
    ref = Kc * A.cubic_f(np.array(th, dtype=float), 0.0)
    assert np.max(np.abs(F - ref)) < 0.03 * Kc / 4, (F, ref)
    assert abs(F[9] - Kc / 4) < 0.03 * Kc / 4          # theta = 45: the <110> direction


def test_wall_fit_recovers_synthetic_profiles():
    """tanh profiles placed anywhere in an anti-periodic box (also across its
    boundary), with noise, are fitted back."""
    from paper_2103_03517_amd import walls as W
    rng = np.random.default_rng(2)
    nz = 256
    for z0, d, m in [(128.0, 20.0, 0.9), (3.5, 12.0, 0.7), (250.2, 30.0, 0.5), (60.0, 8.0, 0.95)]:
        z = np.arange(nz)
        # the twisted profile: F(z0 + u + k nz) = (-1)^k F(z0 + u), u in [-nz/2, nz/2)
        k = np.floor((z - z0 + nz / 2) / nz)
        u = z - z0 - k * nz
        f = (-1.0) ** k * m * np.tanh(-np.pi * u / d) + rng.normal(0, 0.01, nz)
        mm, zz, dd = W.fit_wall(f)
        assert abs(mm - m) < 0.01, (z0, mm)
        assert abs(dd / d - 1) < 0.03, (z0, dd)
        dz = (zz - z0 + nz / 2) % nz - nz / 2
        assert abs(dz) < 0.5, (z0, zz)


def test_reference_wall_width_at_low_temperature():
    """The CPU reference relaxes a sharp wall in an anti-periodic 2x2x64
    column at T -> 0 to the width pi sqrt(J/(2 Ku)) of the continuum Bloch
    wall (discreteness corrections are O(1/Delta^2) for Delta of ~10 sites)."""
    from oracle import oracle as O
    from paper_2103_03517_amd import walls as W
    J, Ku = 1.0, 0.05
    o = O.OracleLattice(2, 2, 64, J=J, Ku=Ku, seed=2, boundary_z="antiperiodic", init=None)
    o.set_spins(W.initial_wall(2, 2, 64))
    o.sweep(0.002, 3000)
    prof = o.spins().reshape(64, 4, 3).mean(axis=1)[:, 2]
    m, z0, d = W.fit_wall(prof)
    d0 = W.zero_temperature_width(J, Ku)
    assert abs(m - 1) < 0.01
    assert abs(d / d0 - 1) < 0.03, (d, d0)
    assert abs(W.exchange_stiffness(Ku, d) - J / 2) < 0.03 * J


def test_reference_uniaxial_torque_gives_Ku_sin2():
    """Uniaxial term along z on the CPU reference at T -> 0: the integrated
    torque is Ku sin^2 theta and the amplitude fit returns Ku."""
    from oracle import oracle as O
    from paper_2103_03517_amd import anisotropy as A
    Ku, T = 0.03, 0.002
    th = [0, 15, 30, 45, 60, 75, 90]
    scan = []
    for t in th:
        e = A.e_c(t, 0.0)
        o = O.OracleLattice(4, 4, 4, J=1.0, Ku=Ku, eu=(0, 0, 1), seed=5, init="aligned", init_dir=tuple(e))
        o.constrained_sweep(T, tuple(e), 40)
        o.constrained_sweep(T, tuple(e), 60, sample=True)
        ob = o.observables(T)
        scan.append({"theta": t, "phi": 0.0, "T": T, "E_anis": ob["mean_Eanis"], "torque": ob["mean_torque"]})
    res = A.analyse(scan, {}, Ku, kind="uniaxial")
    row = res["rows"][0]
    assert abs(row["K_torque"] / Ku - 1) < 0.03, row
    assert abs(row["K_energy"] / Ku - 1) < 0.03, row


def test_voronoi_film_masks():
    """Grain maps cover the plane, the mean grain area matches the requested
    diameter, and the masks cut exactly the bonds between grains, at both
    ends, keeping every z bond."""
    from paper_2103_03517_amd import films as F
    g, ng = F.voronoi_grains(128, 96, 16, seed=1)
    assert g.shape == (96, 128) and len(np.unique(g)) <= ng
    assert abs(F.grain_areas(g).mean() / (np.pi * 16 ** 2 / 4) - 1) < 0.15
    m = F.grain_bond_masks(g, 3).reshape(3, 96, 128)
    for z in range(3):
        for y in range(0, 96, 7):
            for x in range(0, 128, 5):
                a = int(m[z, y, x])
                assert ((a >> 1) & 1) == (g[y, x] == g[y, (x + 1) % 128])
                assert ((a >> 3) & 1) == (g[y, x] == g[(y + 1) % 96, x])
                assert ((a >> 1) & 1) == (int(m[z, y, (x + 1) % 128]) & 1)
                assert ((a >> 3) & 1) == ((int(m[z, (y + 1) % 96, x]) >> 2) & 1)
                assert (a >> 4) & 3 == 3


def test_multi_bloch_fit_recovers_a_two_term_mixture():
    from paper_2103_03517_amd import films as F
    T = np.linspace(0.05, 1.5, 30)
    w, tc, b = np.array([0.3, 0.7]), np.array([0.9, 1.4]), np.array([0.34, 0.36])
    m = F.multi_bloch(T, w, tc, b)
    fw, ftc, fb, mean_tc, rms = F.fit_multi_bloch(T, m, 2, seed=1)
    assert rms < 2e-3
    assert abs(mean_tc - np.dot(w, tc)) < 0.03
    # one Bloch term: Eq. 3
    m1 = F.bloch(T, 1.44, 0.34)
    fw, ftc, fb, mean_tc, rms = F.fit_multi_bloch(T, m1, 1)
    assert abs(ftc[0] - 1.44) < 0.01 and abs(fb[0] - 0.34) < 0.01


def test_blocking_error_of_a_correlated_series():
    """AR(1) block means with correlation 0.9: the naive batch-means error is
    too small by about sqrt((1 + 0.9)/(1 - 0.9)) = 4.4; the blocking error
    recovers most of it, and for independent blocks it stays at the naive one."""
    from paper_2103_03517_amd.protocols import blocking_se
    rng = np.random.default_rng(4)
    n, rho = 4096, 0.9
    x = np.empty(n)
    x[0] = rng.normal()
    for i in range(1, n):
        x[i] = rho * x[i - 1] + np.sqrt(1 - rho ** 2) * rng.normal()
    naive = x.std(ddof=1) / np.sqrt(n)
    true = np.sqrt((1 + rho) / (1 - rho)) / np.sqrt(n)
    b = float(blocking_se(x[:, None])[0])
    assert naive < 0.4 * true and 0.75 * true < b < 1.5 * true
    y = rng.normal(size=(4096, 1))
    assert abs(float(blocking_se(y)[0]) / (y.std(ddof=1) / 64) - 1) < 0.35


def test_direct_torque_fit_has_no_quadrature_error():
    """On a coarse 30-degree grid the integrated route underestimates the
    amplitude by ~9 %; the direct torque fit returns it exactly."""
    from paper_2103_03517_amd import anisotropy as A
    Ku = 0.01
    rows = []
    for t in (0, 30, 60, 90):
        tau = np.array([0.0, -Ku * np.sin(2 * np.radians(t)), 0.0])    # -tau.e_phi = Ku sin 2 theta at phi = 0
        rows.append({"theta": t, "phi": 0.0, "T": 0.1, "E_anis": Ku * np.sin(np.radians(t)) ** 2,
                     "torque": tau.tolist()})
    res = A.analyse(rows, {}, Ku, kind="uniaxial")["rows"][0]
    assert abs(res["K_torque"] / Ku - 1) < 1e-12
    assert 0.85 < res["K_torque_integrated"] / Ku < 0.95
    for phi in (0.0, 45.0):
        rows = [{"theta": t, "phi": phi, "T": 0.1, "E_anis": 0.05 * A.cubic_f(t, phi),
                 "torque": A.cubic_torque(t, phi, 0.05).tolist()} for t in range(0, 91, 10)]
        assert abs(A.analyse(rows, {}, 0.05)["rows"][0]["K_torque"] / 0.05 - 1) < 1e-12


# --------------------------------------------------------------------------
# Eq. 4: the reduced anisotropy from the easy-axis energy of standard sweeps
# --------------------------------------------------------------------------

def test_eq4_is_one_for_spins_frozen_along_the_easy_axis():
    """T -> 0 limit: every spin along the easy axis gives k_u = k_c = 1
    (energies of aligned reference lattices, not a retyped formula)."""
    from oracle import oracle as O
    from paper_2103_03517_amd import anisotropy as A
    Ku, Kc = 0.03, 0.05
    o = O.OracleLattice(6, 6, 6, J=1.0, Ku=Ku, eu=(0.0, 0.6, 0.8), seed=1, init="aligned",
                        init_dir=(0.0, 0.6, 0.8))
    assert abs(A.k_uniaxial(o.observables(1.0)["E_uni"] / o.n, Ku) - 1.0) < 1e-14
    for axis in ((0, 0, 1), (1, 0, 0), (0, -1, 0)):
        o = O.OracleLattice(6, 6, 6, J=1.0, Kc=Kc, seed=1, init="aligned", init_dir=axis)
        assert abs(A.k_cubic(o.observables(1.0)["E_cub"] / o.n, Kc) - 1.0) < 1e-14
    # and the hard directions give the other end of the scale: k = 1 - 3/2
    # (uniaxial, perpendicular to e) and 1 - 5/3 (cubic, body diagonal)
    o = O.OracleLattice(6, 6, 6, J=1.0, Ku=Ku, eu=(0.0, 0.6, 0.8), seed=1, init="aligned",
                        init_dir=(1.0, 0.0, 0.0))
    assert abs(A.k_uniaxial(o.observables(1.0)["E_uni"] / o.n, Ku) - (1.0 - 1.5)) < 1e-14
    o = O.OracleLattice(6, 6, 6, J=1.0, Kc=Kc, seed=1, init="aligned", init_dir=(1, 1, 1))
    assert abs(A.k_cubic(o.observables(1.0)["E_cub"] / o.n, Kc) - (1.0 - 5.0 / 3.0)) < 1e-14


def test_eq4_is_zero_for_isotropic_spins():
    """T -> infinity limit: spins uniform on the sphere (<(S.e)^2> = 1/3,
    <f> = 1/5) give k_u = k_c = 0, within five standard errors of the
    131072-spin sample (the spread of each per-spin value is taken from the
    sample itself)."""
    from oracle import oracle as O
    from paper_2103_03517_amd import anisotropy as A
    Ku, Kc = 0.02, 0.05
    e = np.array([0.36, 0.48, 0.8])
    o = O.OracleLattice(64, 64, 32, J=1.0, Ku=Ku, eu=tuple(e), Kc=Kc, seed=5, init="random")
    ob = o.observables(1.0)
    S = o.spins()
    n = o.n
    ku = A.k_uniaxial(ob["E_uni"] / n, Ku)
    kc = A.k_cubic(ob["E_cub"] / n, Kc)
    sd_u = np.std(1.5 * (S @ e) ** 2)
    x2, y2, z2 = (S ** 2).T
    sd_c = np.std(5.0 * (x2 * y2 + x2 * z2 + y2 * z2))
    assert abs(ku) < 5 * sd_u / np.sqrt(n), (ku, sd_u)
    assert abs(kc) < 5 * sd_c / np.sqrt(n), (kc, sd_c)


def test_eq4_free_spins_match_boltzmann_integrals():
    """Non-interacting spins (J = 0) at finite temperature: the chain's k_u
    equals <P_2(cos theta)> of the Boltzmann weight exp(Ku cos^2 theta / T),
    and its k_c equals 1 - 5 <f> of exp(-Kc f / T) over the sphere (scipy
    quadrature), within four standard errors."""
    from oracle import oracle as O
    from paper_2103_03517_amd import anisotropy as A
    from scipy import integrate
    from tests.stats import batch_mean_se
    T = 0.5
    Ku = 1.0
    w = lambda x: np.exp(Ku * x * x / T)
    p2 = integrate.quad(lambda x: 0.5 * (3 * x * x - 1) * w(x), 0, 1)[0] / integrate.quad(w, 0, 1)[0]
    o = O.OracleLattice(8, 8, 8, J=0.0, Ku=Ku, seed=31, init="aligned")
    o.sweep(T, 100)
    o.sweep(T, 2000, sample=True)
    mean, se = batch_mean_se(A.k_uniaxial(o.samples()[:, 5], Ku))
    assert abs(mean - p2) < 4 * se + 1e-4, (mean, p2, se)

    Kc = 1.0

    def f(th, ph):
        s, c = np.sin(th), np.cos(th)
        x2, y2, z2 = (s * np.cos(ph)) ** 2, (s * np.sin(ph)) ** 2, c * c
        return x2 * y2 + x2 * z2 + y2 * z2

    wz = integrate.dblquad(lambda th, ph: np.exp(-Kc * f(th, ph) / T) * np.sin(th), 0, 2 * np.pi, 0, np.pi)[0]
    wf = integrate.dblquad(lambda th, ph: f(th, ph) * np.exp(-Kc * f(th, ph) / T) * np.sin(th),
                           0, 2 * np.pi, 0, np.pi)[0]
    kc_exact = 1.0 - 5.0 * wf / wz
    o = O.OracleLattice(8, 8, 8, J=0.0, Kc=Kc, seed=32, init="aligned")
    o.sweep(T, 100)
    o.sweep(T, 2000, sample=True)
    mean, se = batch_mean_se(A.k_cubic(o.samples()[:, 5], Kc))
    assert abs(mean - kc_exact) < 4 * se + 1e-4, (mean, kc_exact, se)


def test_torque_amplitude_error_propagation():
    """fit_torque_amplitude_se: the fit equals fit_torque_amplitude, and its
    error is the exact linear propagation of independent row errors (checked
    against the spread of refits over resampled rows)."""
    from paper_2103_03517_amd import anisotropy as A
    rng = np.random.default_rng(3)
    Kc = 0.05
    rows = []
    for phi in (0.0, 45.0):
        for t in range(0, 91, 10):
            tau = A.cubic_torque(t, phi, Kc)
            rows.append({"theta": float(t), "phi": phi, "torque": tau.tolist(), "g_se": 1e-4})
    K, se = A.fit_torque_amplitude_se(rows, A.cubic_df)
    assert abs(K - A.fit_torque_amplitude(rows, A.cubic_df)) < 1e-15
    assert abs(K / Kc - 1) < 1e-12
    fits = []
    for _ in range(2000):
        rr = []
        for r in rows:
            g = 1e-4 * rng.normal()
            ep = A.e_phi(r["phi"])
            rr.append(dict(r, torque=(np.asarray(r["torque"]) - g * ep).tolist()))
        fits.append(A.fit_torque_amplitude(rr, A.cubic_df))
    assert abs(np.std(fits) / se - 1) < 0.08, (np.std(fits), se)
