"""Measurement protocols built on the sweep library.

``mt_sweep`` runs the increasing-temperature protocol of Sec. 3 (state carried
from one temperature to the next): at each T, equilibration sweeps, then
sampled sweeps split into blocks.  Each block is averaged on the device (the
accumulators are reset between blocks), so the standard errors come from
batch means, which account for the autocorrelation of the chain.  It
reports m(T) (Eq. 3's order parameter), E/N and the susceptibilities of
Eq. 6.

``constrained_scan`` runs the constrained algorithm (Table A2) over a grid of
constraint directions and temperatures and reports the anisotropy energy and
torque per spin.

``batched_mt`` runs many independent m(T) jobs (one lattice and one
temperature each, of uneven sizes) as one batch: equilibration, then sampled
sweeps whose block statistics come from the cumulative accumulators read at
the block ends (no resets, so the jobs need not be aligned).

    python -m paper_2103_03517_amd.protocols mt --precision 32 --size 256
"""
import argparse
import json
import math
import sys

import numpy as np

from . import Batch, Lattice


def blocking_se(x):
    """Standard error of the mean of a correlated series of equal-length
    block means, by the blocking method of Flyvbjerg and Petersen (J. Chem.
    Phys. 91, 461, 1989): merge neighbouring blocks pairwise while at least
    four remain and keep the largest batch-means error over the levels, so
    blocks shorter than the autocorrelation time do not shrink it.  x has
    the blocks along axis 0."""
    x = np.asarray(x, dtype=float)
    if len(x) < 2:
        return np.full(x.shape[1:], np.nan)
    best = x.std(axis=0, ddof=1) / math.sqrt(len(x))
    while len(x) >= 8:
        k = len(x) // 2
        x = 0.5 * (x[0:2 * k:2] + x[1:2 * k:2])
        best = np.maximum(best, x.std(axis=0, ddof=1) / math.sqrt(len(x)))
    return best


def _block_stats(blocks, n, T):
    """Combine equal-length blocks: means, standard errors (blocking
    analysis of the block means), and the susceptibility of the whole
    window (within-block variance plus the variance of the block means)."""
    mean_m = np.array([b["mean_m"] for b in blocks])        # (nb, 4)
    var_m = np.array([b["var_m"] for b in blocks])
    mean_e = np.array([b["mean_E"] for b in blocks])
    nb = len(blocks)
    m = mean_m.mean(axis=0)
    se_m = blocking_se(mean_m)
    var_tot = var_m.mean(axis=0) + mean_m.var(axis=0)
    chi = n * var_tot / T
    chi_b = n * (var_m + (mean_m - m) ** 2) / T
    se_chi = blocking_se(chi_b)
    e = float(mean_e.mean())
    se_e = float(blocking_se(mean_e[:, None])[0])
    out = {"T": T, "m": m.tolist(), "se_m": se_m.tolist(), "E": e, "se_E": se_e,
           "chi": chi.tolist(), "se_chi": se_chi.tolist(), "blocks": nb}
    if all("mean_Eanis" in b for b in blocks):
        ea = np.array([b["mean_Eanis"] for b in blocks])
        out["Eanis"] = float(ea.mean())
        out["se_Eanis"] = float(blocking_se(ea[:, None])[0])
    # stationarity: the first and second halves of the window, each with its
    # own blocking error, differ by stat_z standard errors (|m| and E/N); a
    # chain still relaxing from its start shows a large |stat_z|
    if nb >= 8:
        h = nb // 2
        for key, x in (("stat_z_m", mean_m[:, 0]), ("stat_z_E", mean_e)):
            a, b = x[:h], x[h:2 * h]
            se = math.hypot(blocking_se(a[:, None])[0], blocking_se(b[:, None])[0])
            out[key] = float((a.mean() - b.mean()) / se) if se > 0 else 0.0
    return out


def mt_sweep(temps, size=256, precision=32, equil=2000, samples=4000, block=200, seed=7,
             init="random", J=1.0, Ku=0.005, eu=(0.0, 0.0, 1.0), instance=0, log=None):
    """m(T), E(T), chi(T) along an ascending temperature list, one lattice."""
    g = Lattice(size, size, size, precision=precision, J=J, Ku=Ku, eu=eu, seed=seed,
                instance=instance, init=init)
    out = []
    for T in temps:
        g.sweep(T, equil)
        blocks = []
        for _ in range(max(samples // block, 1)):
            g.reset_stats()
            g.sweep(T, block, sample=True)
            blocks.append(g.observables())
        r = _block_stats(blocks, g.n, T)
        r["theta_deg"] = blocks[-1]["theta_deg"]
        out.append(r)
        if log:
            log(f"T={T:.3f} m={r['m'][0]:.6f}+-{r['se_m'][0]:.1e} chi_l={r['chi'][0]:.4g} "
                f"E/N={r['E']:.6f} theta={r['theta_deg']}")
    g.close()
    return out


def mt_gate(temps, size=256, equil=2000, samples=8000, block=200, init="aligned", seeds=(7, 8), Ku=0.005,
            log=None):
    """FP32 against FP64 along the increasing-temperature protocol: mt_sweep
    at both precisions with independent Philox keys (seeds), and per
    temperature |dm| of <|m|>, its z-score, the z-scores of <E>/N and chi_l,
    the runs' stationarity z-scores (first against second half of each
    window) and the gate of compare_precisions."""
    r32 = mt_sweep(temps, size=size, precision=32, equil=equil, samples=samples, block=block, seed=seeds[0],
                   init=init, Ku=Ku, log=log)
    r64 = mt_sweep(temps, size=size, precision=64, equil=equil, samples=samples, block=block, seed=seeds[1],
                   init=init, Ku=Ku, log=log)
    for r in r32 + r64:
        r["edge"] = size
    rows = compare_precisions(r32, r64)
    for c, a, b in zip(rows, r32, r64):
        c.update(m32=a["m"][0], m64=b["m"][0], E32=a["E"], E64=b["E"], chi32=a["chi"][0], chi64=b["chi"][0])
    return {"fp32": r32, "fp64": r64, "compare": rows}


def block_stats_from_reads(reads, n, T):
    """Block statistics from cumulative observables read at the end of each
    block: block sums are differences of the running sums (n mean, n (var +
    mean^2)) between consecutive reads."""
    blocks = []
    prev = None
    for r in reads:
        ns = r["samples"]
        m1 = ns * np.asarray(r["mean_m"])
        m2 = ns * (np.asarray(r["var_m"]) + np.asarray(r["mean_m"]) ** 2)
        e1 = ns * r["mean_E"]
        a1 = ns * r.get("mean_Eanis", 0.0)
        if prev is not None:
            k = ns - prev[0]
            mean = (m1 - prev[1]) / k
            var = (m2 - prev[2]) / k - mean ** 2
            blocks.append({"mean_m": mean, "var_m": np.maximum(var, 0.0), "mean_E": (e1 - prev[3]) / k,
                           "mean_Eanis": (a1 - prev[4]) / k})
        else:
            blocks.append({"mean_m": m1 / ns, "var_m": np.asarray(r["var_m"]), "mean_E": r["mean_E"],
                           "mean_Eanis": r.get("mean_Eanis", 0.0)})
        prev = (ns, m1, m2, e1, a1)
    return _block_stats(blocks, n, T)


def c4_jobs(count=64, seed=4, edges=(48, 64, 80, 96, 128), t_lo=0.05, t_hi=1.7):
    """The batched workload: cubic edges drawn uniformly from `edges` and
    temperatures uniform in [t_lo, t_hi), from one seeded generator."""
    rng = np.random.default_rng(seed)
    e = rng.choice(np.asarray(edges), size=count)
    t = rng.uniform(t_lo, t_hi, size=count)
    return [(int(a), float(b)) for a, b in zip(e, t)]


def batched_mt(jobs, precision=32, equil=1000, samples=4000, block=200, seed=4, J=1.0, Ku=0.01,
               tune=True, trial_sweeps=3, graph=0, timer=None, log=None, tail=0):
    """Independent m(T) runs, job i = (edge, T) on an edge^3 periodic lattice
    started along the easy axis (Philox key `seed`, instance i), advanced
    together in one batch.  equil + samples sweeps are timed (info run_s);
    `tail` more sampled sweeps then continue the same chains untimed, and the
    statistics cover all sampled blocks.  Returns per-job results and the
    batch timings."""
    import time
    import torch
    lats = [Lattice(e, e, e, precision=precision, J=J, Ku=Ku, eu=(0.0, 0.0, 1.0), seed=seed,
                    instance=i, init="aligned") for i, (e, _) in enumerate(jobs)]
    T = [t for _, t in jobs]
    B = Batch(lats)
    info = {"tune_s": 0.0}
    if tune:
        t0 = time.perf_counter()
        info["shapes"] = B.tune(T, trial_sweeps)
        info["tune_s"] = time.perf_counter() - t0
        info["chunk_bytes"] = B.chunk_bytes()
    if graph:
        B.set_graph(graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.sweep(T, equil)
    reads = [[] for _ in jobs]
    nblk = max(samples // block, 1)
    for _ in range(nblk):
        B.sweep(T, block, sample=True)
        for i, o in enumerate(B.observables()):
            reads[i].append(o)
    torch.cuda.synchronize()
    info["run_s"] = time.perf_counter() - t0
    for _ in range(tail // block):
        B.sweep(T, block, sample=True)
        for i, o in enumerate(B.observables()):
            reads[i].append(o)
    out = []
    for i, (e, t) in enumerate(jobs):
        r = block_stats_from_reads(reads[i], lats[i].n, t)
        r.update(edge=e, theta_deg=reads[i][-1]["theta_deg"], sweeps=reads[i][-1]["sweeps_done"])
        out.append(r)
    spins = sum(l.n for l in lats)
    info["updates"] = spins * (equil + nblk * block)
    info["spins"] = spins
    if log:
        log(f"batch of {len(jobs)} jobs, {spins} spins: {info['run_s']:.3f} s, "
            f"{info['updates'] / info['run_s'] / 1e9:.2f} G updates/s")
    B.close()
    for l in lats:
        l.close()
    return out, info


def compare_precisions(r32, r64):
    """Per job, FP32 against FP64 (runs with independent random keys, so the
    errors add in quadrature): |dm| of m(T) = <|m|> and its z-score (|dm| over
    the combined blocking error), the z-scores of <E>/N, of <m_z> and of the
    longitudinal susceptibility chi_l, and the gate of m(T) and E: both within
    3 standard errors, and |dm| <= 1e-3 wherever the resolution allows it
    (3 SE below 1e-3).  <m_z> and chi_l are reported, not gated: on small
    lattices at low T the direction of the whole moment relaxes over
    thousands of sweeps, which a window of a few ten thousand sweeps does
    not resolve (its blocking error is itself uncertain).  Also the runs'
    stationarity z-scores (first against second half of each window)."""
    def z(d, s):
        return d / s if s > 0 else (0.0 if d == 0 else math.inf)

    rows = []
    for a, b in zip(r32, r64):
        dm = abs(a["m"][0] - b["m"][0])
        se = math.hypot(a["se_m"][0], b["se_m"][0])
        zE = z(abs(a["E"] - b["E"]), math.hypot(a["se_E"], b["se_E"]))
        zz = z(abs(a["m"][3] - b["m"][3]), math.hypot(a["se_m"][3], b["se_m"][3]))
        zc = z(abs(a["chi"][0] - b["chi"][0]), math.hypot(a["se_chi"][0], b["se_chi"][0]))
        resolvable = 3.0 * se < 1e-3
        r = {"edge": a["edge"], "T": a["T"], "dm": dm, "se": se, "dm_over_se": z(dm, se),
             "dE_over_se": zE, "dmz_over_se": zz, "dchi_over_se": zc, "resolves_1e-3": resolvable}
        r["pass"] = r["dm_over_se"] <= 3.0 and zE <= 3.0 and (dm <= 1e-3 or not resolvable)
        if "stat_z_m" in a and "stat_z_m" in b:
            r["stat_z"] = max(abs(a["stat_z_m"]), abs(b["stat_z_m"]), abs(a["stat_z_E"]), abs(b["stat_z_E"]))
        rows.append(r)
    return rows


def ec_of(theta_deg, phi_deg):
    t, p = math.radians(theta_deg), math.radians(phi_deg)
    return (math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t))


def constrained_scan(thetas, phis, temps, size=128, precision=32, sweeps=3000, equil=1000,
                     seed=3, Kc=0.05, Ku=0.0, J=1.0, block=100, log=None):
    """Anisotropy energy and torque per spin with the moment held along
    e_C(theta, phi), each run started along e_C.  The sampled sweeps are read
    every `block` sweeps, so each run also carries the blocking standard
    error of its torque along e_phi (g_se) and of its anisotropy energy."""
    out = []
    run = 0
    for phi in phis:
        ephi = np.array([-math.sin(math.radians(phi)), math.cos(math.radians(phi)), 0.0])
        for T in temps:
            for th in thetas:
                ec = ec_of(th, phi)
                g = Lattice(size, size, size, precision=precision, J=J, Kc=Kc, Ku=Ku, seed=seed,
                            instance=run, init="aligned", init_dir=ec)
                g.constrained_sweep(T, ec, equil)
                gb, eb, prev = [], [], (0, np.zeros(3), 0.0)
                left = sweeps - equil
                while left > 0:
                    n = min(block, left)
                    g.constrained_sweep(T, ec, n, sample=True)
                    left -= n
                    o = g.observables()
                    ns = o["torque_samples"]
                    tsum = ns * np.asarray(o["mean_torque"])
                    esum = ns * o["mean_Eanis"]
                    gb.append(-float((tsum - prev[1]) @ ephi) / (ns - prev[0]))
                    eb.append((esum - prev[2]) / (ns - prev[0]))
                    prev = (ns, tsum, esum)
                g.close()
                r = {"theta": th, "phi": phi, "T": T, "E_anis": o["mean_Eanis"],
                     "E": o["mean_E"], "torque": o["mean_torque"], "m": o["mean_m"][0],
                     "g_se": float(blocking_se(np.array(gb)[:, None])[0]),
                     "E_anis_se": float(blocking_se(np.array(eb)[:, None])[0])}
                out.append(r)
                run += 1
                if log:
                    log(f"phi={phi} T={T} theta={th} E_anis={r['E_anis']:.6e} "
                        f"torque={np.round(r['torque'], 7).tolist()}")
    return out


def unconstrained_m(temps, size=128, precision=32, equil=2000, samples=4000, block=200, seed=3, Kc=0.05,
                    Ku=0.0, J=1.0):
    """<|m|> of independent unconstrained chains started along z (an easy
    axis of the cubic term), one per temperature, run as one batch."""
    lats = [Lattice(size, size, size, precision=precision, J=J, Kc=Kc, Ku=Ku, seed=seed, instance=1000 + i,
                    init="aligned") for i in range(len(temps))]
    B = Batch(lats)
    B.sweep(temps, equil)
    reads = [[] for _ in temps]
    for _ in range(max(samples // block, 1)):
        B.sweep(temps, block, sample=True)
        for i, o in enumerate(B.observables()):
            reads[i].append(o)
    out = {}
    for i, T in enumerate(temps):
        r = block_stats_from_reads(reads[i], lats[i].n, T)
        out[T] = (r["m"][0], r["se_m"][0])
    B.close()
    for l in lats:
        l.close()
    return out


def anisotropy_run(size=128, precision=32, thetas=tuple(range(0, 91, 10)), phis=(0.0, 45.0),
                   temps=(0.2, 0.4, 0.6, 0.8, 1.0, 1.2, 1.4), sweeps=3000, equil=1000, Kc=0.05, log=None):
    """The constrained scan, the unconstrained m(T) at the same temperatures,
    and K(T) with its Callen-Callen exponent (anisotropy.analyse)."""
    from . import anisotropy as A
    scan = constrained_scan(list(thetas), list(phis), list(temps), size=size, precision=precision,
                            sweeps=sweeps, equil=equil, Kc=Kc, log=log)
    m = unconstrained_m(list(temps), size=size, precision=precision, Kc=Kc)
    res = A.analyse(scan, {T: v[0] for T, v in m.items()}, Kc)
    res["m_se"] = {str(T): v[1] for T, v in m.items()}
    res["scan"] = scan
    if log:
        for r in res["rows"]:
            log(f"T={r['T']:.2f} m={r['m']:.5f} K_torque={r['K_torque']:.5e} K_energy={r['K_energy']:.5e}")
        log(f"n (torque) = {res.get('n_torque')}, n (energy) = {res.get('n_energy')}")
    return res


def eq4_run(temps, kind="cubic", K=0.05, size=128, precision=32, equil=1000, samples=2000, block=100,
            seed=3, J=1.0):
    """Eq. 4 route: standard sweeps of one lattice per temperature, started
    along z (the easy axis of both forms), run as one batch; k(T) from the
    mean anisotropy energy per spin (anisotropy.k_cubic / k_uniaxial), with
    its blocking standard error, and <|m|> from the same chains.  Returns
    rows {T, k, se_k, m, se_m, Eanis, se_Eanis} and the wall time."""
    import time
    import torch
    from . import anisotropy as A
    kw = dict(Kc=K, Ku=0.0) if kind == "cubic" else dict(Kc=0.0, Ku=K, eu=(0.0, 0.0, 1.0))
    t0 = time.perf_counter()
    lats = [Lattice(size, size, size, precision=precision, J=J, seed=seed, instance=2000 + i, init="aligned",
                    **kw) for i in range(len(temps))]
    B = Batch(lats)
    B.sweep(list(temps), equil)
    reads = [[] for _ in temps]
    for _ in range(max(samples // block, 1)):
        B.sweep(list(temps), block, sample=True)
        for i, o in enumerate(B.observables()):
            reads[i].append(o)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kfun, slope = (A.k_cubic, 5.0 / K) if kind == "cubic" else (A.k_uniaxial, 1.5 / K)
    rows = []
    for i, T in enumerate(temps):
        r = block_stats_from_reads(reads[i], lats[i].n, T)
        rows.append({"T": T, "k": float(kfun(r["Eanis"], K)), "se_k": slope * r["se_Eanis"],
                     "m": r["m"][0], "se_m": r["se_m"][0], "Eanis": r["Eanis"], "se_Eanis": r["se_Eanis"]})
    B.close()
    for l in lats:
        l.close()
    return rows, wall


def eq4_vs_constrained(temps=(0.2, 0.4, 0.6, 0.8, 1.0, 1.2, 1.4), size=128, precision=32, Kc=0.05,
                       thetas=tuple(range(0, 91, 10)), phis=(0.0, 45.0), sweeps=3000, equil=1000, log=None):
    """Cubic K(T)/K(0) two ways at the same temperatures: the torque route of
    constrained scans (Table A2) and Eq. 4 from standard sweeps along the easy
    axis, with their standard errors, the Callen-Callen exponents of both
    against m(T) of the standard runs, and the wall time of each route."""
    import time
    import torch
    from . import anisotropy as A
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scan = constrained_scan(list(thetas), list(phis), list(temps), size=size, precision=precision,
                            sweeps=sweeps, equil=equil, Kc=Kc, log=log)
    torch.cuda.synchronize()
    t_constrained = time.perf_counter() - t0
    e4, t_eq4 = eq4_run(list(temps), "cubic", Kc, size=size, precision=precision, equil=equil,
                        samples=sweeps - equil)
    rows = []
    for r in e4:
        T = r["T"]
        sel = [x for x in scan if x["T"] == T]
        Kt, se_Kt = A.fit_torque_amplitude_se(sel, A.cubic_df)
        kt, se_kt = Kt / Kc, se_Kt / Kc
        se = math.hypot(se_kt, r["se_k"])
        rows.append({"T": T, "m": r["m"], "k_torque": kt, "se_k_torque": se_kt, "k_eq4": r["k"],
                     "se_k_eq4": r["se_k"], "diff_over_se": (r["k"] - kt) / se if se > 0 else float("nan")})
        if log:
            log(f"T={T:.2f} m={r['m']:.5f} K/K0 torque {kt:.5f}+-{se_kt:.1e}  Eq.4 {r['k']:.5f}+-{r['se_k']:.1e}"
                f"  diff/se {rows[-1]['diff_over_se']:+.2f}")
    res = {"Kc": Kc, "size": size, "rows": rows, "t_constrained_s": t_constrained, "t_eq4_s": t_eq4,
           "constrained_runs": len(scan), "sweeps_per_run": sweeps}
    good = [x for x in rows if 0 < x["m"] < 1 and x["m"] > 0.6]
    if len(good) >= 2:
        ms = [x["m"] for x in good]
        res["n_torque_low"] = A.callen_callen_exponent([x["k_torque"] for x in good], 1.0, ms)
        res["n_eq4_low"] = A.callen_callen_exponent([x["k_eq4"] for x in good], 1.0, ms)
    return res


def eq4_convergence(Kcs=(0.05, 0.02, 0.01), temps=(0.4, 0.8), size=64, thetas=tuple(range(0, 91, 15)),
                    sweeps=3000, equil=1000, log=None):
    """Eq. 4 against the torque route as the anisotropy shrinks: for each Kc,
    k_eq4 - k_torque at each temperature with its combined error.  The two
    routes agree to first order in Kc/J (Callen-Callen theory), so the
    difference should shrink in proportion to Kc."""
    out = []
    for Kc in Kcs:
        r = eq4_vs_constrained(temps=temps, size=size, Kc=Kc, thetas=thetas, sweeps=sweeps, equil=equil)
        for row in r["rows"]:
            se = math.hypot(row["se_k_torque"], row["se_k_eq4"])
            out.append({"Kc": Kc, "T": row["T"], "m": row["m"], "k_torque": row["k_torque"],
                        "k_eq4": row["k_eq4"], "diff": row["k_eq4"] - row["k_torque"], "se_diff": se})
            if log:
                log(f"Kc={Kc} T={row['T']}: k_torque {row['k_torque']:.5f} k_eq4 {row['k_eq4']:.5f} "
                    f"diff {row['k_eq4'] - row['k_torque']:+.5f} +- {se:.5f}")
    return out


def uniaxial_K(temps, size=64, precision=32, thetas=(0, 15, 30, 45, 60, 75, 90), Ku=0.01, J=1.0, sweeps=3000,
               equil=1000, seed=8):
    """K(T) of a uniaxial term along z from constrained runs at a few angles
    (torque route, anisotropy.analyse with the sin^2 shape)."""
    from . import anisotropy as A
    scan = []
    run = 0
    for T in temps:
        for th in thetas:
            ec = ec_of(th, 0.0)
            g = Lattice(size, size, size, precision=precision, J=J, Ku=Ku, eu=(0.0, 0.0, 1.0), seed=seed,
                        instance=run, init="aligned", init_dir=ec)
            g.constrained_sweep(T, ec, equil)
            g.constrained_sweep(T, ec, sweeps - equil, sample=True)
            o = g.observables()
            g.close()
            scan.append({"theta": th, "phi": 0.0, "T": T, "E_anis": o["mean_Eanis"], "torque": o["mean_torque"]})
            run += 1
    res = A.analyse(scan, {}, Ku, kind="uniaxial")
    return {r["T"]: r["K_torque"] for r in res["rows"]}


def wall_run(temps, shape=(64, 64, 512), precision=32, J=1.0, Ku=0.01, equil=5000, samples=20000, every=250,
             seed=6, K_of_T=None, log=None):
    """Domain-wall width across temperatures (Sec. 3, Eq. 5): one lattice per
    temperature, anti-periodic along z and started from the T = 0 wall
    profile, all in one batch; the plane profile of m_z is fitted every
    `every` sampled sweeps and the widths averaged.  With K_of_T,
    A(T) = K Delta^2/pi^2."""
    from . import walls as Wm
    nx, ny, nz = shape
    lats = []
    for i, T in enumerate(temps):
        g = Lattice(nx, ny, nz, precision=precision, J=J, Ku=Ku, eu=(0.0, 0.0, 1.0), seed=seed, instance=i,
                    init="wall", init_width=Wm.zero_temperature_width(J, Ku), boundary_z="antiperiodic")
        lats.append(g)
    B = Batch(lats)
    B.sweep(list(temps), equil)
    fits = [[] for _ in temps]
    # also the plain average of the profiles (the wall is free to wander
    # along z, so this average is wider than the snapshots)
    psum = [np.zeros(nz) for _ in temps]
    nprof = 0
    for _ in range(max(samples // every, 1)):
        B.sweep(list(temps), every, sample=True)
        nprof += 1
        for i, g in enumerate(lats):
            prof = g.plane_means()[:, 2]
            psum[i] += prof
            try:
                fits[i].append(Wm.fit_wall(prof, delta_guess=Wm.zero_temperature_width(J, Ku)))
            except RuntimeError:
                pass
    obs = B.observables()
    out = []
    for i, T in enumerate(temps):
        f = np.array(fits[i]) if fits[i] else np.zeros((0, 3))
        r = {"T": T, "fits": len(f), "mean_E": obs[i]["mean_E"]}
        if len(f):
            r.update(m_wall=float(f[:, 0].mean()), delta=float(f[:, 2].mean()),
                     se_delta=float(f[:, 2].std(ddof=1) / math.sqrt(len(f))) if len(f) > 1 else float("nan"))
            try:
                r["delta_mean_profile"] = Wm.fit_wall(psum[i] / nprof,
                                                      delta_guess=Wm.zero_temperature_width(J, Ku))[2]
            except RuntimeError:
                pass
            if K_of_T is not None and T in K_of_T:
                r["K"] = K_of_T[T]
                r["A"] = Wm.exchange_stiffness(K_of_T[T], r["delta"])
                if "delta_mean_profile" in r:
                    r["A_mean_profile"] = Wm.exchange_stiffness(K_of_T[T], r["delta_mean_profile"])
        out.append(r)
        if log:
            log(f"T={T:.3f} wall fits {r['fits']}: Delta={r.get('delta', float('nan')):.3f} "
                f"m={r.get('m_wall', float('nan')):.4f} A={r.get('A', float('nan'))}")
    B.close()
    for g in lats:
        g.close()
    return out


def stiffness_run(temps=(0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 1.2), Ku=0.01, J=1.0,
                  shape=(64, 64, 512), log=None):
    """Exchange stiffness A(T) = K(T) Delta(T)^2 / pi^2 with K(T) from
    constrained runs and m(T) from unconstrained runs, and the exponent k of
    A(T)/A(0) = m^k (A(0) = J/2) over the low-temperature points (m > 0.6)."""
    from . import anisotropy as A
    K = uniaxial_K(list(temps), Ku=Ku, J=J)
    walls = wall_run(list(temps), shape=shape, Ku=Ku, J=J, K_of_T=K, log=log)
    m = unconstrained_m(list(temps), size=64, Kc=0.0, Ku=Ku, J=J)
    rows = []
    for w in walls:
        w["m"] = m[w["T"]][0]
        rows.append(w)
    low = [r for r in rows if "A" in r and r["m"] > 0.6 and r["A"] > 0]
    res = {"rows": rows, "A0": J / 2.0}
    if len(low) >= 2:
        res["k"] = A.callen_callen_exponent([r["A"] for r in low], J / 2.0, [r["m"] for r in low])
    lowp = [r for r in low if r.get("A_mean_profile", 0) > 0]
    if len(lowp) >= 2:
        # the same from the width of the time-averaged profile
        res["k_mean_profile"] = A.callen_callen_exponent([r["A_mean_profile"] for r in lowp], J / 2.0,
                                                         [r["m"] for r in lowp])
    if log:
        log(f"A(T) ~ m^k: k = {res.get('k')} (width of the time-averaged profile: {res.get('k_mean_profile')})")
    return res


def film_mt(temps, shape=(256, 256, 5), diameter=16.0, precision=32, J=1.0, Ku=0.01, equil=1000, samples=2000,
            block=200, seed=9, grains=True, n_terms=(1, 2, 4, 8, 12), log=None):
    """m(T) of a film with an open z boundary, granular (Voronoi grains of
    mean diameter `diameter`, no exchange between grains) or continuous,
    along ascending temperatures with the state carried over (the paper's
    increasing-temperature protocol), then the multi-Bloch fit of Eq. 8
    for each number of terms in n_terms."""
    from . import films as F
    nx, ny, nz = shape
    g = Lattice(nx, ny, nz, precision=precision, J=J, Ku=Ku, eu=(0.0, 0.0, 1.0), seed=seed, init="aligned",
                boundary_z="open", bond_masks=grains)
    info = {"shape": list(shape), "grains": 0}
    if grains:
        gm, ng = F.voronoi_grains(nx, ny, diameter, seed)
        g.set_bond_masks(F.grain_bond_masks(gm, nz))
        info.update(grains=int(len(np.unique(gm))), diameter=diameter)
    rows = []
    for T in temps:
        g.sweep(T, equil)
        blocks = []
        for _ in range(max(samples // block, 1)):
            g.reset_stats()
            g.sweep(T, block, sample=True)
            blocks.append(g.observables())
        r = _block_stats(blocks, g.n, T)
        rows.append(r)
        if log:
            log(f"film {shape} grains={info['grains']} T={T:.3f} m={r['m'][0]:.5f}+-{r['se_m'][0]:.1e}")
    g.close()
    T = np.array([r["T"] for r in rows])
    m = np.array([r["m"][0] for r in rows])
    fits = []
    for nb in n_terms:
        w, tc, b, mean_tc, rms = F.fit_multi_bloch(T, m, nb)
        fits.append({"terms": nb, "w": w.tolist(), "Tc": tc.tolist(), "beta": b.tolist(), "mean_Tc": mean_tc,
                     "rms": rms})
        if log:
            log(f"  multi-Bloch N_B={nb}: mean Tc = {mean_tc:.4f}, rms = {rms:.2e}")
    info.update(rows=rows, fits=fits)
    return info


def film_grid(n=1024, thicknesses=(5, 10, 15), diameters=(8.0, 16.0, 24.0), temps=None, equil=1000,
              samples=2000, block=200, n_terms=(1, 4, 8), log=None):
    """The granular-film workload: n x n films of each thickness (open z),
    Voronoi grains of each mean diameter and the continuous film, each swept
    along ascending temperatures (film_mt); returns per film the grain count,
    m(T) and the multi-Bloch fits of Eq. 8 with their mean T_C."""
    import time
    if temps is None:
        temps = np.round(np.arange(0.1, 1.61, 0.1), 3).tolist()
    out = []
    for nz in thicknesses:
        for d in list(diameters) + [None]:
            t0 = time.perf_counter()
            r = film_mt(list(temps), shape=(n, n, nz), diameter=d if d else 16.0, grains=d is not None,
                        equil=equil, samples=samples, block=block, n_terms=n_terms, log=log)
            r["wall_s"] = time.perf_counter() - t0
            r["nz"] = nz
            r["diameter"] = d
            out.append(r)
            if log:
                mt = {f["terms"]: round(f["mean_Tc"], 4) for f in r["fits"]}
                log(f"film {n}x{n}x{nz} d={d}: grains={r['grains']} mean Tc by N_B {mt} ({r['wall_s']:.1f} s)")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("mt", help="increasing-temperature m(T) protocol")
    a.add_argument("--size", type=int, default=256)
    a.add_argument("--precision", type=int, default=32)
    a.add_argument("--tmin", type=float, default=0.1)
    a.add_argument("--tmax", type=float, default=1.6)
    a.add_argument("--points", type=int, default=16)
    a.add_argument("--equil", type=int, default=2000)
    a.add_argument("--samples", type=int, default=4000)
    a.add_argument("--block", type=int, default=200)
    a.add_argument("--seed", type=int, default=7)
    a.add_argument("--init", default="random", choices=["random", "aligned"])
    a.add_argument("--Ku", type=float, default=0.005)
    b = sub.add_parser("batched", help="batched independent m(T) jobs, FP32 against FP64")
    b.add_argument("--count", type=int, default=64)
    b.add_argument("--equil", type=int, default=1000)
    b.add_argument("--samples", type=int, default=4000)
    b.add_argument("--block", type=int, default=200)
    an = sub.add_parser("anisotropy", help="constrained scan -> K(T) and its m^n scaling")
    an.add_argument("--size", type=int, default=128)
    an.add_argument("--sweeps", type=int, default=3000)
    an.add_argument("--equil", type=int, default=1000)
    an.add_argument("--Kc", type=float, default=0.05)
    w = sub.add_parser("stiffness", help="domain-wall widths -> exchange stiffness A(T)")
    w.add_argument("--nz", type=int, default=512)
    w.add_argument("--cross", type=int, default=64)
    w.add_argument("--Ku", type=float, default=0.01)
    f = sub.add_parser("film", help="granular film m(T) and the multi-Bloch fit")
    f.add_argument("--n", type=int, default=512)
    f.add_argument("--nz", type=int, default=5)
    f.add_argument("--diameter", type=float, default=16.0)
    f.add_argument("--continuous", action="store_true")
    e4 = sub.add_parser("eq4", help="K(T)/K(0) from Eq. 4 against the constrained torque route")
    e4.add_argument("--size", type=int, default=128)
    e4.add_argument("--sweeps", type=int, default=3000)
    e4.add_argument("--equil", type=int, default=1000)
    mg = sub.add_parser("mtgate", help="FP32 against FP64 along the increasing-temperature protocol")
    mg.add_argument("--size", type=int, default=256)
    mg.add_argument("--equil", type=int, default=2000)
    mg.add_argument("--samples", type=int, default=8000)
    mg.add_argument("--block", type=int, default=200)
    ec = sub.add_parser("eq4conv", help="Eq. 4 minus the torque route as Kc shrinks")
    ec.add_argument("--Kc", type=float, nargs="+", default=[0.05, 0.02, 0.01])
    ec.add_argument("--temps", type=float, nargs="+", default=[0.4, 0.8])
    ec.add_argument("--size", type=int, default=64)
    fg = sub.add_parser("films", help="granular films over thickness and grain size (mean Tc table)")
    fg.add_argument("--n", type=int, default=1024)
    fg.add_argument("--nz", type=int, nargs="+", default=[5, 10, 15])
    fg.add_argument("--diameters", type=float, nargs="+", default=[8.0, 16.0, 24.0])
    c = sub.add_parser("constrained", help="constrained-direction scan")
    c.add_argument("--size", type=int, default=128)
    c.add_argument("--precision", type=int, default=32)
    c.add_argument("--sweeps", type=int, default=3000)
    c.add_argument("--equil", type=int, default=1000)
    c.add_argument("--Kc", type=float, default=0.05)
    args = ap.parse_args(argv)

    def log(s):
        print(s, file=sys.stderr, flush=True)

    if args.cmd == "mt":
        temps = np.linspace(args.tmin, args.tmax, args.points).tolist()
        res = mt_sweep(temps, size=args.size, precision=args.precision, equil=args.equil,
                       samples=args.samples, block=args.block, seed=args.seed, init=args.init,
                       Ku=args.Ku, log=log)
    elif args.cmd == "film":
        temps = np.round(np.arange(0.1, 1.61, 0.1), 3).tolist()
        res = film_mt(temps, shape=(args.n, args.n, args.nz), diameter=args.diameter,
                      grains=not args.continuous, log=log)
    elif args.cmd == "stiffness":
        res = stiffness_run(shape=(args.cross, args.cross, args.nz), Ku=args.Ku, log=log)
    elif args.cmd == "films":
        res = film_grid(n=args.n, thicknesses=args.nz, diameters=args.diameters, log=log)
    elif args.cmd == "eq4":
        res = eq4_vs_constrained(size=args.size, sweeps=args.sweeps, equil=args.equil, log=log)
    elif args.cmd == "mtgate":
        temps = np.round(np.linspace(0.1, 1.6, 16), 3).tolist()
        res = mt_gate(temps, size=args.size, equil=args.equil, samples=args.samples, block=args.block, log=log)
    elif args.cmd == "eq4conv":
        res = eq4_convergence(Kcs=args.Kc, temps=args.temps, size=args.size, log=log)
    elif args.cmd == "anisotropy":
        res = anisotropy_run(size=args.size, sweeps=args.sweeps, equil=args.equil, Kc=args.Kc, log=log)
    elif args.cmd == "batched":
        jobs = c4_jobs(args.count)
        r32, i32 = batched_mt(jobs, 32, args.equil, args.samples, args.block, log=log)
        r64, i64 = batched_mt(jobs, 64, args.equil, args.samples, args.block, tune=False, seed=5, log=log)
        res = {"fp32": r32, "fp64": r64, "compare": compare_precisions(r32, r64),
               "info32": {k: v for k, v in i32.items() if k != "shapes"},
               "info64": {k: v for k, v in i64.items() if k != "shapes"}}
    else:
        res = constrained_scan(list(range(0, 91, 10)), [0, 45], [0.2 * k for k in range(1, 8)],
                               size=args.size, precision=args.precision, sweeps=args.sweeps,
                               equil=args.equil, Kc=args.Kc, log=log)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
