"""Temperature dependence of the cubic anisotropy from constrained runs
(Sec. 2 and Sec. 3 of the paper; Callen-Callen scaling).

With the magnetisation held along e_C(theta, phi), the anisotropy torque per
spin <tau> (tau = sum_i S_i x (-dE_anis/dS_i)) is the restoring torque of
the constrained free energy: turning e_C by d(theta) about
e_phi = (-sin phi, cos phi, 0) costs dF = -<tau> . e_phi d(theta).  So

    F(theta) - F(0) = -integral_0^theta <tau> . e_phi d(theta')

(at T -> 0 this is K_c f(e_C) with f = ex^2 ey^2 + ex^2 ez^2 + ey^2 ez^2,
which fixes the sign).  K(T) is the amplitude of the cubic angular
dependence of F, fitted over the scanned directions (directly on the torque,
-<tau>.e_phi = K dF/dtheta, which avoids the quadrature error of a coarse
angle grid; F itself is also integrated), and the exponent n of
K(T)/K(0) = m(T)^n compares with the l(l+1)/2 = 10 of Callen-Callen theory
for the fourth-order (l = 4) cubic term.  The internal-energy route fits the
same shape to <E_anis>(theta) instead.
"""
import math

import numpy as np


def e_c(theta_deg, phi_deg):
    t, p = math.radians(theta_deg), math.radians(phi_deg)
    return np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])


def e_phi(phi_deg):
    p = math.radians(phi_deg)
    return np.array([-math.sin(p), math.cos(p), 0.0])


def cubic_f(theta_deg, phi_deg):
    """f(e_C(theta, phi)) = sin^4 t cos^2 p sin^2 p + sin^2 t cos^2 t."""
    t, p = np.radians(theta_deg), math.radians(phi_deg)
    st, ct = np.sin(t), np.cos(t)
    return st ** 4 * math.cos(p) ** 2 * math.sin(p) ** 2 + st ** 2 * ct ** 2


def uniaxial_f(theta_deg, phi_deg):
    """Angular shape of a uniaxial term along z: 1 - cos^2 t = sin^2 t
    (E_anis = -Ku (S.z)^2 is Ku sin^2 t above its minimum)."""
    return np.sin(np.radians(theta_deg)) ** 2


def cubic_df(theta_deg, phi_deg):
    """d f(e_C(theta, phi)) / d theta of the cubic shape."""
    t, p = np.radians(theta_deg), math.radians(phi_deg)
    st, ct = np.sin(t), np.cos(t)
    return 4 * st ** 3 * ct * math.cos(p) ** 2 * math.sin(p) ** 2 + 2 * st * ct ** 3 - 2 * st ** 3 * ct


def uniaxial_df(theta_deg, phi_deg):
    """d sin^2(theta) / d theta."""
    return np.sin(2 * np.radians(theta_deg))


def cubic_torque(theta_deg, phi_deg, Kc):
    """Torque per spin at T = 0: e x (-Kc grad f(e)) with e = e_C."""
    e = e_c(theta_deg, phi_deg)
    g = 2.0 * Kc * np.array([e[0] * (e[1] ** 2 + e[2] ** 2), e[1] * (e[0] ** 2 + e[2] ** 2),
                             e[2] * (e[0] ** 2 + e[1] ** 2)])
    return np.cross(e, -g)


def free_energy_from_torque(thetas_deg, torques, phi_deg):
    """F(theta) - F(theta[0]) per spin: trapezoidal integral over theta (in
    radians) of -<tau> . e_phi."""
    th = np.radians(np.asarray(thetas_deg, dtype=float))
    g = -np.asarray(torques, dtype=float) @ e_phi(phi_deg)
    F = np.zeros_like(th)
    F[1:] = np.cumsum(0.5 * (g[1:] + g[:-1]) * np.diff(th))
    return F


def fit_cubic_amplitude(curves, shape=None):
    """Least-squares K with F(theta) - F(0) = K f(e_C) over all curves, each
    curve a tuple (thetas_deg, F, phi_deg) starting at theta = 0; f is the
    cubic shape unless another is given (uniaxial_f)."""
    shape = shape or cubic_f
    num = den = 0.0
    for th, F, phi in curves:
        f = shape(np.asarray(th, dtype=float), phi) - float(shape(0.0, phi))
        num += float(np.dot(f, F))
        den += float(np.dot(f, f))
    return num / den


def fit_torque_amplitude(rows, dshape):
    """Least-squares K with -<tau>.e_phi = K dshape/dtheta over the rows
    {theta, phi, torque}: the torque route without the quadrature error of
    integrating over a coarse angle grid."""
    num = den = 0.0
    for r in rows:
        g = -float(np.dot(np.asarray(r["torque"], dtype=float), e_phi(r["phi"])))
        d = float(dshape(float(r["theta"]), r["phi"]))
        num += g * d
        den += d * d
    return num / den


# ---------------------------------------------------------------------------
# Eq. 4: the reduced anisotropy from the easy-axis energy of standard
# (unconstrained) sweeps.  K_easy is the anisotropy energy per spin of the
# ensemble magnetised along an easy axis, measured from its T = 0 value (the
# easy direction), and K_0,hard the T = 0 energy of the hard direction on the
# same scale.  Uniaxial, E = -Ku (S.e)^2: K_easy = Ku (1 - <(S.e)^2>) =
# Ku + <E_uni>/N and K_0,hard = Ku (any direction perpendicular to e), so
# k_u = (3 <(S.e)^2> - 1)/2, the mean second Legendre polynomial.  Cubic,
# E = Kc f(S) (f = 0 along an axis, 1/3 along a body diagonal): K_easy =
# <E_cub>/N = Kc <f> and K_0,hard = Kc/3, so k_c = 1 - 5 <f>.  Both are 1 for
# spins frozen along the easy axis and 0 for isotropic spins (<(S.e)^2> = 1/3,
# <f> = 1/5).
# ---------------------------------------------------------------------------
def k_uniaxial(E_uni, Ku):
    """k_u = 1 - 3 K_easy / (2 K_0,hard) from the mean uniaxial energy per
    spin E_uni = -Ku <(S.e)^2> of a run along the easy axis."""
    K_easy = Ku + np.asarray(E_uni, dtype=float)
    return 1.0 - 3.0 * K_easy / (2.0 * Ku)


def k_cubic(E_cub, Kc):
    """k_c = 1 - 5 K_easy / (3 K_0,hard) from the mean cubic energy per spin
    E_cub = Kc <f> of a run along an easy axis (Kc > 0)."""
    K_easy = np.asarray(E_cub, dtype=float)
    return 1.0 - 5.0 * K_easy / (3.0 * (Kc / 3.0))


def fit_torque_amplitude_se(rows, dshape):
    """fit_torque_amplitude and its standard error from each row's error
    g_se of -<tau>.e_phi (independent runs): K = sum g d / sum d^2, so
    se(K) = sqrt(sum (d g_se)^2) / sum d^2."""
    num = den = var = 0.0
    for r in rows:
        g = -float(np.dot(np.asarray(r["torque"], dtype=float), e_phi(r["phi"])))
        d = float(dshape(float(r["theta"]), r["phi"]))
        num += g * d
        den += d * d
        var += (d * float(r.get("g_se", 0.0))) ** 2
    return num / den, math.sqrt(var) / den


def callen_callen_exponent(K, K0, m):
    """n of K/K0 = m^n by least squares on the logarithms, through the origin."""
    x = np.log(np.asarray(m, dtype=float))
    y = np.log(np.asarray(K, dtype=float) / K0)
    return float(np.dot(x, y) / np.dot(x, x))


def analyse(scan, m_of_T, Kc, kind="cubic"):
    """K(T) from the torque and from <E_anis>, and the exponents n.

    scan: rows {theta, phi, T, E_anis, torque} of a constrained scan;
    m_of_T: {T: <|m|>} from unconstrained runs at the same temperatures;
    kind: "cubic" (Kc f) or "uniaxial" (Ku sin^2 theta about z), Kc being
    the T = 0 constant of that term."""
    shape = cubic_f if kind == "cubic" else uniaxial_f
    dshape = cubic_df if kind == "cubic" else uniaxial_df
    temps = sorted({r["T"] for r in scan})
    phis = sorted({r["phi"] for r in scan})
    out = []
    for T in temps:
        curves_tau, curves_e = [], []
        for phi in phis:
            rows = sorted((r for r in scan if r["T"] == T and r["phi"] == phi), key=lambda r: r["theta"])
            th = [r["theta"] for r in rows]
            if not rows or th[0] != 0:
                continue
            F = free_energy_from_torque(th, [r["torque"] for r in rows], phi)
            E = np.array([r["E_anis"] for r in rows])
            curves_tau.append((th, F, phi))
            curves_e.append((th, E - E[0], phi))
        out.append({"T": T, "K_torque": fit_torque_amplitude([r for r in scan if r["T"] == T], dshape),
                    "K_torque_integrated": fit_cubic_amplitude(curves_tau, shape),
                    "K_energy": fit_cubic_amplitude(curves_e, shape), "m": m_of_T.get(T),
                    "F": {str(c[2]): [float(v) for v in c[1]] for c in curves_tau}})
    res = {"Kc": Kc, "rows": out}
    # over every point with 0 < m < 1, and over the low-temperature range
    # m > 0.6 where the Callen-Callen law is expected to hold
    for tag, m_lo in (("", 0.0), ("_low", 0.6)):
        have_m = [r for r in out if r["m"] is not None and r["K_torque"] > 0 and m_lo < r["m"] < 1]
        if len(have_m) >= 2:
            res["n_torque" + tag] = callen_callen_exponent([r["K_torque"] for r in have_m], Kc,
                                                           [r["m"] for r in have_m])
            good_e = [r for r in have_m if r["K_energy"] > 0]
            if len(good_e) >= 2:
                res["n_energy" + tag] = callen_callen_exponent([r["K_energy"] for r in good_e], Kc,
                                                               [r["m"] for r in good_e])
    return res
