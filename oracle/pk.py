"""Plasma concentrations of the intravascular module.

Test infrastructure only.

Each drug's plasma concentration obeys a one-compartment linear elimination
dG/dt = -k G between doses (Eq. intrachemo3 for cyclophosphamide, k = cl_3/u;
the fluorouracil model of the same subsection in its linear regime
G << k_m, k = v_max/k_m) and is reset at each bolus to the dose's value
(the reset equations of that subsection).  The paper evaluates these ODEs in
closed form at the needed time points; so does this module.

A dose is (time in minutes, amount as a multiple of the reference peak
G_ref).  At time t the concentration is a_m G_ref exp(-k (t - t_m)) for the
latest dose t_m <= t, and 0 before the first dose.

``plasma_mm`` is fluorouracil's exact Michaelis-Menten elimination
dG/dt = -v_max G/(k_m + G) instead of its linear regime: separating variables,
k_m ln(G/G_m) + G - G_m = -v_max (t - t_m), i.e.
G = k_m W((G_m/k_m) exp((G_m - v_max (t - t_m))/k_m)) with W the principal
branch of the Lambert W function.

``plasma_epi`` is epirubicin's three-compartment model (the third drug): a
plasma compartment G0 exchanging with two peripheral compartments G1, G2,
all three expressed as amounts over the plasma volume w1 (so G0 is the
plasma concentration), with the rate constants of Table 1's volumes and
clearances, k10 = cl/w1, k12 = q2/w1, k21 = q2/w2, k13 = q3/w1, k31 = q3/w3:
    dG0/dt = -(k10 + k12 + k13) G0 + k21 G1 + k31 G2
    dG1/dt = k12 G0 - k21 G1
    dG2/dt = k13 G0 - k31 G2
(the printed plasma equation has G_{2,1}, G_{2,2} where its two outflow
terms need G_{2,0}; the peripheral equations are as printed).  A bolus resets
the plasma level to a_m G_ref, the peripheral compartments keep their
content.  Between doses the state follows exp(M dt), M the rate matrix above.
"""
import math

import numpy as np
from scipy.linalg import expm
from scipy.special import lambertw


def plasma(t, dose_times, dose_amts, k, G_ref):
    latest = None
    for tm, am in zip(dose_times, dose_amts):
        if tm <= t and (latest is None or tm >= latest[0]):
            latest = (tm, am)
    if latest is None:
        return 0.0
    tm, am = latest
    return am * G_ref * math.exp(-k * (t - tm))


def _latest(t, dose_times, dose_amts):
    latest = None
    for tm, am in zip(dose_times, dose_amts):
        if tm <= t and (latest is None or tm >= latest[0]):
            latest = (tm, am)
    return latest


def plasma_mm(t, dose_times, dose_amts, vmax, km, G_ref):
    latest = _latest(t, dose_times, dose_amts)
    if latest is None:
        return 0.0
    tm, am = latest
    g = am * G_ref
    if g == 0.0:
        return 0.0
    # W(x) at ln x = lx; beyond exp's range, the equation w + ln w = lx by Newton
    lx = math.log(g / km) + (g - vmax * (t - tm)) / km
    if lx < 700.0:
        return km * float(lambertw(math.exp(lx), 0).real)
    w = lx - math.log(lx)
    for _ in range(50):
        dw = (w + math.log(w) - lx) / (1.0 + 1.0 / w)
        w -= dw
        if abs(dw) <= 1e-16 * w:
            break
    return km * w


def epi_rate_matrix(p):
    """Rate matrix M of the three-compartment model (state G0, G1, G2)."""
    k10, k12, k13 = p.epi_cl / p.epi_w1, p.epi_q2 / p.epi_w1, p.epi_q3 / p.epi_w1
    k21, k31 = p.epi_q2 / p.epi_w2, p.epi_q3 / p.epi_w3
    return np.array([[-(k10 + k12 + k13), k21, k31],
                     [k12, -k21, 0.0],
                     [k13, 0.0, -k31]])


def plasma_epi(t, dose_times, dose_amts, p):
    """Epirubicin plasma level at t: doses in ascending time order, each
    resetting G0 to a_m G_ref3 after the state has followed exp(M dt) from the
    previous dose; 0 before the first dose."""
    M = epi_rate_matrix(p)
    x = np.zeros(3)
    tc = None
    for tm, am in zip(dose_times, dose_amts):
        if tm > t:
            break
        if tc is not None:
            x = expm(M * (tm - tc)) @ x
        x[0] = am * p.G_ref3
        tc = tm
    if tc is None:
        return 0.0
    return float((expm(M * (t - tc)) @ x)[0])
