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
"""
import math

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
