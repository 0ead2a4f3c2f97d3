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
"""
import math


def plasma(t, dose_times, dose_amts, k, G_ref):
    latest = None
    for tm, am in zip(dose_times, dose_amts):
        if tm <= t and (latest is None or tm >= latest[0]):
            latest = (tm, am)
    if latest is None:
        return 0.0
    tm, am = latest
    return am * G_ref * math.exp(-k * (t - tm))
