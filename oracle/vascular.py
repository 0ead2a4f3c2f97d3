"""Vessel birth-death process of the vascular module, Eq. (vascular_module).

Test infrastructure only.  Arrays are (nz, ny, nx), flat index = gid.

Every dv_min (Table 1's vessel update interval, a whole number of coupled
steps) the vessel map changes voxel by voxel, from the extracellular VEGF V
just computed and the cell map after this step's cellular automaton:

* a vessel (w > 0) whose V lies outside the viability window
  [V_low, V_high] is removed (w := 0) with probability p_death;
* an empty voxel that is not a vessel, with V inside the window, becomes a
  vessel of perfusion weight w_new with probability proportional to V,
  birth_per_V * V (the paper's extension of its earlier model: birth
  probability proportional to the VEGF concentration).

Vessels and cells never share a voxel, so births need an empty voxel and a
removed vessel leaves one.  Each voxel draws one uniform: Philox4x64-10, key
(seed, 0), counter (gid, step + 1, STREAM_VESSEL, 0), u = (o_0 >> 11) 2^-53;
the event happens when u < probability.  The update runs at the end of the
step n -> n+1 exactly when (n + 1) is a multiple of dv_min / dt_min.
"""
import numpy as np

from . import philox
from .constants import EMPTY, STREAM_VESSEL


def is_update_step(n, p):
    """True when the step n -> n+1 ends on a vessel update time."""
    return (n + 1) % p.dv_steps == 0


def vessel_update(L, w, V, n, seed, p):
    """Returns (w_new, births, deaths) after the vessel update of the step
    n -> n+1 (w unchanged, 0, 0 when no update is due)."""
    w_new = w.copy()
    if not is_update_step(n, p):
        return w_new, 0, 0
    gids = np.arange(L.size, dtype=np.uint64)
    o0, _, _, _ = philox.block_vec(gids, n + 1, STREAM_VESSEL, 0, (seed, 0))
    u = philox.to_unit_vec(o0).reshape(L.shape)
    inside = (V >= p.V_low) & (V <= p.V_high)
    vessel = w > 0.0
    die = vessel & ~inside & (u < p.p_death)
    born = ~vessel & (L == EMPTY) & inside & (u < p.birth_per_V * V)
    w_new[die] = 0.0
    w_new[born] = p.w_new
    return w_new, int(np.count_nonzero(born)), int(np.count_nonzero(die))


def vessel_update_serial(L, w, V, n, seed, p):
    """The same rule written voxel by voxel on coordinates with the scalar
    Philox (a second transcription for the pins)."""
    w_new = w.copy()
    births = deaths = 0
    if (n + 1) % p.dv_steps != 0:
        return w_new, 0, 0
    nz, ny, nx = L.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                gid = x + nx * (y + ny * z)
                u = philox.to_unit(philox.block((gid, n + 1, STREAM_VESSEL, 0), (seed, 0))[0])
                v = V[z, y, x]
                ok = p.V_low <= v <= p.V_high
                if w[z, y, x] > 0.0:
                    if not ok and u < p.p_death:
                        w_new[z, y, x] = 0.0
                        deaths += 1
                elif L[z, y, x] == EMPTY and ok and u < p.birth_per_V * v:
                    w_new[z, y, x] = p.w_new
                    births += 1
    return w_new, births, deaths
