"""Stochastic cellular automaton of the cellular module.

Test infrastructure only.  Arrays are (nz, ny, nx), flat index = gid.

Rules (section "Stochastic cellular automaton for the cellular module" and
the numerical treatment of the CA; conflict priority from Algorithm 2):

* A cancer cell is committed when its cycle phi >= 1 (after this step's ODE).
* A committed cell is killed by drug i (two drugs, three with the third-drug
  option) with probability
  I(G_i / G_ref_i; 1, b_i), the regularised incomplete beta function, which
  for a = 1 equals 1 - (1 - x)^b.  Each drug is an independent trial with its
  own uniform; the cell dies if any trial kills.  x is clipped to [0, 1] and
  the power is evaluated by repeated multiplication (integer b), so the
  decision is made with correctly rounded operations only.
* Otherwise the daughter goes to the Moore neighbour (26 in 3-D, 8 when
  nz = 1) that is empty, is not a vessel, and has the highest oxygen; the
  first strict maximum in ascending gid order wins ties.  With no such
  neighbour the cell's cycle is reset to 0 and no daughter is made.
* Updates are asynchronous: every decision reads the state before the CA
  update.  When several parents choose the same site, the parent with the
  higher phi wins (Algorithm 2); equal phi -> lower parent gid.  A losing
  parent is treated as having found no space.
* Successful division: parent and daughter get phi = P = V_c = 0 and the
  daughter's site becomes cancer.  Killed cell: site emptied, state zeroed.

Random numbers: Philox4x64-10, key (seed, 0), counter (gid, step + 1,
STREAM_KILL, 0), where ``step`` is the index n of the step n -> n+1;
u_{i-1} = (o_{i-1} >> 11) 2^-53 is drug i's uniform.

The implementation is the two-phase propose / resolve / finalize form.
"""
import numpy as np

from . import philox
from .constants import (CANCER, CODE_KILL, CODE_NONE, CODE_NOSPACE, EMPTY,
                        STREAM_KILL)


def moore_offsets():
    """(dz, dy, dx) of the 26 Moore neighbours in ascending-gid order, and
    their direction codes 0..25."""
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
            for dx in (-1, 0, 1) if (dz, dy, dx) != (0, 0, 0)]
    return offs


OFFSETS = moore_offsets()
OPPOSITE = [OFFSETS.index((-dz, -dy, -dx)) for (dz, dy, dx) in OFFSETS]


def _shifted(a, off, fill):
    """b[z,y,x] = a[z+dz, y+dy, x+dx], ``fill`` outside the lattice."""
    dz, dy, dx = off
    nz, ny, nx = a.shape
    b = np.full_like(a, fill)
    zs, zd = (slice(dz, nz), slice(0, nz - dz)) if dz >= 0 else (slice(0, nz + dz), slice(-dz, nz))
    ys, yd = (slice(dy, ny), slice(0, ny - dy)) if dy >= 0 else (slice(0, ny + dy), slice(-dy, ny))
    xs, xd = (slice(dx, nx), slice(0, nx - dx)) if dx >= 0 else (slice(0, nx + dx), slice(-dx, nx))
    b[zd, yd, xd] = a[zs, ys, xs]
    return b


def _inside(shape, off):
    return _shifted(np.ones(shape, dtype=bool), off, False)


def kill_probability(G, G_ref, b):
    x = np.minimum(np.maximum(G / G_ref, 0.0), 1.0)
    y = 1.0 - x
    pw = y.copy()
    for _ in range(b - 1):
        pw = pw * y
    return 1.0 - pw


def kill_uniforms(gids, step, seed):
    o0, o1, o2, _ = philox.block_vec(gids.astype(np.uint64), step + 1, STREAM_KILL, 0,
                                     (seed, 0))
    return philox.to_unit_vec(o0), philox.to_unit_vec(o1), philox.to_unit_vec(o2)


def propose(L, w, K, G1, G2, phi, step, seed, p, G3=None):
    """Proposal code per voxel: direction 0..25, NOSPACE, KILL or NONE."""
    shape = L.shape
    code = np.full(shape, CODE_NONE, dtype=np.uint8)
    committed = (L == CANCER) & (phi >= 1.0)
    gids = np.flatnonzero(committed)
    if gids.size == 0:
        return code
    u0, u1, u2 = kill_uniforms(gids, step, seed)
    p1 = kill_probability(G1.ravel()[gids], p.G_ref[0], p.b_int[0])
    p2 = kill_probability(G2.ravel()[gids], p.G_ref[1], p.b_int[1])
    killed = (u0 < p1) | (u1 < p2)
    if G3 is not None:   # third drug: its own trial with the third uniform
        killed = killed | (u2 < kill_probability(G3.ravel()[gids], p.G_ref3, p.b_int3))

    best_k = np.full(gids.size, -np.inf)
    best_d = np.full(gids.size, CODE_NOSPACE, dtype=np.uint8)
    for d, off in enumerate(OFFSETS):
        inside = _inside(shape, off).ravel()[gids]
        nL = _shifted(L, off, 255).ravel()[gids]
        nw = _shifted(w, off, 1.0).ravel()[gids]
        nK = _shifted(K, off, -np.inf).ravel()[gids]
        cand = inside & (nL == EMPTY) & (nw == 0.0)
        better = cand & (nK > best_k)
        best_k = np.where(better, nK, best_k)
        best_d = np.where(better, np.uint8(d), best_d)
    c = np.where(killed, np.uint8(CODE_KILL), best_d)
    code.ravel()[gids] = c
    return code


def resolve(L, w, phi, code):
    """Winner per empty non-vessel voxel: direction code (target -> parent)
    of the winning parent, or NONE."""
    shape = L.shape
    nvox = L.size
    gid = np.arange(nvox, dtype=np.int64).reshape(shape)
    target = (L == EMPTY) & (w == 0.0)
    win = np.full(shape, CODE_NONE, dtype=np.uint8)
    best_phi = np.full(shape, -np.inf)
    best_gid = np.full(shape, np.iinfo(np.int64).max, dtype=np.int64)
    for d, off in enumerate(OFFSETS):
        # parent s = t + off proposes t iff its code is the direction s -> t
        s_code = _shifted(code, off, CODE_NONE)
        s_phi = _shifted(phi, off, -np.inf)
        s_gid = _shifted(gid, off, -1)
        points = target & (s_code == OPPOSITE[d])
        better = points & ((s_phi > best_phi) | ((s_phi == best_phi) & (s_gid < best_gid)))
        best_phi = np.where(better, s_phi, best_phi)
        best_gid = np.where(better, s_gid, best_gid)
        win = np.where(better, np.uint8(d), win)
    return win


def finalize(L, phi, P, Vc, code, win):
    """Apply kills, divisions and resets.  Returns new (L, phi, P, Vc) and an
    event dict."""
    shape = L.shape
    Ln, phin, Pn, Vn = L.copy(), phi.copy(), P.copy(), Vc.copy()
    killed = code == CODE_KILL
    nospace = code == CODE_NOSPACE
    won = np.zeros(shape, dtype=bool)
    lost = np.zeros(shape, dtype=bool)
    for d, off in enumerate(OFFSETS):
        mine = code == d
        t_win = _shifted(win, off, CODE_NONE)     # win of my target
        ok = mine & (t_win == OPPOSITE[d])
        won |= ok
        lost |= mine & ~ok
    daughter = win != CODE_NONE

    Ln[killed] = EMPTY
    for arr in (phin, Pn, Vn):
        arr[killed] = 0.0
        arr[won] = 0.0
        arr[daughter] = 0.0
    phin[nospace | lost] = 0.0
    Ln[daughter] = CANCER
    ev = dict(committed=int(np.count_nonzero(code != CODE_NONE)),
              kills=int(np.count_nonzero(killed)),
              divisions=int(np.count_nonzero(won)),
              nospace=int(np.count_nonzero(nospace)),
              lost=int(np.count_nonzero(lost)))
    return Ln, phin, Pn, Vn, ev


def ca_update(L, w, K, G1, G2, phi, P, Vc, step, seed, p, G3=None):
    code = propose(L, w, K, G1, G2, phi, step, seed, p, G3)
    win = resolve(L, w, phi, code)
    return finalize(L, phi, P, Vc, code, win) + (code, win)
