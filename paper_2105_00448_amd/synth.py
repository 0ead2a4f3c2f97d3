"""Seeded synthetic tissue generator.

Stands in for the patient MRI / histology maps the paper initialises from
(patient-specific initialisation subsection), which are not available: it
reproduces their qualitative structure, heterogeneous cell density and
perfusion, on a cubic voxel lattice.

* density rho(x) = clip(sum_g A_g exp(-|x - mu_g|^2 / (2 sigma_g^2)), 0, 1)
  with mu_g ~ U[0, n)^3, sigma_g ~ U[0.1, 0.3] n, A_g ~ U[0.3, 1.0];
* vessels: Bernoulli(vessel_frac) voxels with perfusion weight
  w ~ lognormal(0, 0.5); all other voxels have w = 0;
* cells on non-vessel voxels: Bernoulli(rho), cancer with probability
  ``cancer_frac`` else stroma.

This module holds no arithmetic of the model itself; both the HIP path and
the CPU oracle consume its arrays as inputs.  Arrays are (nz, ny, nx) C-order
so the flat index is gid = x + nx*(y + ny*z).
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Tissue:
    cell: np.ndarray      # uint8 (nz, ny, nx): 0 empty, 1 cancer, 2 stroma
    w: np.ndarray         # float64 (nz, ny, nx): perfusion weight, 0 = no vessel
    seed: int

    @property
    def shape(self):
        return self.cell.shape


def _rng(seed, salt):
    return np.random.Generator(np.random.Philox(key=[int(seed), int(salt)]))


def density(shape, n_gauss, rng):
    """Separable sum of Gaussians, evaluated as a rank-n_gauss tensor sum."""
    nz, ny, nx = shape
    n = max(shape)
    mu = rng.uniform(0.0, 1.0, size=(n_gauss, 3)) * np.array([nx, ny, nz])
    sig = rng.uniform(0.1, 0.3, size=n_gauss) * n
    amp = rng.uniform(0.3, 1.0, size=n_gauss)
    xs, ys, zs = np.arange(nx), np.arange(ny), np.arange(nz)
    ex = np.exp(-((xs[None, :] - mu[:, 0:1]) ** 2) / (2 * sig[:, None] ** 2))
    ey = np.exp(-((ys[None, :] - mu[:, 1:2]) ** 2) / (2 * sig[:, None] ** 2))
    ez = np.exp(-((zs[None, :] - mu[:, 2:3]) ** 2) / (2 * sig[:, None] ** 2)) * amp[:, None]
    rho = np.empty(shape)
    # rho[z, y, x] = sum_g ez[g, z] ey[g, y] ex[g, x], in y-chunks to bound memory
    ychunk = max(1, (1 << 22) // max(1, n_gauss * nx))
    for y0 in range(0, ny, ychunk):
        y1 = min(ny, y0 + ychunk)
        yx = (ey[:, y0:y1, None] * ex[:, None, :]).reshape(n_gauss, -1)
        rho[:, y0:y1, :] = (ez.T @ yx).reshape(nz, y1 - y0, nx)
    return np.clip(rho, 0.0, 1.0)


def make_tissue(shape, n_gauss, seed, vessel_frac=0.10, cancer_frac=0.8):
    if isinstance(shape, int):
        shape = (shape, shape, shape)
    rng = _rng(seed, 0)
    rho = density(shape, n_gauss, rng)
    u = rng.random(shape)
    vessel = u < vessel_frac
    w = np.zeros(shape)
    nv = int(vessel.sum())
    w[vessel] = rng.lognormal(0.0, 0.5, size=nv)
    occ = (~vessel) & (rng.random(shape) < rho)
    cancer = rng.random(shape) < cancer_frac
    cell = np.zeros(shape, dtype=np.uint8)
    cell[occ & cancer] = 1
    cell[occ & ~cancer] = 2
    return Tissue(cell=cell, w=w, seed=int(seed))


def uniform_tissue(shape, cell_density, vessel_density, seed, cancer_frac=0.8):
    """Cells and vessels scattered uniformly at the given voxel fractions (the
    paper's solver-performance setting: cell density 0.4, vascular density
    0.12): vessels Bernoulli(vessel_density) with w ~ lognormal(0, 0.5), cells
    on the other voxels with probability cell_density / (1 - vessel_density),
    cancer with probability ``cancer_frac`` else stroma."""
    rng = _rng(seed, 1)
    vessel = rng.random(shape) < vessel_density
    w = np.zeros(shape)
    w[vessel] = rng.lognormal(0.0, 0.5, size=int(vessel.sum()))
    occ = (~vessel) & (rng.random(shape) < cell_density / (1.0 - vessel_density))
    cancer = rng.random(shape) < cancer_frac
    cell = np.zeros(shape, dtype=np.uint8)
    cell[occ & cancer] = 1
    cell[occ & ~cancer] = 2
    return Tissue(cell=cell, w=w, seed=int(seed))


@dataclass
class DoseSchedule:
    """Bolus times (min) and amounts (multiples of the reference peak), per drug."""
    times: tuple
    amts: tuple


def bolus_schedule(steps, dt_min=30.0, amount=1.0):
    """Both drugs dosed at the listed step indices (time = step * dt)."""
    t = tuple(float(s) * dt_min for s in steps)
    a = tuple(float(amount) for _ in steps)
    return DoseSchedule(times=(t, t), amts=(a, a))


def ensemble(n_reps, seed0=1000, edge_lo=48, edge_hi=96, n_gauss=8, dt_min=30.0):
    """Replicates of uneven cubic edge n ~ U{edge_lo..edge_hi}, seeds seed0 + r,
    both drugs dosed once on day d ~ U{0, 1, 2} with amount ~ U[0.5, 1.5]."""
    rng = _rng(seed0, 7)
    reps = []
    for r in range(n_reps):
        n = int(rng.integers(edge_lo, edge_hi + 1))
        day = int(rng.integers(0, 3))
        amt = float(rng.uniform(0.5, 1.5))
        tis = make_tissue(n, n_gauss, seed0 + r)
        t = (day * 1440.0,)
        sched = DoseSchedule(times=(t, t), amts=((amt,), (amt,)))
        reps.append((tis, sched))
    return reps
