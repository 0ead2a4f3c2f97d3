"""Pins of the oracle's reaction-diffusion operator and implicit solve
(Eqs. oxygen / chemo discretised on the voxel lattice) against facts that do
not come from the oracle itself."""
import numpy as np
import pytest

from oracle import lattice


def dct_mode(shape, k):
    """Product of cos(pi k_d (i_d + 1/2) / n_d): an exact eigenvector of the
    zero-flux 7-point Laplacian with eigenvalue sum_d 4 sin^2(pi k_d/(2 n_d))."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    f = np.ones(shape)
    lam = 0.0
    for g, n, kk in zip(grids, shape, k):
        f = f * np.cos(np.pi * kk * (g + 0.5) / n)
        lam += 4.0 * np.sin(np.pi * kk / (2.0 * n)) ** 2
    return f, lam


@pytest.mark.parametrize("shape,k", [((5, 4, 6), (1, 2, 3)), ((3, 7, 2), (2, 0, 1)),
                                     ((1, 1, 9), (0, 0, 4)), ((4, 4, 4), (3, 3, 3))])
def test_laplacian_dct_eigenvectors(shape, k):
    f, lam = dct_mode(shape, k)
    np.testing.assert_allclose(-lattice.laplacian_apply(f), lam * f, atol=1e-13)


@pytest.mark.parametrize("method", ["lu", "cg"])
def test_implicit_solve_of_a_dct_mode(method):
    shape, k = (6, 5, 7), (1, 3, 2)
    f, lam = dct_mode(shape, k)
    a, c = 24.0, 0.0433
    u = lattice.solve(np.full(shape, c), a, f, method=method, rtol=1e-14)
    np.testing.assert_allclose(u, f / (c + a * lam), rtol=0, atol=1e-12 * np.abs(f / (c + a * lam)).max())


def test_1d_uniform_uptake_closed_form():
    """1-D lattice, uniform uptake c, unit source in the first voxel.  The
    discrete solution is A rho^i + B rho^-i with a (rho + 1/rho) = c + 2a in the
    interior; the two zero-flux end equations fix A and B."""
    n, a, c, s = 40, 262.5, 46.0, 1.0
    rho = ((c + 2 * a) - np.sqrt((c + 2 * a) ** 2 - 4 * a * a)) / (2 * a)
    i = np.arange(n)
    # end equations: (c+a) u0 - a u1 = s ;  (c+a) u_{n-1} - a u_{n-2} = 0
    M = np.array([[(c + a) - a * rho, (c + a) - a / rho],
                  [(c + a) * rho ** (n - 1) - a * rho ** (n - 2),
                   (c + a) * rho ** (-(n - 1)) - a * rho ** (-(n - 2))]])
    A, B = np.linalg.solve(M, [s, 0.0])
    exact = A * rho ** i + B * rho ** (-i.astype(float))
    b = np.zeros((1, 1, n))
    b[0, 0, 0] = s
    u = lattice.solve(np.full((1, 1, n), c), a, b, method="lu")
    np.testing.assert_allclose(u.ravel(), exact, rtol=1e-11)


def test_1d_continuum_limit_is_cosh_profile():
    """Refining h at fixed D, c, length: the discrete steady profile with a
    flux source at x=0 converges to cosh((L-x)/l)/cosh(L/l) at O(h^2)."""
    D, c, length = 1.0, 4.0, 2.0
    ell = np.sqrt(D / c)
    errs = []
    for n in (40, 80, 160):
        h = length / n
        a = D / h ** 2
        b = np.zeros((1, 1, n))
        b[0, 0, 0] = 1.0 / h     # unit boundary flux into the first cell
        u = lattice.solve(np.full((1, 1, n), c), a, b).ravel()
        x = (np.arange(n) + 0.5) * h
        ref = ell / D * np.cosh((length - x) / ell) / np.sinh(length / ell)
        errs.append(np.max(np.abs(u - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def test_uniform_uptake_and_source_gives_constant():
    shape = (4, 5, 6)
    u = lattice.solve(np.full(shape, 3.0), 262.5, np.full(shape, 12.0))
    np.testing.assert_allclose(u, 4.0, rtol=1e-13)


def test_conservation_with_pure_time_term():
    """c = 1/dt only: summing the equations, the zero-flux Laplacian drops out,
    so sum(u^{n+1}) = dt * sum(b) = sum(u^n) for b = u^n/dt."""
    rng = np.random.default_rng(3)
    shape = (5, 6, 7)
    un = rng.random(shape)
    dt = 30.0
    u = lattice.solve(np.full(shape, 1.0 / dt), 24.0, un / dt)
    assert abs(u.sum() - un.sum()) < 1e-11 * un.sum()


def test_operator_symmetric_and_positive():
    rng = np.random.default_rng(4)
    shape = (4, 6, 5)
    c = rng.random(shape) + 0.01
    u, v = rng.standard_normal(shape), rng.standard_normal(shape)
    Au = lattice.operator_apply(c, 262.5, u)
    Av = lattice.operator_apply(c, 262.5, v)
    assert abs((Au * v).sum() - (u * Av).sum()) < 1e-10 * np.abs(Au * v).sum()
    # M-matrix: nonnegative data gives a nonnegative solution
    b = rng.random(shape)
    b[b < 0.7] = 0.0
    x = lattice.solve(c, 262.5, b)
    assert x.min() >= 0.0


def test_shift_form_matches_kronecker_matrix():
    rng = np.random.default_rng(5)
    shape = (3, 4, 5)
    c = rng.random(shape)
    u = rng.standard_normal(shape)
    A = lattice.operator_matrix(c, 7.0)
    np.testing.assert_allclose(lattice.operator_apply(c, 7.0, u).ravel(), A @ u.ravel(),
                               rtol=1e-13, atol=1e-13)
