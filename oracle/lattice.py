"""Reaction-diffusion systems of the extravascular module on the voxel lattice.

Test infrastructure only.

Arrays are shaped (nz, ny, nx) in C order, so the flat index of voxel
(x, y, z) is the global id gid = x + nx*(y + ny*z).

The Laplacian is the voxel-centred 7-point difference with zero-flux faces:
(Lap u)_i = sum over existing face neighbours j of (u_j - u_i).  A missing
neighbour (outside the lattice) contributes nothing, which is the natural
(homogeneous Neumann) boundary of the paper's weak form of Eqs. (oxygen) and
(chemo) when no boundary data are given.

Every implicit-Euler update of those equations is a linear system

    c_i u_i - a (Lap u)_i = b_i,      a = D / h^2,

with c > 0, i.e. a symmetric M-matrix.  Its exact solution is the oracle's
result; ``solve`` computes it by sparse LU (``method="lu"``) or, for timing
large lattices, by SciPy's CG to a tight tolerance (``method="cg"``).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian_apply(u):
    """(Lap u) for an (nz, ny, nx) array, zero-flux faces."""
    out = np.zeros_like(u)
    for axis in range(3):
        n = u.shape[axis]
        if n < 2:
            continue
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        diff = u[tuple(hi)] - u[tuple(lo)]   # u_{i+1} - u_i across each face
        out[tuple(lo)] += diff
        out[tuple(hi)] -= diff
    return out


def operator_apply(c, a, u):
    """A u = c*u - a*Lap(u)."""
    return c * u - a * laplacian_apply(u)


def _lap1d(n):
    if n == 1:
        return sp.csr_matrix((1, 1))
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    off = -np.ones(n - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr")


def laplacian_matrix(shape):
    """Sparse matrix of -Lap (positive semidefinite graph Laplacian)."""
    nz, ny, nx = shape
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(sp.kron(Iz, Iy), _lap1d(nx))
            + sp.kron(sp.kron(Iz, _lap1d(ny)), Ix)
            + sp.kron(sp.kron(_lap1d(nz), Iy), Ix)).tocsr()


def operator_matrix(c, a):
    """Sparse matrix of A = diag(c) - a*Lap."""
    return (sp.diags(c.ravel()) + a * laplacian_matrix(c.shape)).tocsc()


def solve(c, a, b, x0=None, method="cg", rtol=1e-15):
    """Solution of (diag(c) - a Lap) u = b.

    ``method="lu"``: sparse direct solve (SuperLU, minimum-degree ordering of
    A + A^T), the plain definition; its fill grows fast in 3-D, so it serves
    the small pin cases.
    ``method="cg"`` (default): SciPy's conjugate gradient with diagonal
    scaling from ``x0`` to relative residual ``rtol`` = 1e-15, i.e. the exact
    solution up to cond(A) * 1e-15.  Checked against the LU solution in the
    oracle's tests.
    """
    A = operator_matrix(c, a)
    if method == "lu":
        u = spla.splu(A, permc_spec="MMD_AT_PLUS_A",
                      options=dict(SymmetricMode=True)).solve(b.ravel())
    elif method == "cg":
        d = A.diagonal()
        M = sp.diags(1.0 / d)
        if not np.any(b):
            return np.zeros(c.shape)
        u, info = spla.cg(A.tocsr(), b.ravel(), M=M,
                          x0=None if x0 is None else x0.ravel(),
                          rtol=rtol, atol=0.0, maxiter=100000)
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge (info={info})")
    else:
        raise ValueError(method)
    return u.reshape(c.shape)
