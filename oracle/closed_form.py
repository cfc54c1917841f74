"""Exact f(A)b by routes independent of Krylov methods (oracle pins only).

* Dirichlet Laplacian stencils are diagonalised by the orthonormal DST-I in
  every grid direction: A = S diag(lambda) S with
  lambda = sum_d (2 - 2 cos(pi j_d / (N_d + 1))), so f(A) b = S f(lambda) S b
  in O(n log n) (scipy's DST as a library step).  This is the converged
  reference f(A)b that Section 5 obtains with expm/sqrtm or many Arnoldi steps.
* Small dense matrices by eigendecomposition X f(Lambda) X^{-1} b.
* Diagonal matrices: f(A) b = f(diag) * b.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import matfun


def is_dirichlet_laplacian(st) -> bool:
    c, xm, xp, ym, yp, zm, zp = st.coeff
    if st.dim == 2:
        return (c, xm, xp, ym, yp) == (4.0, -1.0, -1.0, -1.0, -1.0) and st.nz == 1
    return (c, xm, xp, ym, yp, zm, zp) == (6.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0)


def laplacian_eigs(st) -> np.ndarray:
    dims = (st.nz, st.ny, st.nx) if st.dim == 3 else (st.ny, st.nx)
    lam = 0.0
    for ax, N in enumerate(dims):
        l1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, N + 1) / (N + 1))
        shape = [1] * len(dims)
        shape[ax] = N
        lam = lam + l1.reshape(shape)
    return lam


def laplacian_fAb(st, f, b: np.ndarray) -> np.ndarray:
    if not is_dirichlet_laplacian(st):
        raise ValueError("closed form needs the Dirichlet Laplacian stencil")
    dims = (st.nz, st.ny, st.nx) if st.dim == 3 else (st.ny, st.nx)
    B = np.asarray(b, dtype=np.float64).reshape(dims)
    C = sfft.dstn(B, type=1, norm="ortho")
    C *= matfun.fscalar(f, laplacian_eigs(st))
    return sfft.dstn(C, type=1, norm="ortho").ravel()


def dense_fAb(A: np.ndarray, f, b: np.ndarray, symmetric: bool = False) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    if symmetric:
        lam, X = np.linalg.eigh(A)
        return X @ (matfun.fscalar(f, lam) * (X.T @ b))
    lam, X = np.linalg.eig(A)
    z = np.linalg.solve(X, b.astype(complex))
    r = X @ (matfun.fscalar(f, lam.astype(complex)) * z)
    return r.real


def diagonal_fAb(d: np.ndarray, f, b: np.ndarray) -> np.ndarray:
    return matfun.fscalar(f, np.asarray(d, dtype=np.float64)) * b


def kronecker_exp_fAb(st, alpha: float, b: np.ndarray) -> np.ndarray:
    """exp(alpha A) b for any constant-coefficient 5/7-point stencil, at any size.

    Such an operator is a Kronecker sum: with the centre coefficient c split
    evenly over the d grid directions, A = T_z (+) T_y (+) T_x where T_x is the
    n_x x n_x tridiagonal matrix with c/d on the diagonal, the x-1 coefficient
    below it and the x+1 coefficient above it (Dirichlet: rows end at the
    boundary).  The summands commute, so exp(alpha A) = E_z (x) E_y (x) E_x
    with E_. = expm(alpha T_.), and the product with b (reshaped to the grid,
    x fastest) is one dense n_. x n_. product along each grid axis.  This is
    the converged f(A)b of Section 5 for the exponential of the 3D
    convection-diffusion operators, exact up to the rounding of three dense
    products (no Krylov method involved).  b is one vector (length n) or the
    (n, nrhs) array of several right-hand sides.
    """
    import scipy.linalg as sl

    c, xm, xp, ym, yp, zm, zp = (float(v) for v in st.coeff)
    d = 3 if st.dim == 3 else 2

    def factor(N, lo, hi):
        T = np.diag(np.full(N, c / d)) + np.diag(np.full(N - 1, lo), -1) + np.diag(np.full(N - 1, hi), 1)
        return sl.expm(alpha * T)

    Ex = factor(st.nx, xm, xp)
    Ey = factor(st.ny, ym, yp)
    Ez = factor(st.nz, zm, zp) if d == 3 else None
    B = np.asarray(b, dtype=np.float64)
    cols = B.reshape(st.n, -1)
    out = np.empty_like(cols)
    for q in range(cols.shape[1]):
        X = np.ascontiguousarray(cols[:, q]).reshape(st.nz, st.ny, st.nx)
        X = X @ Ex.T                      # x: the fastest index
        X = np.matmul(Ey, X)              # y: for every z plane
        if Ez is not None:
            X = (Ez @ X.reshape(st.nz, -1)).reshape(st.nz, st.ny, st.nx)
        out[:, q] = X.ravel()
    return out.reshape(B.shape)
