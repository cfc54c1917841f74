"""f(K) e_1 for a small dense matrix K (oracle side, test infrastructure).

Section 5 evaluates f on the compressed matrices with MATLAB's expm and sqrtm;
the oracle uses scipy's counterparts (scaling-and-squaring Pade for exp, the
Schur method for the square root) as library steps.

Supported f (the function classes of the workloads):
  exp   f(z) = exp(alpha z)
  pow   f(z) = (z + sigma)^p, p in {+1/2, -1/2}  (principal branch)
  poly  f(z) = sum_j coef[j] z^j
  sign  f(z) = sign(Re z)  (scalars only: the closed forms of sign(A) b)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl


def _real(M: np.ndarray) -> np.ndarray:
    M = np.asarray(M)
    if np.iscomplexobj(M):
        scale = max(1.0, float(np.abs(M).max()))
        if float(np.abs(M.imag).max()) > 1e-8 * scale:
            raise ArithmeticError("matrix function of a real matrix came out complex")
        M = M.real
    return np.asarray(M, dtype=np.float64)


def fmat(f, K: np.ndarray) -> np.ndarray:
    """The full matrix f(K)."""
    K = np.asarray(K, dtype=np.float64)
    m = K.shape[0]
    if f.kind == "exp":
        return sl.expm(f.alpha * K)
    if f.kind == "pow":
        R = _real(sl.sqrtm(K + f.sigma * np.eye(m)))
        if f.p == 0.5:
            return R
        if f.p == -0.5:
            return sl.solve(R, np.eye(m))
        raise ValueError("p must be +-1/2")
    if f.kind == "poly":
        F = np.zeros((m, m))
        P = np.eye(m)
        for c in f.coef:
            F += c * P
            P = P @ K
        return F
    raise ValueError(f.kind)


def fmat_e1(f, K: np.ndarray) -> np.ndarray:
    """f(K) e_1."""
    K = np.asarray(K, dtype=np.float64)
    m = K.shape[0]
    e1 = np.zeros(m)
    e1[0] = 1.0
    if f.kind == "pow" and f.p == -0.5:
        R = _real(sl.sqrtm(K + f.sigma * np.eye(m)))
        return sl.solve(R, e1)
    if f.kind == "poly":
        y = np.zeros(m)
        for c in reversed(f.coef):       # Horner on the vector
            y = K @ y + c * e1
        return y
    return fmat(f, K)[:, 0]


def fscalar(f, z: np.ndarray) -> np.ndarray:
    """f applied to scalars (eigenvalues); used by the closed forms."""
    z = np.asarray(z)
    if f.kind == "exp":
        return np.exp(f.alpha * z)
    if f.kind == "pow":
        return (z + f.sigma) ** f.p
    if f.kind == "poly":
        y = np.zeros_like(z, dtype=np.result_type(z, float))
        for c in reversed(f.coef):
            y = y * z + c
        return y
    if f.kind == "sign":
        # the matrix sign function maps each eigenvalue to the sign of its
        # real part (Section 5.1.3; undefined on the imaginary axis)
        return np.sign(np.real(z))
    raise ValueError(f.kind)
