"""The synthetic operators A as explicit scipy sparse matrices (oracle side).

The paper accesses A only through matrix-vector products (Section 1; Table 1
"matrix access").  The oracle assembles A explicitly from its definition so
that its matvec is independent of the GPU stencil/CSR kernels:
a constant-coefficient stencil is a Kronecker sum of 1-D shift matrices,
row = x + nx*(y + ny*z) (x fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _shift_pair(N: int, lo: float, hi: float) -> sp.csr_matrix:
    """N x N matrix with `lo` on the sub-diagonal (neighbour -1) and `hi` on the super-diagonal."""
    return sp.diags([np.full(N - 1, lo), np.full(N - 1, hi)], [-1, 1], shape=(N, N), format="csr")


def stencil_matrix(st) -> sp.csr_matrix:
    c, xm, xp, ym, yp, zm, zp = (float(v) for v in st.coeff)
    Ix, Iy, Iz = (sp.identity(k, format="csr") for k in (st.nx, st.ny, st.nz))
    A = c * sp.identity(st.n, format="csr")
    if st.nx > 1:
        A = A + sp.kron(Iz, sp.kron(Iy, _shift_pair(st.nx, xm, xp)))
    if st.ny > 1:
        A = A + sp.kron(Iz, sp.kron(_shift_pair(st.ny, ym, yp), Ix))
    if st.nz > 1:
        A = A + sp.kron(_shift_pair(st.nz, zm, zp), sp.kron(Iy, Ix))
    return sp.csr_matrix(A)


def csr_matrix(rowptr, col, val) -> sp.csr_matrix:
    n = len(rowptr) - 1
    return sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(rowptr)), shape=(n, n))


def as_matrix(op) -> sp.csr_matrix:
    """A workload operator (Stencil or (rowptr, col, val)) as a float64 scipy CSR matrix."""
    if hasattr(op, "coeff"):
        return stencil_matrix(op)
    if sp.issparse(op):
        return sp.csr_matrix(op, dtype=np.float64)
    if isinstance(op, np.ndarray):
        return sp.csr_matrix(op)
    return csr_matrix(*op)
