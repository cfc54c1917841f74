"""MI355X (gfx950) sketched Krylov f(A)b: HIP kernels behind a C ABI (libfab.so).

The method is that of Cortinovis, Kressner & Nakatsukasa, "Speeding up Krylov
subspace methods for computing f(A)b via randomization": a k-truncated
Krylov basis (Algorithm 2), a subspace-embedding sketch of the basis
(Section 2.1.1), the compression recovered from a sketched least-squares
problem (eqs. (6)-(7), Remark 3) and the combination ||b|| V_m f(H_hat) e_1
(Algorithm 4).  This package is the thin Python binding; see include/fab.h.
"""
from .fab import (  # noqa: F401
    Context, FabError, Matrix, Request, load_library, make_params, LIB_PATH,
    OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EBUSY, ENOTFOUND,
)
