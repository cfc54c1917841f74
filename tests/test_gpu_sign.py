"""sign(A) b = (A^2)^{-1/2} (A b) on the HIP path (FAB_F_SIGN) against the
oracle ``krylov.sign_fAb`` (the same method on the exact FP64 A^2) and exact
values: a diagonal operator whose A^2 has 8 distinct eigenvalues (exact at
m = 8), and a shifted, indefinite 2D Laplacian stencil with a non-integer
centre, whose square is not representable in FP32 (the library applies A
twice per step in FP64).  Parity bars: 1e-10 (FP64 basis), 1e-6 (FP32 basis).
Blocking and served calls agree bit for bit; a CSR copy of the same operator
(A applied twice by the CSR product) agrees with the stencil result."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import krylov, operators, sketch as osk

pytestmark = pytest.mark.gpu

SIGN = W.FuncSpec("sign")


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2212_12758_amd import Context

    assert torch.cuda.is_available()
    c = Context(0, arena_bytes=4 << 30)
    yield c
    c.close()


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def test_sign_diagonal_exact(ctx):
    from paper_2212_12758_amd import make_params

    d = np.repeat([-3.0, -2.0, -1.5, -0.75, 0.5, 1.25, 2.5, 3.25], 100)
    M = sp.diags(d).tocsr()
    op = (M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float32))
    b = W.rhs(d.size, 4)
    A = ctx.matrix(op)
    print("case sign diagonal", flush=True)
    out, info = ctx.solve(A, _dev(b), SIGN, make_params(8, 2, 20, "sparse_sign", 8, 3, "fp64", "none"))
    assert krylov.relerr(out.cpu().numpy(), np.sign(d) * b) < 1e-12
    assert abs(info[0]["beta"] - np.linalg.norm(d * b)) < 1e-12 * np.linalg.norm(d * b)
    A.destroy()


def test_sign_shifted_laplacian_parity_and_serving(ctx):
    from paper_2212_12758_amd import make_params

    N, shift = 24, 1.3
    st = W.Stencil(2, N, N, 1, (4.0 - shift, -1.0, -1.0, -1.0, -1.0, 0.0, 0.0))
    Aor = operators.as_matrix(st)
    b = W.rhs(st.n, 4)
    m, k, s = 30, 2, 80
    sk = osk.Sketch("srht", st.n, s, 7, 8)
    ref = krylov.sign_fAb(Aor, b, m, k, sk, "sketch")
    A = ctx.matrix(st)
    print("case sign lap24 fp64", flush=True)
    p = make_params(m, k, s, "srht", 8, 7, "fp64", "sketch")
    out, info, dg = ctx.solve(A, _dev(b), SIGN, p, diag=True)
    out = out.cpu().numpy()
    H = ref["Hbar"]
    assert np.abs(dg["hbar"] - H[:, :m]).max() <= 1e-11 * np.abs(H).max()
    assert abs(info[0]["beta"] - np.linalg.norm(Aor @ b)) <= 1e-13 * np.linalg.norm(Aor @ b)
    assert krylov.relerr(out, ref["f"]) < 1e-10
    print("case sign lap24 fp32", flush=True)
    out32, _ = ctx.solve(A, _dev(b), SIGN, make_params(m, k, s, "srht", 8, 7, "fp32", "sketch"))
    assert krylov.relerr(out32.cpu().numpy(), ref["f"]) < 1e-6
    print("case sign lap24 csr fp64", flush=True)
    # the CSR copy holds FP32 values (the centre 2.7 is rounded), so its
    # reference is the oracle on that rounded matrix
    opc = (Aor.indptr.astype(np.int32), Aor.indices.astype(np.int32), Aor.data.astype(np.float32))
    refc = krylov.sign_fAb(operators.as_matrix(opc), b, m, k, sk, "sketch")
    Ac = ctx.matrix(opc)
    outc, _ = ctx.solve(Ac, _dev(b), SIGN, p)
    assert krylov.relerr(outc.cpu().numpy(), refc["f"]) < 1e-10
    Ac.destroy()
    print("case sign served", flush=True)
    o = _dev(np.zeros(st.n))
    ctx.submit(A, _dev(b), SIGN, p, o).wait()
    assert np.array_equal(o.cpu().numpy(), out)
    A.destroy()
