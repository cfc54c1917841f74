"""The CSR operator product and the sparse sign sketch at sizes where every
streaming block has four waves (n * nrhs >= 2^20), on a matrix whose degree
mix exercises the chunked product: rows of 1..23 nonzeros, empty rows, and
long rows that span several chunks of the workgroup and a block boundary.

Parity: Hbar of eq. (3), Theta V and the result against the oracle's
Algorithm 2 + sketch-and-solve (and Algorithm 1 for the sketched
Gram-Schmidt basis) in FP64; the same solve repeated gives the same bits
(fixed-order sums in the product and in the sketch accumulators).
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, operators, sketch as osk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2212_12758_amd import Context

    assert torch.cuda.is_available()
    c = Context(0, arena_bytes=8 << 30)
    yield c
    c.close()


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def ragged_csr(n: int, seed: int):
    """Random nonsymmetric CSR matrix (int32/FP32) with a ragged degree mix:
    1..23 nonzeros per row, every 1000th row empty, and rows of 9000 and 5000
    nonzeros (the latter in the last row block).  Diagonal shifted so that the
    spectrum sits in the left half plane."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(1, 24, n)
    deg[::1000] = 0
    deg[100] = 9000
    deg[n - 3] = 5000
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = rng.integers(0, n, nnz).astype(np.int32)
    val = (rng.standard_normal(nnz) / 8.0).astype(np.float32)
    # rows with entries get a diagonal entry of -4 in their first slot
    rows = np.repeat(np.arange(n), deg)
    first = rowptr[:-1][deg > 0]
    col[first] = np.arange(n)[deg > 0]
    val[first] = -4.0
    assert rows.size == nnz
    return rowptr.astype(np.int32), col, val


N_LARGE = (1 << 20) + 37


@pytest.fixture(scope="module")
def big():
    op = ragged_csr(N_LARGE, 11)
    return op, operators.as_matrix(op), W.rhs(N_LARGE, 12)


def test_csr_ragged_large_truncated_sparse_sign(ctx, big):
    from paper_2212_12758_amd import make_params

    op, Aor, b = big
    m, k, s = 8, 2, 40
    f = W.FuncSpec("exp", alpha=-0.05)
    sk = osk.Sketch("sparse_sign", N_LARGE, s, 5, 8)
    ref = krylov.nt(Aor, b, f, m, k, sk, "sketch")
    A = ctx.matrix(op)
    p = make_params(m, k, s, "sparse_sign", 8, 5, "fp64", "sketch")
    print("case csr ragged n=2^20+37 truncated fp64", flush=True)
    out, info, dg = ctx.solve(A, _dev(b), f, p, diag=True)
    out = out.cpu().numpy()
    H = ref["Hbar"]
    assert info[0]["m_used"] == m
    assert np.abs(dg["hbar"] - H).max() <= 1e-12 * np.abs(H).max()
    np.testing.assert_allclose(dg["sv"], ref["SV"], rtol=0, atol=1e-11)
    assert krylov.relerr(out, ref["f"]) < 1e-10
    for rep in range(2):
        o2, _, dg2 = ctx.solve(A, _dev(b), f, p, diag=True)
        assert np.array_equal(o2.cpu().numpy(), out), rep
        assert np.array_equal(dg2["sv"], dg["sv"]), rep
    print("case csr ragged n=2^20+37 truncated fp32", flush=True)
    o32, _ = ctx.solve(A, _dev(b), f, make_params(m, k, s, "sparse_sign", 8, 5, "fp32", "sketch"))
    assert krylov.relerr(o32.cpu().numpy(), ref["f"]) < 1e-6
    A.destroy()


def test_csr_ragged_large_sketched_gs(ctx, big):
    from paper_2212_12758_amd import make_params

    op, Aor, b = big
    # the sketched Gram-Schmidt recurrence amplifies rounding about tenfold per
    # step on this matrix (column j of Theta V agrees to ~10^(j-15)), so m = 6
    m, s = 6, 40
    f = W.FuncSpec("exp", alpha=-0.05)
    sk = osk.Sketch("sparse_sign", N_LARGE, s, 6, 8)
    ref = krylov.sgs(Aor, b, f, m, sk)
    A = ctx.matrix(op)
    p = make_params(m, 2, s, "sparse_sign", 8, 6, "fp64", "lsqr", 1e-11, basis="sketched_gs")
    print("case csr ragged n=2^20+37 sketched GS fp64", flush=True)
    out, info, dg = ctx.solve(A, _dev(b), f, p, diag=True)
    out = out.cpu().numpy()
    H = ref["Hbar"]
    assert info[0]["m_used"] == m
    assert np.abs(dg["hbar"] - H).max() <= 1e-10 * np.abs(H).max()
    assert np.abs(dg["sv"][:, : m + 1] - ref["S"]).max() < 1e-10
    assert krylov.relerr(out, ref["f"]) < 1e-10
    o2, _ = ctx.solve(A, _dev(b), f, p)
    assert np.array_equal(o2.cpu().numpy(), out)
    A.destroy()


def test_csr_multi_rhs_long_rows(ctx):
    """nrhs = 4 (product chunks of 1024 nonzeros x 4 right-hand sides) with a
    row longer than a chunk; every column against the oracle."""
    from paper_2212_12758_amd import make_params

    n, nr = 6000, 4
    op = ragged_csr(n, 21)
    Aor = operators.as_matrix(op)
    B = W.rhs(n, 22, nr)
    m, k, s = 10, 3, 40
    f = W.FuncSpec("exp", alpha=-0.05)
    A = ctx.matrix(op)
    print("case csr ragged n=6000 nrhs=4", flush=True)
    out, info = ctx.solve(A, _dev(B), f, make_params(m, k, s, "srht", 8, 7, "fp64", "sketch"))
    out = out.cpu().numpy()
    for q in range(nr):
        sk = osk.Sketch("srht", n, s, 7, 8)
        ref = krylov.nt(Aor, np.ascontiguousarray(B[:, q]), f, m, k, sk, "sketch")
        assert krylov.relerr(out[:, q], ref["f"]) < 1e-10, q
    A.destroy()
