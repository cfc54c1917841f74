"""Served single-rhs requests merged into block solves (continuous batching:
requests queued together on one resident matrix with the same function and
parameters run as the columns of one nrhs > 1 solve, the operator applied to
the whole block in each step -- Algorithm 2 on a block of vectors).

Each merged request's result equals its result alone (a blocking solve) and
the oracle's f_m within the stated tolerance: 1e-6 with the FP32 basis, 1e-10
with the FP64 basis (the block groups the reductions differently, so the bits
differ).  fab_hold makes the grouping deterministic: a burst submitted while
admission is held is merged by the queue order when it is released.
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
    c = Context(0, arena_bytes=4 << 30)
    yield c
    c.close()


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _burst(ctx, jobs):
    """Submit (A, b, f, params) jobs while admission is held; returns (out, info) per job."""
    import torch

    ctx.hold(True)
    try:
        subs = []
        for A, b, f, p in jobs:
            bd = _dev(b)
            o = torch.empty_like(bd)
            subs.append((o, ctx.submit(A, bd, f, p, o), bd))
    finally:
        ctx.hold(False)
    res = []
    for o, r, _ in subs:
        info = r.wait()
        res.append((o.cpu().numpy(), info[0]))
    return res


@pytest.mark.parametrize("prec,tol,nreq,sketch,s", [("fp32", 1e-6, 16, "srht", 120), ("fp64", 1e-10, 8, "srht", 120),
                                                   ("fp32", 1e-6, 8, "sparse_sign", 80)])
def test_merged_requests_equal_alone_and_oracle(ctx, prec, tol, nreq, sketch, s):
    from paper_2212_12758_amd import make_params

    st = W.convdiff3d(24, 50.0)
    f = W.FuncSpec("exp", alpha=-1e-3)
    m, k = 30, 4
    p = make_params(m, k, s, sketch, 8, 7, prec, "sketch", tol)
    A = ctx.matrix(st)
    Aor = operators.as_matrix(st)
    bs = [W.rhs(st.n, 100 + q) for q in range(nreq)]
    print(f"case merged {prec} {sketch} x{nreq}", flush=True)
    res = _burst(ctx, [(A, b, f, p) for b in bs])
    for q, (got, info) in enumerate(res):
        assert info["block_rhs"] == nreq, q
        alone, _ = ctx.solve(A, _dev(bs[q]), f, p)
        assert krylov.relerr(got, alone.cpu().numpy()) < tol, q
        assert krylov.relerr(got, krylov.fm(Aor, bs[q], f, m)) < tol, q
    A.destroy()


def test_grouping_by_parameters_power_of_two_and_limit(ctx):
    from paper_2212_12758_amd import make_params

    st = W.laplacian2d(48)
    A = ctx.matrix(st)
    f1, f2 = W.FuncSpec("exp", alpha=-0.5), W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    p = make_params(25, 2, 60, "srht", 8, 3, "fp64", "sketch", 1e-10)
    bs = [W.rhs(st.n, 200 + q) for q in range(13)]
    # 7 requests of f1 interleaved with 6 of f2: blocks are formed from the
    # queue head, the largest power of two of the compatible queued requests:
    # f1 4 + 2 + 1 (the last on its own), f2 4 + 2
    jobs = [(A, bs[q], f1 if q % 2 == 0 else f2, p) for q in range(13)]
    kinds = [j[2] for j in jobs]
    print("case grouping", flush=True)
    res = _burst(ctx, jobs)
    n1 = kinds.count(f1)
    sizes1 = sorted(info["block_rhs"] for (_, info), kd in zip(res, kinds) if kd is f1)
    sizes2 = sorted(info["block_rhs"] for (_, info), kd in zip(res, kinds) if kd is f2)
    def expect(n):
        out, left = [], n
        while left:
            g = 1
            while 2 * g <= left and 2 * g <= 32:
                g *= 2
            out += [g] * g
            left -= g
        return sorted(out)
    assert sizes1 == expect(n1) and sizes2 == expect(len(kinds) - n1)
    # sketch-and-solve (Remark 3) is not converged to f_m at m = 25 here: the
    # oracle is the same method, Algorithm 4 with the same sketch, in FP64
    Aor = operators.as_matrix(st)
    sk = osk.Sketch("srht", st.n, 60, 3, 8)
    for (got, info), (_, b, fk, _) in zip(res, jobs):
        assert krylov.relerr(got, krylov.nt(Aor, b, fk, 25, 2, sk, "sketch")["f"]) < 1e-10
    # merging off: every request alone, bit for bit the blocking result
    ctx.set_block_limit(1)
    try:
        res = _burst(ctx, [(A, b, f1, p) for b in bs[:4]])
    finally:
        ctx.set_block_limit(32)
    for (got, info), b in zip(res, bs[:4]):
        assert info["block_rhs"] == 1
        alone, _ = ctx.solve(A, _dev(b), f1, p)
        assert np.array_equal(got, alone.cpu().numpy())
    A.destroy()
