"""The cheap approximations as served modes: Algorithm 5 (y = 0, eq. (8);
FAB_LS_NONE) and sketch-and-solve (Remark 3; FAB_LS_SKETCH), which equals
sFOM (eq. (9)).  Blocking and served (fab_submit) calls against the oracle's
Algorithms 4/5 and sFOM on a nonsymmetric operator, where the truncated
basis is not orthonormal and the three results differ; served results must
equal blocking ones bit for bit, also when the two modes run concurrently."""
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


def test_served_algorithm5_and_sfom(ctx):
    from paper_2212_12758_amd import make_params

    st = W.convdiff3d(20, 50.0)
    b = W.rhs(st.n, 61)
    f = W.FuncSpec("exp", alpha=-3e-2)   # ||alpha A|| = 30: not converged at m = 20
    m, k, s = 20, 2, 80
    Aor = operators.as_matrix(st)
    sk = osk.Sketch("srht", st.n, s, 6, 8)
    ref_none = krylov.nt(Aor, b, f, m, k, sk, "none")["f"]
    ref_sk = krylov.nt(Aor, b, f, m, k, sk, "sketch")["f"]
    ref_sfom = krylov.sfom(Aor, b, f, m, k, sk)
    assert krylov.relerr(ref_sk, ref_sfom) < 1e-10          # Remark 3
    assert krylov.relerr(ref_none, ref_sk) > 1e-4            # the modes differ here (1.4e-3)
    A = ctx.matrix(st)
    outs = {}
    for ls, ref in (("none", ref_none), ("sketch", ref_sk)):
        print(f"case served mode {ls}", flush=True)
        p = make_params(m, k, s, "srht", 8, 6, "fp64", ls)
        out, info = ctx.solve(A, _dev(b), f, p)
        out = out.cpu().numpy()
        assert krylov.relerr(out, ref) < 1e-10, ls
        outs[ls] = out
    # served, both modes in flight at once (merging off: two requests of one
    # mode would otherwise run as one block solve)
    ctx.set_block_limit(1)
    reqs = []
    for ls in ("none", "sketch", "none", "sketch"):
        o = _dev(np.zeros(st.n))
        reqs.append((ls, o, ctx.submit(A, _dev(b), f, make_params(m, k, s, "srht", 8, 6, "fp64", ls), o)))
    for ls, o, r in reqs:
        r.wait()
        assert np.array_equal(o.cpu().numpy(), outs[ls]), ls
    ctx.set_block_limit(32)
    A.destroy()


def test_wait_while_another_thread_submits(ctx):
    """fab_wait blocks with the context lock released while another thread
    keeps submitting (the request table grows and rehashes meanwhile): every
    request completes with the blocking call's result, bit for bit when it ran
    on its own, within the FP32-basis tolerance when the scheduler merged it
    with other queued copies into a block solve."""
    import queue
    import threading

    import torch

    from paper_2212_12758_amd import make_params

    st = W.laplacian2d(32)
    A = ctx.matrix(st)
    f = W.FuncSpec("exp", alpha=-0.5)
    p = make_params(20, 2, 50, "srht", 8, 3, "fp32", "sketch")
    b = _dev(W.rhs(st.n, 9))
    ref, _ = ctx.solve(A, b, f, p)
    ref = ref.cpu().numpy()
    print("case wait while submitting", flush=True)
    q, outs, errs = queue.Queue(), [], []

    def submitter():
        try:
            for _ in range(200):
                o = torch.empty_like(b)
                r = ctx.submit(A, b, f, p, o)
                outs.append((o, r))
                q.put(r)
        except Exception as e:   # reported by the main thread
            errs.append(e)
        q.put(None)

    t = threading.Thread(target=submitter)
    t.start()
    done = 0
    while True:
        r = q.get()
        if r is None:
            break
        r.wait()
        done += 1
    t.join()
    assert not errs and done == 200
    for o, r in outs:
        got = o.cpu().numpy()
        if r.info[0]["block_rhs"] == 1:
            assert np.array_equal(got, ref)
        else:
            assert krylov.relerr(got, ref) < 1e-6
    A.destroy()


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_served_auto_policies_match_blocking(ctx, tol):
    """FAB_PREC_AUTO with FAB_LS_AUTO on an unconverged inverse square root
    (the least-squares gate fails, so the refinement runs): the served call
    takes the same decisions as the blocking one (the precision is judged on
    the solve's own result, before the refinement) and returns the same
    result bit for bit.  At tol = 1e-8 the FP32 rounding estimate fails, so
    both calls recompute with an FP64 basis and then refine: that rerun must
    refine too (it once came back unrefined, 2.5e-2 off f_m), and the result
    meets tol against f_m."""
    from paper_2212_12758_amd import make_params

    st = W.laplacian2d(128)
    b = W.rhs(st.n, 71)
    f = W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    m, k, s = 60, 3, 120
    ref = krylov.fm(operators.as_matrix(st), b, f, m)
    A = ctx.matrix(st)
    p = make_params(m, k, s, "srht", 8, 9, "auto", "auto", tol)
    print(f"case auto policies tol={tol}", flush=True)
    out_b, info_b = ctx.solve(A, _dev(b), f, p)
    info_b = info_b[0]
    assert info_b["ls_iters"] > 0                       # the refinement ran
    if tol < 1e-6:
        assert info_b["fell_back"] == 1                 # FP32 rounding alone exceeds tol / 2
    ctx.set_block_limit(1)
    o = _dev(np.zeros(st.n))
    info_s = ctx.submit(A, _dev(b), f, p, o).wait()[0]
    ctx.set_block_limit(32)
    for key in ("fell_back", "ls_iters", "prec_used"):
        assert info_s[key] == info_b[key], key
    assert np.array_equal(o.cpu().numpy(), out_b.cpu().numpy())
    assert krylov.relerr(out_b.cpu().numpy(), ref) <= tol
    A.destroy()
