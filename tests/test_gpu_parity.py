"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: relative 2-norm error 1e-10 for the FP64-basis form and 1e-6 for
the FP32-basis form against the oracle's f_m (eq. (4)) at the same m;
stage-by-stage (Hbar of eq. (3), Theta V, y of eq. (7), f(H_hat) e_1) against
the oracle's step-by-step Algorithm 2 + sketch-and-solve in FP64.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import closed_form, krylov, operators, sketch as osk

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-6


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


def _params(w, prec, ls="sketch", m=None, seed=None):
    from paper_2212_12758_amd import make_params

    return make_params(m or w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed if seed is None else seed, prec, ls)


def _solve(ctx, w, A, b, prec, ls="sketch", diag=False):
    out = ctx.solve(A, _dev(b), w.f, _params(w, prec, ls), diag=diag)
    if diag:
        return out[0].cpu().numpy(), out[1], out[2]
    return out[0].cpu().numpy(), out[1]


def _oracle(w, Aor, b, ls="sketch"):
    sk = osk.Sketch(w.sketch, w.n, w.s, w.sketch_seed, w.zeta)
    return krylov.nt(Aor, b, w.f, w.m, w.k, sk, ls), sk


# ------------------------------------------------------------------ config 1: 2D Laplacian, exp, sparse sign
def test_config1_lap2d_exp_fp64_stagewise(ctx):
    w = W.config("lap2d_100_exp")
    print("case lap2d_100 fp64", flush=True)
    Aor = operators.as_matrix(w.op)
    b = W.rhs(w.n, w.b_seed)
    A = ctx.matrix(w.op)
    out, info, dg = _solve(ctx, w, A, b, "fp64", diag=True)
    ref, sk = _oracle(w, Aor, b)
    fm = krylov.fm(Aor, b, w.f, w.m)
    assert info[0]["m_used"] == w.m and not info[0]["breakdown"]
    # Hbar (eq. (3)) and the norms
    H = ref["Hbar"]
    assert np.abs(dg["hbar"] - H).max() <= 1e-12 * np.abs(H).max()
    assert math.isclose(info[0]["beta"], np.linalg.norm(b), rel_tol=1e-14)
    # Theta v_1 = Theta b / ||b||: exact sketch pattern (indices, signs) check
    sv0 = sk.apply(b / np.linalg.norm(b))
    np.testing.assert_allclose(dg["sv"][:, 0], sv0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(dg["sv"], ref["SV"], rtol=0, atol=1e-11)
    np.testing.assert_allclose(dg["c"], ref["c"], rtol=0, atol=1e-11 * np.abs(ref["c"]).max())
    assert krylov.relerr(out, ref["f"]) < TOL64
    assert krylov.relerr(out, fm) < TOL64
    A.destroy()


def test_config1_lap2d_exp_fp32(ctx):
    w = W.config("lap2d_100_exp")
    Aor = operators.as_matrix(w.op)
    b = W.rhs(w.n, w.b_seed)
    A = ctx.matrix(w.op)
    out, info = _solve(ctx, w, A, b, "fp32")
    fm = krylov.fm(Aor, b, w.f, w.m)
    assert krylov.relerr(out, fm) < TOL32
    assert krylov.relerr(out, closed_form.laplacian_fAb(w.op, w.f, b)) < TOL32
    A.destroy()


# ------------------------------------------------------------------ 3D convection-diffusion, SRHT, ragged sizes
@pytest.mark.parametrize("N", [24, 31])
def test_convdiff_srht_ragged_fp64_and_fp32(ctx, N):
    base = W.config("convdiff3d_128_exp", scale=N)
    w = W.Workload(base.name, base.op, base.b_seed, 1, base.f, m=40, k=4, s=100, sketch="srht", sketch_seed=7)
    print(f"case convdiff N={N}", flush=True)
    Aor = operators.as_matrix(w.op)
    b = W.rhs(w.n, w.b_seed)
    A = ctx.matrix(w.op)
    out64, info64, dg = _solve(ctx, w, A, b, "fp64", diag=True)
    ref, sk = _oracle(w, Aor, b)
    fm = krylov.fm(Aor, b, w.f, w.m)
    H = ref["Hbar"]
    assert np.abs(dg["hbar"] - H).max() <= 1e-11 * np.abs(H).max()
    np.testing.assert_allclose(dg["sv"][:, 0], sk.apply(b / np.linalg.norm(b)), rtol=0, atol=1e-13)
    assert krylov.relerr(out64, ref["f"]) < TOL64
    assert krylov.relerr(out64, fm) < TOL64
    out32, info32 = _solve(ctx, w, A, b, "fp32")
    assert krylov.relerr(out32, fm) < TOL32
    A.destroy()


# ------------------------------------------------------------------ CSR random geometric graph, inverse square root
@pytest.mark.parametrize("n", [5000, 8192])
def test_rgg_csr_invsqrt_sparse_sign(ctx, n):
    print(f"case rgg n={n}", flush=True)
    op = W.rgg_laplacian(n, seed=3)
    w = W.Workload("rgg", op, 3, 1, W.FuncSpec("pow", sigma=1e-3, p=-0.5), m=30, k=2, s=60,
                   sketch="sparse_sign", zeta=8, sketch_seed=3)
    Aor = operators.as_matrix(op)
    b = W.rhs(n, 3)
    A = ctx.matrix(op)
    out64, info64, dg = _solve(ctx, w, A, b, "fp64", diag=True)
    ref, sk = _oracle(w, Aor, b)
    np.testing.assert_allclose(dg["sv"][:, 0], sk.apply(b / np.linalg.norm(b)), rtol=0, atol=1e-13)
    assert np.abs(dg["hbar"] - ref["Hbar"]).max() <= 1e-11 * np.abs(ref["Hbar"]).max()
    assert krylov.relerr(dg["c"], ref["c"]) < 1e-9
    assert krylov.relerr(out64, ref["f"]) < 1e-9
    A.destroy()


def test_sqrt_exp_functions_on_laplacian(ctx):
    st = W.laplacian2d(40, 37)
    b = W.rhs(st.n, 11)
    Aor = operators.as_matrix(st)
    A = ctx.matrix(st)
    for f in (W.FuncSpec("pow", sigma=0.0, p=0.5), W.FuncSpec("pow", sigma=1e-3, p=-0.5),
              W.FuncSpec("exp", alpha=-2.0)):
        print(f"case lap2d 40x37 {f}", flush=True)
        w = W.Workload("x", st, 11, 1, f, m=60, k=2, s=130, sketch="sparse_sign", sketch_seed=5)
        fm = krylov.fm(Aor, b, f, w.m)
        out, info = _solve(ctx, w, A, b, "fp64", ls="none")
        assert krylov.relerr(out, fm) < TOL64, f
    A.destroy()


# ------------------------------------------------------------------ exactness
def test_polynomial_exact_gpu(ctx):
    st = W.convdiff3d(12, 10.0)
    Aor = operators.as_matrix(st)
    b = W.rhs(st.n, 21)
    coef = (0.3, -1.0, 0.25, 2e-3, -5e-6, 1e-8)
    f = W.FuncSpec("poly", coef=coef)
    ref = np.zeros(st.n)
    for c in reversed(coef):
        ref = Aor @ ref + c * b
    A = ctx.matrix(st)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-6)):
        w = W.Workload("p", st, 21, 1, f, m=6, k=2, s=20, sketch="srht", sketch_seed=4)
        for ls in ("sketch", "none"):
            out, _ = _solve(ctx, w, A, b, prec, ls=ls)
            assert krylov.relerr(out, ref) < tol, (prec, ls)
    A.destroy()


def test_lucky_breakdown_gpu(ctx):
    d = np.repeat([0.5, 1.0, 2.0, 3.5, 5.0], 200).astype(np.float32)
    n = d.size
    M = sp.diags(d.astype(np.float64)).tocsr()
    op = (M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float32))
    b = W.rhs(n, 1)
    A = ctx.matrix(op)
    f = W.FuncSpec("exp", alpha=-1.0)
    w = W.Workload("diag", op, 1, 1, f, m=12, k=2, s=40, sketch="sparse_sign", sketch_seed=2)
    out, info = _solve(ctx, w, A, b, "fp64")
    assert info[0]["breakdown"] == 1 and info[0]["m_used"] == 5
    assert krylov.relerr(out, closed_form.diagonal_fAb(d, f, b)) < 1e-12
    A.destroy()


# ------------------------------------------------------------------ multiple right-hand sides
@pytest.mark.parametrize("nrhs", [2, 8])
def test_multi_rhs_equals_single(ctx, nrhs):
    st = W.convdiff3d(20, 50.0)
    w = W.Workload("mr", st, 50, nrhs, W.FuncSpec("exp", alpha=-1e-3), m=30, k=4, s=80, sketch="srht",
                   sketch_seed=5)
    B = W.rhs(st.n, 50, nrhs)
    A = ctx.matrix(st)
    outB, infoB = _solve(ctx, w, A, B, "fp64")
    Aor = operators.as_matrix(st)
    for r in range(nrhs):
        o1, _ = _solve(ctx, w, A, np.ascontiguousarray(B[:, r]), "fp64")
        assert krylov.relerr(outB[:, r], o1) < 1e-13
        assert krylov.relerr(outB[:, r], krylov.fm(Aor, B[:, r], w.f, w.m)) < TOL64
    A.destroy()


# ------------------------------------------------------------------ serving: same alone and in the mix
def test_serving_mix_equals_alone(ctx):
    import torch

    cases = []
    for i, (N, f) in enumerate([(20, W.FuncSpec("exp", alpha=-1e-3)), (33, W.FuncSpec("exp", alpha=-2e-3)),
                                (16, W.FuncSpec("exp", alpha=-1e-3))]):
        st = W.convdiff3d(N, 50.0)
        cases.append((st, f, W.rhs(st.n, 100 + i)))
    st2 = W.laplacian2d(64)
    cases.append((st2, W.FuncSpec("pow", sigma=1e-3, p=-0.5), W.rhs(st2.n, 7)))
    mats = [ctx.matrix(c[0]) for c in cases]
    from paper_2212_12758_amd import make_params

    params = [make_params(40, 3, 90, "srht", 8, 1000 + i, "fp32", "sketch") for i in range(len(cases))]
    # repeats of one case would be merged into block solves (equal to the
    # result alone within the tolerance, tests/test_gpu_serving_blocks.py);
    # without merging the served results are the blocking ones bit for bit
    ctx.set_block_limit(1)
    alone = []
    for (st, f, b), A, p in zip(cases, mats, params):
        o, _ = ctx.solve(A, _dev(b), f, p)
        alone.append(o.cpu().numpy())
    outs, reqs = [], []
    for rep in range(3):
        for (st, f, b), A, p in zip(cases, mats, params):
            bd = _dev(b)
            o = torch.empty_like(bd)
            reqs.append(ctx.submit(A, bd, f, p, o))
            outs.append(o)
    for r in reqs:
        r.wait()
    for j, o in enumerate(outs):
        ref = alone[j % len(cases)]
        assert np.array_equal(o.cpu().numpy(), ref), j        # fixed-order reductions: bitwise
    ctx.set_block_limit(32)
    for A in mats:
        A.destroy()


# ------------------------------------------------------------------ error paths
def test_error_paths(ctx):
    from paper_2212_12758_amd import EINVAL, ENUMERIC, FabError, make_params

    st = W.laplacian2d(30)
    A = ctx.matrix(st)
    b = W.rhs(st.n, 1)
    f = W.FuncSpec("exp", alpha=-1.0)
    with pytest.raises(FabError) as e:
        ctx.solve(A, _dev(b), f, make_params(20, 2, 20, "srht", 8, 1, "fp32"))   # s <= m
    assert e.value.code == EINVAL
    with pytest.raises(FabError) as e:
        ctx.solve(A, _dev(b), f, make_params(20, 9, 60, "srht", 8, 1, "fp32"))   # k > 8
    assert e.value.code == EINVAL
    bn = b.copy()
    bn[17] = np.nan
    with pytest.raises(FabError) as e:
        ctx.solve(A, _dev(bn), f, make_params(20, 2, 60, "srht", 8, 1, "fp32"))
    assert e.value.code == ENUMERIC
    # zero right-hand side: exact zero result, m_used = 0
    o, info = ctx.solve(A, _dev(np.zeros(st.n)), f, make_params(20, 2, 60, "srht", 8, 1, "fp32"))
    assert info[0]["m_used"] == 0 and float(o.abs().max()) == 0.0
    A.destroy()


def test_enomem_tiny_arena():
    import torch

    from paper_2212_12758_amd import ENOMEM, Context, FabError, make_params

    with Context(0, arena_bytes=2 << 20) as c:
        st = W.laplacian3d(64)
        A = c.matrix(st)
        b = torch.zeros(st.n, dtype=torch.float64, device="cuda")
        with pytest.raises(FabError) as e:
            c.solve(A, b, W.FuncSpec("exp", alpha=-1.0), make_params(50, 2, 120, "srht", 8, 1, "fp32"))
        assert e.value.code == ENOMEM
        A.destroy()


# ------------------------------------------------------------------ graph replay equals direct launches
def test_graph_replays_match_direct_launches():
    import os

    import torch

    from paper_2212_12758_amd import Context, make_params

    st = W.convdiff3d(40, 50.0)
    b = _dev(W.rhs(st.n, 9))
    f = W.FuncSpec("exp", alpha=-1e-3)
    p = make_params(40, 4, 100, "srht", 8, 3, "fp32", "sketch")
    os.environ["FAB_NO_GRAPH"] = "1"
    try:
        with Context(0, arena_bytes=1 << 30) as ce:
            Ae = ce.matrix(st)
            ref, _ = ce.solve(Ae, b, f, p)
            ref = ref.cpu().numpy()
            Ae.destroy()
    finally:
        del os.environ["FAB_NO_GRAPH"]
    with Context(0, arena_bytes=1 << 30) as cg:
        Ag = cg.matrix(st)
        out = torch.empty_like(b)
        for rep in range(5):
            junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
            torch.cuda.synchronize()
            cg.solve(Ag, b, f, p, out)
            assert np.array_equal(out.cpu().numpy(), ref), rep
            assert float(junk) == float(junk)
        Ag.destroy()


# ------------------------------------------------------------------ dense stages beyond the LDS/register sizes
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_large_m_global_memory_dense_path(ctx, prec, tol):
    st = W.laplacian2d(72)
    b = W.rhs(st.n, 13)
    Aor = operators.as_matrix(st)
    A = ctx.matrix(st)
    for f in (W.FuncSpec("exp", alpha=-0.5), W.FuncSpec("exp", alpha=-6.0)):     # no squaring / squaring
        w = W.Workload("big_m", st, 13, 1, f, m=120, k=2, s=250, sketch="sparse_sign", sketch_seed=8)
        print(f"case lap2d 72^2 m=120 {prec} {f.alpha}", flush=True)
        out, info = _solve(ctx, w, A, b, prec)
        assert info[0]["m_used"] == 120
        assert krylov.relerr(out, krylov.fm(Aor, b, f, w.m)) < tol
    A.destroy()



# ------------------------------------------------------------------ a-posteriori estimates and the FP64 fallback
def test_estimates_match_oracle_and_auto_precision(ctx):
    from paper_2212_12758_amd import make_params

    base = W.config("convdiff3d_128_exp", scale=24)
    w = W.Workload(base.name, base.op, base.b_seed, 1, base.f, m=40, k=4, s=100, sketch="srht", sketch_seed=7)
    print("case estimates convdiff N=24", flush=True)
    Aor = operators.as_matrix(w.op)
    b = W.rhs(w.n, w.b_seed)
    A = ctx.matrix(w.op)
    fm = krylov.fm(Aor, b, w.f, w.m)
    # FP64 basis with the estimates (ls auto): the values follow their definitions
    p64 = make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "fp64", "auto", 1e-10)
    out, info = ctx.solve(A, _dev(b), w.f, p64)
    ref, sk = _oracle(w, Aor, b)
    est = krylov.estimates(ref, w.f, 2.0**-53)
    for key in ("ls_gate", "conv_est", "round_est"):
        assert info[0][key] == pytest.approx(est[key], rel=1e-6, abs=1e-15), key
    assert info[0]["err_est"] == max(info[0]["ls_gate"], info[0]["round_est"])
    assert krylov.relerr(out.cpu().numpy(), fm) < TOL64
    # automatic precision, loose tolerance: the FP32 basis is accepted
    pa = make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "auto", "auto", 1e-6)
    out, info = ctx.solve(A, _dev(b), w.f, pa)
    assert info[0]["fell_back"] == 0 and info[0]["prec_used"] == 1
    assert info[0]["round_est"] <= 1e-6 / 4
    assert krylov.relerr(out.cpu().numpy(), fm) < TOL32
    # automatic precision, tolerance below FP32 rounding: recomputed with an FP64 basis
    pt = make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "auto", "auto", 1e-11)
    out, info = ctx.solve(A, _dev(b), w.f, pt)
    assert info[0]["fell_back"] == 1 and info[0]["prec_used"] == 2
    assert krylov.relerr(out.cpu().numpy(), fm) < TOL64
    # the same through the serving path
    outs = _dev(np.zeros(w.n))
    req = ctx.submit(A, _dev(b), w.f, pt, outs)
    info = req.wait()
    assert info[0]["fell_back"] == 1 and info[0]["prec_used"] == 2
    assert krylov.relerr(outs.cpu().numpy(), fm) < TOL64
    A.destroy()


def test_estimates_sqrt_variants_and_breakdown(ctx):
    from paper_2212_12758_amd import make_params

    st = W.laplacian2d(40, 37)
    b = W.rhs(st.n, 11)
    Aor = operators.as_matrix(st)
    A = ctx.matrix(st)
    f = W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    w = W.Workload("lap", st, 11, 1, f, m=30, k=2, s=70, sketch="sparse_sign", sketch_seed=4)
    print("case estimates invsqrt", flush=True)
    # tolerance loose enough that the gate passes: no refinement, the
    # estimates of the sketch-and-solve result are reported
    p = make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "fp64", "auto", 1.0)
    out, info = ctx.solve(A, _dev(b), f, p)
    assert info[0]["ls_iters"] == 0
    ref, sk = _oracle(w, Aor, b)
    est = krylov.estimates(ref, f, 2.0**-53)
    for key in ("ls_gate", "conv_est"):
        assert info[0][key] == pytest.approx(est[key], rel=1e-5, abs=1e-14), key
    # lucky breakdown: exact result, both estimates 0
    d = np.repeat([0.5, 1.0, 2.0, 3.5, 5.0], 40)
    M = sp.diags(d).tocsr()
    bd = W.rhs(len(d), 3)
    Ad = ctx.matrix((M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float32)))
    fe = W.FuncSpec("exp", alpha=-0.3)
    pd = make_params(12, 2, 40, "sparse_sign", 8, 2, "fp64", "auto", 1e-10)
    out, info = ctx.solve(Ad, _dev(bd), fe, pd)
    assert info[0]["breakdown"] == 1 and info[0]["m_used"] == 5
    assert info[0]["ls_gate"] == 0.0 and info[0]["conv_est"] == 0.0
    assert krylov.relerr(out.cpu().numpy(), closed_form.diagonal_fAb(d, fe, bd)) < 1e-12
    Ad.destroy()
    A.destroy()


# ------------------------------------------------------------------ LSQR refinement of the least squares
def test_lsqr_refinement_recovers_exact_least_squares(ctx):
    """Unconverged inverse square root: sketch-and-solve moves the result by
    ~1e-2 from f_m, the exact least-squares solution reaches f_m (Lemma 2);
    the preconditioned LSQR refinement (AUTO after the gate, or forced) must
    close that gap, through the blocking and the serving path alike."""
    from paper_2212_12758_amd import make_params

    st = W.laplacian2d(64)
    b = W.rhs(st.n, 5)
    f = W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    m = 60
    w = W.Workload("lap64", st, 5, 1, f, m=m, k=2, s=2 * (m + 1), sketch="sparse_sign", sketch_seed=9)
    print("case lsqr lap64 invsqrt", flush=True)
    Aor = operators.as_matrix(st)
    A = ctx.matrix(st)
    fm = krylov.fm(Aor, b, f, m)
    ref_sk, _ = _oracle(w, Aor, b)
    out_sk, info_sk = _solve(ctx, w, A, b, "fp64", ls="sketch")
    assert krylov.relerr(out_sk, ref_sk["f"]) < 1e-9
    err_sk = krylov.relerr(out_sk, fm)
    assert err_sk > 1e-3
    for ls in ("auto", "lsqr"):
        p = make_params(m, 2, w.s, "sparse_sign", 8, 9, "fp64", ls, 1e-11)
        out, info = ctx.solve(A, _dev(b), f, p)
        out = out.cpu().numpy()
        assert info[0]["ls_iters"] >= 1 and info[0]["ls_limit"] == 0, (ls, info[0])
        assert krylov.relerr(out, fm) < 1e-10, (ls, krylov.relerr(out, fm))
        assert krylov.relerr(out, fm) < 1e-3 * err_sk
    outs = _dev(np.zeros(st.n))
    p = make_params(m, 2, w.s, "sparse_sign", 8, 9, "fp64", "auto", 1e-11)
    info_s = ctx.submit(A, _dev(b), f, p, outs).wait()
    out_b, info_b = ctx.solve(A, _dev(b), f, p)
    assert info_s[0]["ls_iters"] == info_b[0]["ls_iters"] >= 1
    assert np.array_equal(outs.cpu().numpy(), out_b.cpu().numpy())
    A.destroy()
