"""Parity of the sketched Gram-Schmidt basis (Algorithm 1) and Algorithm 3 on
the HIP path with the CPU oracle (``krylov.sketched_gs_basis`` / ``krylov.sgs``).

Tolerances: the Hessenberg matrix and the sketched basis agree with the
oracle's FP64 construction to 1e-9 relative (both run one classical
Gram-Schmidt step per column, so rounding differences stay at the level of
the sketch's conditioning); the result agrees with the oracle's exact
least-squares Algorithm 3 to 1e-10 (FP64 basis, tol = 1e-11: LSQR stops at
the Paige-Saunders test ||M^T r|| <= (tol/10) ||M||_F ||r||) and to 1e-6 with
an FP32 basis.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import closed_form, krylov, operators, sketch as osk

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


def _p(w, prec, ls="lsqr", tol=1e-11, m=None, basis="sketched_gs"):
    from paper_2212_12758_amd import make_params

    return make_params(m or w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, prec, ls, tol, basis=basis)


def _sk(w):
    return osk.Sketch(w.sketch, w.n, w.s, w.sketch_seed, w.zeta)


def _stagewise(ctx, w, b, ncols=None, tol_f=1e-10):
    """ncols: leading Hessenberg / sketch columns compared elementwise.  Like any
    Krylov recurrence, the construction amplifies rounding differences step by
    step (in the oracle alone, a relative perturbation of b by 1e-16 moves
    column 59 of H by 7e-4 on the 3D Laplacian with s = 63), so long runs are
    compared through what does not depend on that: Theta V orthonormal and the
    result, which depends only on the Krylov subspace."""
    Aor = operators.as_matrix(w.op)
    sk = _sk(w)
    ref = krylov.sgs(Aor, b, w.f, w.m, sk)
    A = ctx.matrix(w.op)
    out, info, dg = ctx.solve(A, _dev(b), w.f, _p(w, "fp64"), diag=True)
    out = out.cpu().numpy()
    mu = ref["m_used"]
    assert info[0]["m_used"] == mu and info[0]["breakdown"] == int(ref["breakdown"])
    H = ref["Hbar"]
    nc = mu if ncols is None else min(ncols, mu)
    assert np.abs(dg["hbar"][: nc + 1, :nc] - H[: nc + 1, :nc]).max() <= 1e-9 * np.abs(H).max()
    assert abs(info[0]["beta"] - ref["r11"]) <= 1e-13 * ref["r11"]
    SV = dg["sv"][:, : mu + 1]
    assert np.abs(SV[:, : nc + 1] - ref["S"][:, : nc + 1]).max() < 1e-9
    # one classical Gram-Schmidt step per column, as printed, loses
    # orthonormality when s is close to m (the oracle alone reaches 4e-3 on the
    # 3D Laplacian with m = 60, s = 63): no more than the oracle's own loss
    orth_ref = np.abs(ref["S"].T @ ref["S"] - np.eye(mu + 1)).max()
    assert np.abs(SV.T @ SV - np.eye(mu + 1)).max() <= max(10 * orth_ref, 1e-12)
    print("ls_iters", info[0]["ls_iters"], "relerr", krylov.relerr(out, ref["f"]), flush=True)
    assert info[0]["ls_limit"] == 0
    assert krylov.relerr(out, ref["f"]) < tol_f
    return A, Aor, ref, out, info


# ------------------------------------------------------------------ stencil, SRHT, ragged tiles
@pytest.mark.parametrize("N", [24, 31])
def test_bg_convdiff_srht_stagewise(ctx, N):
    base = W.config("convdiff3d_128_exp", scale=N)
    w = W.Workload(base.name, base.op, base.b_seed, 1, base.f, m=40, k=2, s=100, sketch="srht", sketch_seed=7)
    print(f"case bg convdiff N={N}", flush=True)
    b = W.rhs(w.n, w.b_seed)
    A, Aor, ref, out64, info = _stagewise(ctx, w, b)
    fm = krylov.fm(Aor, b, w.f, w.m)
    assert krylov.relerr(out64, fm) < 1e-10
    out32, info32 = ctx.solve(A, _dev(b), w.f, _p(w, "fp32", tol=1e-6))
    assert krylov.relerr(out32.cpu().numpy(), ref["f"]) < 1e-6
    A.destroy()


# ------------------------------------------------------------------ CSR graph, sparse sign, inverse square root
def test_bg_rgg_csr_sparse_sign_stagewise(ctx):
    print("case bg rgg n=5000", flush=True)
    op = W.rgg_laplacian(5000, seed=3)
    w = W.Workload("rgg", op, 3, 1, W.FuncSpec("pow", sigma=1e-3, p=-0.5), m=30, k=2, s=60,
                   sketch="sparse_sign", zeta=8, sketch_seed=3)
    b = W.rhs(w.n, 3)
    A, Aor, ref, out, info = _stagewise(ctx, w, b)
    assert info[0]["ls_iters"] >= 1
    A.destroy()


# ------------------------------------------------------------------ the timing workload, scaled: s = floor(1.05 m)
def test_bg_lap3d_invsqrt_small_sketch(ctx):
    print("case bg lap3d N=24 invsqrt", flush=True)
    base = W.config("lap3d_80_invsqrt", scale=24)
    m = 60
    w = W.Workload(base.name, base.op, base.b_seed, 1, base.f, m=m, k=2, s=int(1.05 * m), sketch="srht",
                   sketch_seed=base.sketch_seed)
    b = W.rhs(w.n, w.b_seed)
    # with s = 1.05 m one Gram-Schmidt pass leaves Theta V far from
    # orthonormal; preconditioned by the factor R of Theta V_m, LSQR still
    # meets its test within the iteration limit (about 95 iterations)
    A, Aor, ref, out, info = _stagewise(ctx, w, b, ncols=20)
    assert krylov.relerr(out, krylov.fm(Aor, b, w.f, m)) < 1e-10
    A.destroy()


# ------------------------------------------------------------------ the repeated Gram-Schmidt step on the sketch
def test_bg2_keeps_sketch_orthonormal_with_small_sketch(ctx):
    """s = 63 rows for m = 60: one pass loses the orthonormality of Theta V
    (the oracle alone reaches 3e-2), the repeated step keeps it to rounding;
    its result is the Arnoldi approximation f_m (exact least squares, here
    LSQR to convergence)."""
    st = W.laplacian3d(16)
    b = W.rhs(st.n, 4)
    m, s = 60, 63
    f = W.FuncSpec("pow", sigma=0.0, p=-0.5)
    w = W.Workload("lap3d16", st, 4, 1, f, m=m, k=2, s=s, sketch="srht", sketch_seed=5)
    Aor = operators.as_matrix(st)
    sk = _sk(w)
    ref = krylov.sgs(Aor, b, f, m, sk, passes=2)
    fm = krylov.fm(Aor, b, f, m)
    A = ctx.matrix(st)
    print("case bg2 lap3d16 fp64", flush=True)
    out, info, dg = ctx.solve(A, _dev(b), f, _p(w, "fp64", basis="sketched_gs2"), diag=True)
    out = out.cpu().numpy()
    assert info[0]["m_used"] == m and info[0]["breakdown"] == 0
    SV = dg["sv"]
    assert np.abs(SV.T @ SV - np.eye(m + 1)).max() < 1e-12
    H = ref["Hbar"]
    assert np.abs(dg["hbar"][:21, :20] - H[:21, :20]).max() <= 1e-9 * np.abs(H).max()
    assert krylov.relerr(out, ref["f"]) < 1e-10
    assert krylov.relerr(out, fm) < 1e-10
    print("case bg2 lap3d16 fp32", flush=True)
    out32, info32 = ctx.solve(A, _dev(b), f, _p(w, "fp32", tol=1e-6, basis="sketched_gs2"))
    assert krylov.relerr(out32.cpu().numpy(), fm) < 1e-6
    A.destroy()


# ------------------------------------------------------------------ invariant subspace
def test_bg_lucky_breakdown(ctx):
    d = np.repeat([0.5, 1.0, 2.0, 3.5, 5.0], 200)
    M = sp.diags(d).tocsr()
    op = (M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float32))
    b = W.rhs(d.size, 1)
    f = W.FuncSpec("exp", alpha=-1.0)
    A = ctx.matrix(op)
    for sketch in ("sparse_sign", "srht"):
        print(f"case bg breakdown {sketch}", flush=True)
        w = W.Workload("diag", op, 1, 1, f, m=12, k=2, s=40, sketch=sketch, sketch_seed=2)
        out, info = ctx.solve(A, _dev(b), f, _p(w, "fp64"))
        assert info[0]["breakdown"] == 1 and info[0]["m_used"] == 5
        assert krylov.relerr(out.cpu().numpy(), closed_form.diagonal_fAb(d, f, b)) < 1e-12
    A.destroy()


# ------------------------------------------------------------------ several right-hand sides, serving path
def test_bg_multi_rhs_and_serving(ctx):
    st = W.convdiff3d(20, 50.0)
    nrhs = 4
    w = W.Workload("mr", st, 50, nrhs, W.FuncSpec("exp", alpha=-1e-3), m=30, k=2, s=80, sketch="srht",
                   sketch_seed=5)
    B = W.rhs(st.n, 50, nrhs)
    A = ctx.matrix(st)
    print("case bg nrhs=4", flush=True)
    outB, infoB = ctx.solve(A, _dev(B), w.f, _p(w, "fp64"))
    outB = outB.cpu().numpy()
    Aor = operators.as_matrix(st)
    sk = _sk(w)
    for r in range(nrhs):
        ref = krylov.sgs(Aor, np.ascontiguousarray(B[:, r]), w.f, w.m, sk)
        assert krylov.relerr(outB[:, r], ref["f"]) < 1e-10, r
    print("case bg serving", flush=True)
    outs = _dev(np.zeros_like(B))
    info_s = ctx.submit(A, _dev(B), w.f, _p(w, "fp64"), outs).wait()
    assert np.array_equal(outs.cpu().numpy(), outB)
    assert [i["ls_iters"] for i in info_s] == [i["ls_iters"] for i in infoB]
    A.destroy()


def test_bg_auto_policies_refine(ctx):
    """With the sketched Gram-Schmidt basis the sketched least-squares solution
    is ~0 (Theta V is orthonormal), so FAB_LS_AUTO always refines by LSQR:
    Algorithm 3.  AUTO precision keeps the FP32 basis when its estimate passes."""
    from paper_2212_12758_amd import make_params

    st = W.laplacian2d(64)
    b = W.rhs(st.n, 5)
    f = W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    m = 60
    A = ctx.matrix(st)
    Aor = operators.as_matrix(st)
    fm = krylov.fm(Aor, b, f, m)
    print("case bg auto lap64 invsqrt", flush=True)
    p = make_params(m, 2, 2 * (m + 1), "sparse_sign", 8, 9, "auto", "auto", 1e-6, basis="sketched_gs")
    out, info = ctx.solve(A, _dev(b), f, p)
    assert info[0]["ls_iters"] >= 1
    assert krylov.relerr(out.cpu().numpy(), fm) < 1e-6
    ps = make_params(m, 2, 2 * (m + 1), "sparse_sign", 8, 9, "fp64", "sketch", 1e-6, basis="sketched_gs")
    out_s, info_s = ctx.solve(A, _dev(b), f, ps)
    assert info_s[0]["ls_iters"] == 0
    A.destroy()


def test_bg_invalid_basis(ctx):
    from paper_2212_12758_amd import EINVAL, FabError, make_params

    st = W.laplacian2d(30)
    A = ctx.matrix(st)
    b = _dev(W.rhs(st.n, 1))
    f = W.FuncSpec("exp", alpha=-1.0)
    with pytest.raises(FabError) as e:
        ctx.solve(A, b, f, make_params(20, 2, 60, "srht", 8, 1, "fp64", "lsqr", basis=4))
    assert e.value.code == EINVAL
    A.destroy()


# ------------------------------------------------------------------ beyond the LDS / register sizes
def test_bg2_large_m_global_paths(ctx):
    """m = 150, s = 320: the sketch columns exceed the LDS of the Gram-Schmidt
    step (chunked staging), R_m the full-storage LDS of the LSQR step (m > 140:
    packed triangle in LDS), H_hat the LDS of the quadrature square root
    (m > 128, four rows per lane) and the registers of the sketched QR
    (Householder in global memory), against the oracle's Algorithm 3 and
    Arnoldi's f_m; also the truncated basis with sketch-and-solve on the same
    problem.  m = 210, s = 440: R_m beyond the packed LDS size (global memory
    in the LSQR step)."""
    from paper_2212_12758_amd import make_params

    st = W.laplacian3d(24)
    b = W.rhs(st.n, 8)
    f = W.FuncSpec("pow", sigma=0.0, p=-0.5)
    m, s = 150, 320
    w = W.Workload("lap3d24", st, 8, 1, f, m=m, k=2, s=s, sketch="srht", sketch_seed=8)
    Aor = operators.as_matrix(st)
    sk = _sk(w)
    ref = krylov.sgs(Aor, b, f, m, sk, passes=2)
    fm = krylov.fm(Aor, b, f, m)
    A = ctx.matrix(st)
    print("case bg2 lap3d24 m=150 fp64", flush=True)
    out, info, dg = ctx.solve(A, _dev(b), f, _p(w, "fp64", basis="sketched_gs2"), diag=True)
    out = out.cpu().numpy()
    assert info[0]["m_used"] == m and info[0]["ls_iters"] >= 1
    SV = dg["sv"]
    assert np.abs(SV.T @ SV - np.eye(m + 1)).max() < 1e-12
    assert krylov.relerr(out, ref["f"]) < 1e-10
    assert krylov.relerr(out, fm) < 1e-10
    print("case truncated lap3d24 m=150 fp64", flush=True)
    out_t, _ = ctx.solve(A, _dev(b), f, make_params(m, 2, s, "srht", 8, 8, "fp64", "sketch"))
    ref_t = krylov.nt(Aor, b, f, m, 2, sk, "sketch")["f"]
    assert krylov.relerr(out_t.cpu().numpy(), ref_t) < 1e-10
    A.destroy()
    # m = 210 needs a larger grid: on 24^3 the Krylov space of that size is
    # numerically degenerate (kappa(V) ~ 1e10 in the oracle, ||H_hat|| ~ 1e11)
    st2 = W.laplacian3d(40)
    b2 = W.rhs(st2.n, 8)
    m2, s2 = 210, 440
    f2 = W.FuncSpec("exp", alpha=-0.05)
    w2 = W.Workload("lap3d40", st2, 8, 1, f2, m=m2, k=2, s=s2, sketch="srht", sketch_seed=8)
    ref2 = krylov.sgs(operators.as_matrix(st2), b2, f2, m2, _sk(w2), passes=2)
    A2 = ctx.matrix(st2)
    print("case bg2 lap3d40 m=210 fp64", flush=True)
    out2, info2 = ctx.solve(A2, _dev(b2), f2, _p(w2, "fp64", basis="sketched_gs2"))
    assert info2[0]["m_used"] == m2 and info2[0]["ls_iters"] >= 1
    assert krylov.relerr(out2.cpu().numpy(), ref2["f"]) < 1e-10
    A2.destroy()


def test_exp_norm_beyond_work_bound_is_refused(ctx):
    """The Taylor action needs ceil(||alpha H_hat||_1 / 4) steps; beyond 4096
    of them the solve returns FAB_ENUMERIC at once instead of running for a
    time proportional to the norm."""
    from paper_2212_12758_amd import ENUMERIC, FabError, make_params

    st = W.laplacian2d(30)
    b = W.rhs(st.n, 3)
    A = ctx.matrix(st)
    print("case exp refused", flush=True)
    with pytest.raises(FabError) as e:
        ctx.solve(A, _dev(b), W.FuncSpec("exp", alpha=-1e4), make_params(20, 2, 60, "srht", 8, 1, "fp64", "sketch"))
    assert e.value.code == ENUMERIC
    # just inside the bound: a result (||H_hat||_1 <= 16 for this Laplacian)
    out, _ = ctx.solve(A, _dev(b), W.FuncSpec("exp", alpha=-1.0), make_params(20, 2, 60, "srht", 8, 1, "fp64", "sketch"))
    assert np.isfinite(out.cpu().numpy()).all()
    A.destroy()


# ------------------------------------------------------------------ exact least squares through the Gram matrix
def test_gram_least_squares_exact_and_fallback(ctx):
    """FAB_LS_GRAM: with the two-pass sketched basis the normal equations give
    the exact least-squares solution of Algorithm 3 (oracle: dense lstsq) with
    no LSQR iteration; on the truncated basis of a graph Laplacian, whose
    conditioning is lost, the factorisation is refused and the result is the
    LSQR one, bit for bit."""
    from paper_2212_12758_amd import make_params

    st = W.laplacian3d(16)
    b = W.rhs(st.n, 4)
    m, s = 60, 63
    f = W.FuncSpec("pow", sigma=0.0, p=-0.5)
    w = W.Workload("lap3d16", st, 4, 1, f, m=m, k=2, s=s, sketch="srht", sketch_seed=5)
    Aor = operators.as_matrix(st)
    ref = krylov.sgs(Aor, b, f, m, _sk(w), passes=2)
    A = ctx.matrix(st)
    print("case gram bg2 lap3d16", flush=True)
    # kappa_1 of the Gram factor is 815 here (kappa_2 41; the oracle's basis,
    # numpy): accepted while kappa_1^2 u <= tol/10 (tol = 1e-9: bound 949),
    # refused for tol = 1e-10 (bound 300), where LSQR runs instead
    out, info = ctx.solve(A, _dev(b), f, _p(w, "fp64", ls="gram", tol=1e-9, basis="sketched_gs2"))
    assert info[0]["ls_iters"] == 0
    assert krylov.relerr(out.cpu().numpy(), ref["f"]) < 1e-11
    assert krylov.relerr(out.cpu().numpy(), krylov.fm(Aor, b, f, m)) < 1e-11
    out, info = ctx.solve(A, _dev(b), f, _p(w, "fp64", ls="gram", tol=1e-10, basis="sketched_gs2"))
    assert info[0]["ls_iters"] >= 1 and info[0]["ls_limit"] == 0
    assert krylov.relerr(out.cpu().numpy(), ref["f"]) < 1e-10
    A.destroy()
    n, m = 4096, 120
    op = W.rgg_laplacian(n, seed=3)
    fr = W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    br = W.rhs(n, 3)
    A = ctx.matrix(op)
    print("case gram fallback rgg4096", flush=True)
    # the truncated basis of this graph has lost its rank (kappa(V) ~ 1e12),
    # although every Cholesky pivot stays O(1): the kappa_1(R) estimate
    # refuses the factorisation, so FAB_LS_GRAM falls back to the LSQR path
    # and returns the same bits
    pg = make_params(m, 2, 2 * m, "sparse_sign", 8, 3, "fp64", "gram", 1e-10)
    pl = make_params(m, 2, 2 * m, "sparse_sign", 8, 3, "fp64", "lsqr", 1e-10)
    og, ig = ctx.solve(A, _dev(br), fr, pg)
    ol, il = ctx.solve(A, _dev(br), fr, pl)
    print("gram", ig[0], "lsqr", il[0], flush=True)
    assert ig[0]["ls_iters"] >= 1 and ig[0]["ls_iters"] == il[0]["ls_iters"]
    assert np.array_equal(og.cpu().numpy(), ol.cpu().numpy())
    A.destroy()
