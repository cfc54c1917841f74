"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to something the mathematics or an
independent routine fixes: published generator outputs, a library Hadamard
matrix, dense eigendecomposition, closed forms, invariants and exactness
results stated in the paper.  A plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand) fails at least one of them; the
mutation tests at the end plant such slips and check that they are caught.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import workloads as W
from oracle import closed_form, krylov, matfun, operators, rng, sketch

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
GOLD = os.path.join(os.path.dirname(__file__), "golden")
EXP1 = W.FuncSpec("exp", alpha=-1.0)


def _rand_nonsym(n, seed, shift=0.0):
    r = np.random.default_rng(seed)
    return r.standard_normal((n, n)) / math.sqrt(n) + shift * np.eye(n)


def _rand_spd(n, seed, lo=0.5, hi=4.0):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    return (Q * np.linspace(lo, hi, n)) @ Q.T


# --------------------------------------------------------------------------- RNG
def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt")) if l.startswith("0x")]
    assert [rng.out(0, i) for i in range(4)] == vals
    assert list(rng.values(0, 0, np.arange(3))) == [rng.value(0, 0, i) for i in range(3)]


# --------------------------------------------------------------------------- SRHT
@pytest.mark.parametrize("p", [0, 1, 3, 6, 10])
def test_fwht_matches_library_sylvester_hadamard(p):
    n = 1 << p
    x = np.random.default_rng(p).standard_normal((n, 3))
    np.testing.assert_allclose(sketch.fwht(x), sl.hadamard(n) @ x, rtol=0, atol=1e-12 * n)


@pytest.mark.parametrize("n,s,seed", [(37, 11, 5), (64, 64, 1), (1000, 40, 9)])
def test_srht_is_scaled_rows_of_HD(n, s, seed):
    npad = sketch.next_pow2(n)
    rows = sketch.srht_rows(n, s, seed)
    assert len(set(rows.tolist())) == s and rows.min() >= 0 and rows.max() < npad
    d = sketch.srht_signs(n, seed)
    ref = sl.hadamard(npad)[rows][:, :n] * d[None, :] / math.sqrt(s)
    np.testing.assert_allclose(sketch.srht_apply(np.eye(n), s, seed), ref, atol=1e-14)
    np.testing.assert_allclose(sketch.srht_dense(n, s, seed), ref, atol=0)


def test_srht_embedding_statistics():
    n, m, s = 4096, 20, 200
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((n, m)))
    norms, conds = [], []
    for seed in range(40):
        SQ = sketch.srht_apply(Q, s, seed)
        sv = np.linalg.svd(SQ, compute_uv=False)
        conds.append(sv[0] / sv[-1])
        norms.append(np.sum(SQ[:, 0] ** 2))
    assert abs(np.mean(norms) - 1.0) < 0.1          # E ||Theta x||^2 = ||x||^2
    assert np.median(conds) < 3.0                    # subspace embedding for s = 10 m
    signs = sketch.srht_signs(100000, 3)
    assert abs(signs.mean()) < 0.02


# --------------------------------------------------------------------------- sparse sign
def test_sparse_sign_columns_exact_structure():
    n, s, zeta = 5000, 82, 8
    rows, signs = sketch.sparse_sign_pattern(n, s, zeta, 1)
    assert rows.min() >= 0 and rows.max() < s
    assert all(len(set(r)) == zeta for r in rows.tolist())
    T = sketch.sparse_sign_matrix(n, s, zeta, 1)
    colnorm = np.sqrt(np.asarray(T.multiply(T).sum(axis=0))).ravel()
    np.testing.assert_allclose(colnorm, 1.0, rtol=1e-15)     # each column has unit norm
    assert set(np.unique(T.data).round(12)) == {round(1 / math.sqrt(zeta), 12), round(-1 / math.sqrt(zeta), 12)}


def test_sparse_sign_floyd_is_uniform():
    n, s, zeta = 200000, 40, 8
    rows, signs = sketch.sparse_sign_pattern(n, s, zeta, 7)
    counts = np.bincount(rows.ravel(), minlength=s)
    expected = n * zeta / s
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 2.5 * s                                     # dof = s-1
    assert abs(signs.mean()) < 0.01


def test_sparse_sign_embedding():
    n, m, s = 3000, 15, 150
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((n, m)))
    conds = [np.linalg.cond(sketch.Sketch("sparse_sign", n, s, seed).apply(Q)) for seed in range(10)]
    assert np.median(conds) < 3.0


# --------------------------------------------------------------------------- operators
def test_stencil_matrix_entries():
    st = W.Stencil(3, 4, 3, 2, (7.0, -1.0, -2.0, -3.0, -4.0, -5.0, -6.0))
    A = operators.stencil_matrix(st).toarray()
    idx = lambda x, y, z: x + 4 * (y + 3 * z)
    assert A[idx(1, 1, 1), idx(1, 1, 1)] == 7.0
    assert A[idx(1, 1, 1), idx(0, 1, 1)] == -1.0 and A[idx(1, 1, 1), idx(2, 1, 1)] == -2.0
    assert A[idx(1, 1, 1), idx(1, 0, 1)] == -3.0 and A[idx(1, 1, 1), idx(1, 2, 1)] == -4.0
    assert A[idx(1, 1, 1), idx(1, 1, 0)] == -5.0 and A[idx(1, 1, 0), idx(1, 1, 1)] == -6.0
    assert A[idx(3, 0, 0), idx(0, 1, 0)] == 0.0        # no wrap-around at the x boundary
    assert np.count_nonzero(A[idx(0, 0, 0)]) == 4


def test_convdiff_scaling_and_upwinding():
    st = W.convdiff3d(8, 50.0)
    A = operators.stencil_matrix(st)
    absA = abs(A)
    assert math.isclose(absA.sum(axis=1).max(), 1e3, rel_tol=1e-12)
    assert math.isclose(absA.sum(axis=0).max(), 1e3, rel_tol=1e-12)
    c, xm, xp = st.coeff[:3]
    assert xm < xp < 0 < c                             # upstream neighbour carries the convection
    assert np.linalg.norm(A.toarray(), 2) <= 1e3


def test_rgg_laplacian_properties():
    rowptr, col, val = W.rgg_laplacian(4096, seed=3)
    L = operators.csr_matrix(rowptr, col, val)
    assert abs(L - L.T).max() == 0
    np.testing.assert_allclose(np.asarray(L.sum(axis=1)).ravel(), 0.0, atol=0)
    deg = np.diff(rowptr) - 1
    assert 8.0 < deg.mean() < 11.0
    assert all(np.all(np.diff(col[rowptr[i]:rowptr[i + 1]]) > 0) for i in range(0, 4096, 97))


# --------------------------------------------------------------------------- matrix functions
def test_matfun_against_eigendecomposition():
    K = _rand_spd(30, 1)
    lam, X = np.linalg.eigh(K)
    e1 = np.eye(30)[:, 0]
    for f in (W.FuncSpec("exp", alpha=-0.7), W.FuncSpec("pow", sigma=1e-3, p=0.5),
              W.FuncSpec("pow", sigma=1e-3, p=-0.5), W.FuncSpec("poly", coef=(1.0, -2.0, 0.5))):
        ref = X @ (matfun.fscalar(f, lam) * X[0])
        np.testing.assert_allclose(matfun.fmat_e1(f, K), ref, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(matfun.fmat(f, K)[:, 0], ref, rtol=1e-11, atol=1e-12)
    assert np.allclose(e1, e1)


def test_matfun_sqrt_nonsymmetric_squares_back():
    K = np.triu(_rand_nonsym(25, 4, shift=3.0), -1)   # Hessenberg, spectrum in the right half plane
    R = matfun.fmat(W.FuncSpec("pow", sigma=0.0, p=0.5), K)
    np.testing.assert_allclose(R @ R, K, atol=1e-11)
    x = matfun.fmat_e1(W.FuncSpec("pow", sigma=0.0, p=-0.5), K)
    np.testing.assert_allclose(R @ x, np.eye(25)[:, 0], atol=1e-11)


# --------------------------------------------------------------------------- Arnoldi and f_m
def test_arnoldi_relation_and_orthonormality():
    A = sp.csr_matrix(_rand_nonsym(200, 3))
    b = np.random.default_rng(4).standard_normal(200)
    U, K, beta, mu = krylov.arnoldi(A, b, 40)
    assert mu == 40
    nA = np.linalg.norm(A.toarray(), 2)
    assert np.abs(U @ U.T - np.eye(41)).max() < 1e-13
    assert np.abs(A @ U[:40].T - U.T @ K).max() < 1e-13 * nA
    assert np.all(np.tril(K, -2) == 0)
    np.testing.assert_allclose(U[0] * beta, b, rtol=1e-15)
    np.testing.assert_allclose(U[:40] @ (A @ U[:40].T), K[:40], atol=1e-13 * nA)


@pytest.mark.parametrize("f", [W.FuncSpec("exp", alpha=-0.5), W.FuncSpec("pow", sigma=0.1, p=0.5),
                               W.FuncSpec("pow", sigma=0.1, p=-0.5)])
def test_fm_full_dimension_equals_dense_fAb(f):
    n = 40
    A = _rand_spd(n, 11, lo=0.1, hi=3.0)
    b = np.random.default_rng(5).standard_normal(n)
    ref = closed_form.dense_fAb(A, f, b, symmetric=True)
    assert krylov.relerr(krylov.fm(sp.csr_matrix(A), b, f, n), ref) < 1e-11


def test_fm_nonsymmetric_converges_to_dense():
    n = 300
    A = _rand_nonsym(n, 8)
    b = np.random.default_rng(9).standard_normal(n)
    ref = closed_form.dense_fAb(A, EXP1, b)
    np.testing.assert_allclose(ref, sl.expm(-A) @ b, rtol=1e-10, atol=1e-12)
    assert krylov.relerr(krylov.fm(sp.csr_matrix(A), b, EXP1, 30), ref) < 1e-12


def test_minimal_polynomial_exactness_and_breakdown():
    d = np.repeat([0.5, 1.0, 2.0, 3.5, 5.0], 40)            # 5 distinct eigenvalues
    A = sp.diags(d)
    b = np.random.default_rng(1).standard_normal(d.size)
    U, K, beta, mu = krylov.arnoldi(A, b, 12)
    assert mu == 5
    for f in (EXP1, W.FuncSpec("pow", sigma=0.0, p=-0.5)):
        ref = closed_form.diagonal_fAb(d, f, b)
        assert krylov.relerr(krylov.fm(A, b, f, 12), ref) < 1e-12
        r = krylov.nt(A, b, f, 12, 2, None, "none")           # symmetric, k=2: also breaks down at 5
        assert r["breakdown"] and r["m_used"] == 5
        assert krylov.relerr(r["f"], ref) < 1e-11


def test_polynomial_exactness_all_variants():
    """Every method is exact for polynomials of degree <= m-1 (consequence of Theorem 6)."""
    n, m = 400, 8
    A = sp.csr_matrix(_rand_nonsym(n, 21))
    b = np.random.default_rng(22).standard_normal(n)
    coef = (0.3, -1.0, 0.25, 2.0, -0.5, 0.1, 0.05, -0.01)      # degree 7 = m - 1
    f = W.FuncSpec("poly", coef=coef)
    ref = np.zeros(n)
    for c in reversed(coef):                                   # Horner with explicit matvecs
        ref = A @ ref + c * b
    sk = sketch.Sketch("srht", n, 3 * m, 5)
    assert krylov.relerr(krylov.fm(A, b, f, m), ref) < 1e-12
    for ls in ("exact", "sketch", "none"):
        assert krylov.relerr(krylov.nt(A, b, f, m, 2, sk, ls)["f"], ref) < 1e-10
    assert krylov.relerr(krylov.sfom(A, b, f, m, 2, sk), ref) < 1e-10


# --------------------------------------------------------------------------- closed forms
def test_dst_closed_form_matches_dense_eigendecomposition():
    for st in (W.laplacian2d(7, 5), W.laplacian3d(5)):
        A = operators.stencil_matrix(st).toarray()
        b = np.random.default_rng(st.n).standard_normal(st.n)
        for f in (EXP1, W.FuncSpec("pow", sigma=1e-3, p=-0.5)):
            np.testing.assert_allclose(closed_form.laplacian_fAb(st, f, b),
                                       closed_form.dense_fAb(A, f, b, symmetric=True), rtol=1e-11, atol=1e-12)


def test_fm_at_config1_matches_dst_closed_form():
    w = W.config("lap2d_100_exp")
    A = operators.as_matrix(w.op)
    b = W.rhs(w.n, w.b_seed)
    assert krylov.relerr(krylov.fm(A, b, w.f, w.m), closed_form.laplacian_fAb(w.op, w.f, b)) < 1e-13


def test_kronecker_exp_closed_form_matches_dense_expm():
    # nonsymmetric (upwind) operator with distinct grid sides, so a transposed
    # factor or a swapped axis changes the result
    cd = W.convdiff3d(5, 100.0).coeff
    for st in (W.Stencil(3, 6, 5, 4, cd), W.laplacian2d(7, 5), W.Stencil(2, 7, 5, 1, cd[:5] + (0.0, 0.0))):
        A = operators.stencil_matrix(st).toarray()
        b = np.random.default_rng(st.n).standard_normal((st.n, 3))
        alpha = -0.7 / np.abs(A).sum(axis=1).max() * 1e3 if st.dim == 3 else -0.3
        ref = sl.expm(alpha * A) @ b
        got = closed_form.kronecker_exp_fAb(st, alpha, b)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        # one column at a time gives the same
        np.testing.assert_allclose(closed_form.kronecker_exp_fAb(st, alpha, b[:, 1]), got[:, 1], rtol=0, atol=0)
    # a transposed x factor is a plausible slip; it is visible on the upwind operator
    st = W.Stencil(3, 6, 5, 4, cd)
    A = operators.stencil_matrix(st).toarray()
    At = operators.stencil_matrix(W.Stencil(3, 6, 5, 4, (cd[0], cd[2], cd[1]) + cd[3:])).toarray()
    b = np.random.default_rng(1).standard_normal(st.n)
    assert krylov.relerr(sl.expm(-0.7 * At) @ b, sl.expm(-0.7 * A) @ b) > 1e-3


def test_kronecker_exp_matches_dst_and_converged_fm():
    st = W.laplacian3d(9)
    b = np.random.default_rng(2).standard_normal(st.n)
    np.testing.assert_allclose(closed_form.kronecker_exp_fAb(st, -1.0, b),
                               closed_form.laplacian_fAb(st, EXP1, b), rtol=1e-12, atol=1e-13)
    # the scaled 3D convection-diffusion exponential with ||tA||_inf = 1: full
    # Arnoldi has converged long before m = 200, so f_m equals exp(tA) b
    w = W.config("convdiff3d_256_exp_8rhs", scale=14)
    b = W.rhs(w.n, w.b_seed)
    ref = closed_form.kronecker_exp_fAb(w.op, w.f.alpha, b)
    assert krylov.relerr(krylov.fm(operators.as_matrix(w.op), b, w.f, 40), ref) < 1e-13


# --------------------------------------------------------------------------- Algorithm 2 and the compression
def test_truncated_basis_relation_window_orthogonality():
    n, m, k = 500, 30, 3
    A = sp.csr_matrix(_rand_nonsym(n, 31))
    b = np.random.default_rng(32).standard_normal(n)
    V, H, beta, mu, brk = krylov.truncated_arnoldi(A, b, m, k)
    assert not brk and mu == m
    np.testing.assert_allclose(A @ V[:m].T, V.T @ H, atol=1e-12)           # eq. (3)
    G = V @ V.T
    for i in range(m + 1):
        for j in range(max(0, i - k), i):
            assert abs(G[i, j]) < 1e-13
    np.testing.assert_allclose(np.diag(G), 1.0, atol=1e-14)
    assert np.all(np.triu(H[:m, :m], k) == 0)                                 # band: k - 1 above the diagonal
    assert np.all(np.tril(H, -2) == 0)


def test_compression_update_eq6_and_gamma_b():
    n, m, k = 300, 12, 2
    A = _rand_nonsym(n, 41)
    b = np.random.default_rng(42).standard_normal(n)
    V, H, beta, mu, _ = krylov.truncated_arnoldi(sp.csr_matrix(A), b, m, k)
    Vm = V[:m].T
    P = np.linalg.pinv(Vm)
    y = P @ V[m]
    lhs = P @ A @ Vm
    rhs = H[:m].copy()
    rhs[:, -1] += H[m, m - 1] * y
    np.testing.assert_allclose(lhs, rhs, atol=1e-10)
    e1 = np.zeros(m)
    e1[0] = np.linalg.norm(b)
    np.testing.assert_allclose(P @ b, e1, atol=1e-10)


def test_basis_invariance_lemma2():
    n, m = 250, 15
    A = _rand_nonsym(n, 51)
    b = np.random.default_rng(52).standard_normal(n)
    f = W.FuncSpec("exp", alpha=-0.3)
    U, K, beta, _ = krylov.arnoldi(sp.csr_matrix(A), b, m)
    R = np.triu(np.random.default_rng(53).standard_normal((m, m))) + 3 * np.eye(m)
    V = U[:m].T @ R
    P = np.linalg.pinv(V)
    alt = V @ (matfun.fmat(f, P @ A @ V) @ (P @ b))
    assert krylov.relerr(alt, krylov.fm(sp.csr_matrix(A), b, f, m)) < 1e-11
    r = krylov.nt(sp.csr_matrix(A), b, f, m, 3, None, "exact")
    assert krylov.relerr(r["f"], krylov.fm(sp.csr_matrix(A), b, f, m)) < 1e-11


def test_lanczos_equivalence_symmetric_k2():
    n, m = 400, 10
    A = sp.csr_matrix(_rand_spd(n, 61))
    b = np.random.default_rng(62).standard_normal(n)
    U, K, _, _ = krylov.arnoldi(A, b, m)
    V, H, _, _, _ = krylov.truncated_arnoldi(A, b, m, 2)
    np.testing.assert_allclose(H, K, atol=1e-12)
    np.testing.assert_allclose(np.abs(V @ U.T), np.eye(m + 1), atol=1e-11)


def test_sfom_equals_sketch_and_solve_remark3():
    n, m = 600, 8
    A = sp.csr_matrix(_rand_nonsym(n, 71, shift=0.5))
    b = np.random.default_rng(72).standard_normal(n)
    f = W.FuncSpec("exp", alpha=-3.0)
    for kind in ("srht", "sparse_sign"):
        sk = sketch.Sketch(kind, n, 2 * m, 3)
        a = krylov.sfom(A, b, f, m, 2, sk)
        bb = krylov.nt(A, b, f, m, 2, sk, "sketch")["f"]
        assert krylov.relerr(a, bb) < 1e-9
        assert krylov.relerr(a, krylov.fm(A, b, f, m)) > 1e-12       # not trivially converged


# --------------------------------------------------------------------------- mutation tests (planted slips)
def test_planted_sign_slip_in_algorithm2_is_caught(monkeypatch):
    orig = krylov.truncated_arnoldi

    def slipped(A, b, m, k):
        V, H, beta, mu, brk = orig(A, b, m, k)
        H = H.copy()
        H[0, 1] = -H[0, 1]            # a wrong sign on one coefficient
        return V, H, beta, mu, brk

    n, m, k = 300, 10, 3
    A = sp.csr_matrix(_rand_nonsym(n, 81))
    b = np.random.default_rng(82).standard_normal(n)
    V, H, *_ = slipped(A, b, m, k)
    assert np.linalg.norm(A @ V[:m].T - V.T @ H) > 1e-3


def test_planted_transpose_slip_in_fm_is_caught():
    n, m = 200, 20
    A = _rand_nonsym(n, 91)
    b = np.random.default_rng(92).standard_normal(n)
    U, K, beta, mu = krylov.arnoldi(sp.csr_matrix(A), b, m)
    wrong = beta * (U[:m].T @ matfun.fmat(EXP1, K[:m, :m].T)[:, 0])
    ref = closed_form.dense_fAb(A, EXP1, b)
    assert krylov.relerr(krylov.fm(sp.csr_matrix(A), b, EXP1, m), ref) < 1e-12
    assert krylov.relerr(wrong, ref) > 1e-6


def test_estimates_definitions_pinned():
    """a-posteriori quantities: the order-m_d variant equals the method run at
    m_d (same basis prefix, leading block of the same QR factor); the gate is
    exactly 0 without a least-squares column; the sketched norms agree with
    the true norms of V_m x within the embedding distortion."""
    st = W.convdiff3d(14, 50.0)
    A = operators.as_matrix(st)
    b = W.rhs(st.n, 21)
    f = W.FuncSpec("exp", alpha=-2e-3)
    m, k, s = 30, 3, 120
    sk = sketch.Sketch("sparse_sign", st.n, s, 5, 8)
    res = krylov.nt(A, b, f, m, k, sk, "sketch")
    est = krylov.estimates(res, f, 2.0**-53)
    md = m - max(5, m // 10)
    res_d = krylov.nt(A, b, f, md, k, sk, "sketch")
    R = res["R"]
    c = res["c"]
    cd = np.zeros(m)
    cd[:md] = res_d["c"]
    assert np.linalg.norm(R @ (c - cd)) / np.linalg.norm(R @ c) == pytest.approx(est["conv_est"], rel=1e-8)
    V = res["V"][:m].T
    true_conv = np.linalg.norm(V @ (c - cd)) / np.linalg.norm(V @ c)
    assert true_conv / 3 <= est["conv_est"] <= 3 * true_conv
    c0 = krylov.nt(A, b, f, m, k, sk, "none")["c"]
    true_gate = np.linalg.norm(V @ (c - c0)) / np.linalg.norm(V @ c)
    assert true_gate / 3 <= est["ls_gate"] <= 3 * true_gate
    assert est["round_est"] >= 2.0**-53   # sum_j |c_j| ||R e_j|| >= ||R c||
    none = krylov.nt(A, b, f, m, k, sk, "none")
    assert krylov.estimates(none, f, 2.0**-24)["ls_gate"] == 0.0


def _fp32_storage_basis(A, b, m, k):
    """Algorithm 2 with every basis vector rounded to FP32 as it is stored
    (the arithmetic stays FP64): the basis the FP32 path builds."""
    n = b.size
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    beta = float(np.linalg.norm(b))
    V[0] = (b / beta).astype(np.float32)
    for i in range(1, m + 1):
        w = A @ V[i - 1]
        for j in range(max(0, i - k), i):
            H[j, i - 1] = V[j] @ w
            w = w - H[j, i - 1] * V[j]
        H[i, i - 1] = np.linalg.norm(w)
        V[i] = (w / H[i, i - 1]).astype(np.float32)
    return V, H, beta


@pytest.mark.parametrize("case", ["convdiff3d_exp", "lap2d_invsqrt", "rgg_invsqrt"])
def test_round_est_pinned_against_fp32_rounding(case):
    """The rounding estimate round_est = u sum_j |c_j| ||R e_j|| / ||R c||
    (the FAB_PREC_AUTO fallback rule rests on it) against what rounding the
    basis to FP32 actually does, on three operator families:

    * storage rounding: rounding each v_j of the FP64 basis to FP32 moves
      V_m c by `actual`; |fl(x) - x| <= u |x| gives the exact first-order
      bound actual <= u sum_j |c_j| ||v_j|| / ||V_m c||;
    * round_est is that bound with norms taken through the sketch (within
      the embedding distortion, here 25%), and it overestimates `actual` by
      at most C = 20 (rounding errors of different vectors add like random
      vectors, not linearly);
    * on the converged workloads (least-squares gate far below u) the whole
      FP32-storage method, run step by step with rounded vectors, lands
      within round_est of the FP64 result.
    A unit roundoff of 2^-53 or a dropped |c_j| weight fails these bounds."""
    u32 = 2.0 ** -24
    if case == "convdiff3d_exp":
        st = W.convdiff3d(16, 50.0)
        A, b, f = operators.as_matrix(st), W.rhs(st.n, 2), W.FuncSpec("exp", alpha=-1e-3)
        m, k, s, kind = 60, 4, 240, "srht"
    elif case == "lap2d_invsqrt":
        st = W.laplacian2d(64)
        A, b, f = operators.as_matrix(st), W.rhs(st.n, 3), W.FuncSpec("pow", sigma=1e-3, p=-0.5)
        m, k, s, kind = 80, 2, 200, "sparse_sign"
    else:
        A = operators.as_matrix(W.rgg_laplacian(4096, seed=3))
        b, f = W.rhs(4096, 3), W.FuncSpec("pow", sigma=1e-3, p=-0.5)
        m, k, s, kind = 60, 2, 120, "sparse_sign"
    sk = sketch.Sketch(kind, b.size, s, 5, 8)
    res = krylov.nt(A, b, f, m, k, sk, "sketch")
    est = krylov.estimates(res, f, u32)["round_est"]
    mu = res["m_used"]
    V, c = res["V"][:mu].T, res["c"]
    nvc = np.linalg.norm(V @ c)
    actual = np.linalg.norm((V.astype(np.float32).astype(np.float64) - V) @ c) / nvc
    bound = u32 * float(np.abs(c) @ np.linalg.norm(V, axis=0)) / nvc
    assert actual <= bound
    assert 0.8 * bound <= est <= 1.25 * bound
    assert actual <= est <= 20.0 * actual
    # planted slips: FP64's unit roundoff, or the weights |c_j| dropped
    assert krylov.estimates(res, f, 2.0 ** -53)["round_est"] < actual
    R = res["R"][:mu, :mu]
    assert u32 * float(np.linalg.norm(R, axis=0).sum()) / np.linalg.norm(R @ c) > 20.0 * actual
    if case in ("convdiff3d_exp",):
        # end to end: the FP32-storage method (sketch-and-solve, as the FP32 path)
        Vs, H, beta = _fp32_storage_basis(A, b, m, k)
        SV = sk.apply(Vs.T)
        Q, Rs = np.linalg.qr(SV[:, :m])
        y = sl.solve_triangular(Rs, Q.T @ SV[:, m])
        Hh = H[:m, :m].copy()
        Hh[:, m - 1] += H[m, m - 1] * y
        e2e = krylov.relerr(beta * (Vs[:m].T @ matfun.fmat_e1(f, Hh)), res["f"])
        assert est / 20.0 <= e2e <= est


def test_sketched_gs_basis_algorithm1_pinned():
    """Algorithm 1: the sketch of the basis is orthonormal, the Arnoldi-like
    relation (eq. (3)) holds, r_11 = ||Theta b||, and with the exact
    least-squares solution Algorithm 3 returns f_m (Lemma 2) - checked
    against the full Arnoldi approximation and a dense brute force."""
    st = W.convdiff3d(10, 50.0)
    A = operators.as_matrix(st)
    b = W.rhs(st.n, 7)
    sk = sketch.Sketch("srht", st.n, 120, 3, 8)
    m = 30
    V, H, r11, S, mu, brk = krylov.sketched_gs_basis(A, b, m, sk)
    assert mu == m and not brk
    # one classical Gram-Schmidt step per column (as printed): orthonormal to O(kappa u)
    assert np.abs(S.T @ S - np.eye(m + 1)).max() < 1e-7
    assert np.allclose(sk.apply(V.T), S, atol=1e-11)
    assert r11 == pytest.approx(np.linalg.norm(sk.apply(b)), rel=1e-14)
    rel = np.linalg.norm(A @ V[:m].T - V.T @ H) / np.linalg.norm(A @ V[:m].T)
    assert rel < 1e-12
    f = W.FuncSpec("exp", alpha=-2e-3)
    out = krylov.sgs(A, b, f, m, sk)
    fm = krylov.fm(A, b, f, m)
    assert krylov.relerr(out["f"], fm) < 1e-10
    # a planted slip (coefficients not scaled by r_ii) breaks the relation
    Hbad = H.copy()
    Hbad[m, m - 1] *= 1.01
    assert np.linalg.norm(A @ V[:m].T - V.T @ Hbad) / np.linalg.norm(A @ V[:m].T) > 1e-6


def test_sketched_gs_two_passes_pinned():
    """The repeated Gram-Schmidt step on the sketch (not in the paper) keeps
    Theta V orthonormal to rounding where one pass loses it (s = 63 rows for
    m = 60 on a 3D Laplacian), spans the same Krylov subspace (Arnoldi-like
    relation, same f_m with the exact least squares) and agrees with one pass
    where that pass is accurate."""
    st = W.laplacian3d(16)
    A = operators.as_matrix(st)
    b = W.rhs(st.n, 4)
    m, s = 60, 63
    sk = sketch.Sketch("srht", st.n, s, 5, 8)
    _, _, _, S1, _, _ = krylov.sketched_gs_basis(A, b, m, sk, passes=1)
    V, H, r11, S, mu, brk = krylov.sketched_gs_basis(A, b, m, sk, passes=2)
    assert mu == m and not brk
    assert np.abs(S1.T @ S1 - np.eye(m + 1)).max() > 1e-3        # one pass: lost
    assert np.abs(S.T @ S - np.eye(m + 1)).max() < 1e-13         # two passes: kept
    assert np.abs(sk.apply(V.T) - S).max() < 1e-6
    rel = np.linalg.norm(A @ V[:m].T - V.T @ H) / np.linalg.norm(A @ V[:m].T)
    assert rel < 1e-12
    f = W.FuncSpec("pow", sigma=0.0, p=-0.5)
    assert krylov.relerr(krylov.sgs(A, b, f, m, sk, passes=2)["f"], krylov.fm(A, b, f, m)) < 1e-11
    # a well-conditioned sketch: both passes give the same Hessenberg matrix
    st2 = W.convdiff3d(10, 50.0)
    A2 = operators.as_matrix(st2)
    b2 = W.rhs(st2.n, 7)
    sk2 = sketch.Sketch("srht", st2.n, 120, 3, 8)
    H1 = krylov.sketched_gs_basis(A2, b2, 20, sk2, passes=1)[1]
    H2 = krylov.sketched_gs_basis(A2, b2, 20, sk2, passes=2)[1]
    assert np.abs(H1 - H2).max() < 1e-9 * np.abs(H1).max()


def test_whitening_pinned():
    """Whitening (Section 2.1.2): on a graph Laplacian where the truncated
    basis alone loses its conditioning (the exact least-squares result of
    Algorithm 4 is then 10% off f_m), the whitened basis continued by
    Algorithm 1 stays well conditioned, satisfies the Arnoldi-like relation
    (eq. (3)) and gives f_m.  Without a trigger it is Algorithm 2; whitening
    forced at the last step gives Algorithm 1 (the equivalence of Remark 1)."""
    n, m, k = 4096, 120, 2
    op = W.rgg_laplacian(n, seed=3)
    A = operators.as_matrix(op)
    b = W.rhs(n, 3)
    f = W.FuncSpec("pow", sigma=1e-3, p=-0.5)
    sk = sketch.Sketch("sparse_sign", n, 2 * m, 3, 8)
    fm = krylov.fm(A, b, f, m)
    res = krylov.whitened(A, b, f, m, k, sk)
    assert res["whitened_at"] == 90 and res["m_used"] == m
    V, H = res["V"], res["Hbar"]
    sv = np.linalg.svd(V.T, compute_uv=False)
    assert sv[0] / sv[-1] < 100
    assert np.linalg.norm(A @ V[:m].T - V.T @ H) / np.linalg.norm(A @ V[:m].T) < 1e-12
    assert krylov.relerr(res["f"], fm) < 1e-10
    assert krylov.relerr(krylov.nt(A, b, f, m, k, sk, "exact")["f"], fm) > 1e-2
    # the sketch condition is kappa_1 of the triangular factor (a library routine)
    SV = sk.apply(krylov.truncated_arnoldi(A, b, 40, k)[0].T)
    Rq = np.linalg.qr(SV, mode="r")
    assert krylov.sketch_condition(SV) == pytest.approx(np.linalg.cond(Rq, 1), rel=1e-10)
    # no trigger: Algorithm 2
    st = W.convdiff3d(10, 50.0)
    A2 = operators.as_matrix(st)
    b2 = W.rhs(st.n, 7)
    sk2 = sketch.Sketch("srht", st.n, 120, 3, 8)
    Vn, Hn, beta, *_ = krylov.truncated_arnoldi(A2, b2, 30, 2)
    Vw, Hw, scale, _, _, _, at = krylov.whitened_basis(A2, b2, 30, 2, sk2, thresh=np.inf)
    assert at == 0 and scale == beta
    assert np.abs(Hw - Hn).max() == 0.0 and np.abs(Vw - Vn).max() == 0.0
    # whitening forced before the last step: Algorithm 1 (Remark 1)
    Vg, Hg, r11, Sg, *_ = krylov.sketched_gs_basis(A2, b2, 30, sk2)
    Vw, Hw, scale, Sw, _, _, at = krylov.whitened_basis(A2, b2, 30, 2, sk2, thresh=0.0, every=30)
    assert at == 30
    assert scale == pytest.approx(r11, rel=1e-12)
    assert np.abs(Hw - Hg).max() < 1e-9 * np.abs(Hg).max()
    assert np.abs(Vw - Vg).max() < 1e-9
    # a planted slip (H not transformed by R) breaks the relation
    Vb, Hb, *_ = krylov.whitened_basis(A, b, m, k, sk)
    Hbad = Hb.copy()
    Hbad[:5, :4] *= 1.001
    assert np.linalg.norm(A @ Vb[:m].T - Vb.T @ Hbad) / np.linalg.norm(A @ Vb[:m].T) > 1e-6


def test_sign_function_pinned():
    """sign(A) b = (A^2)^{-1/2} (A b) (Section 5.1.3).

    * A non-normal, non-integer operator A = X diag(d) X^{-1} with six
      distinct eigenvalues whose squares are distinct and not representable
      in FP32: the Krylov space of A^2 for A b is invariant after 6 steps, so
      the method at m = 8 with a window k = 8 (full orthogonalisation)
      finds h_{7,6} at rounding level and returns sign(A) b exactly; the
      reference is the dense eigendecomposition X sign(Lambda) X^{-1} b.
      Rounding A^2 to FP32 (a planted slip) moves the result by ~1e-8 and
      fails the 1e-12 bound.
    * Applying the computed sign function twice returns b (sign^2 = I).
    * On a shifted (indefinite) 2D Laplacian with a non-integer centre, A^2
      is the exact FP64 product, and the full-Arnoldi form of the formula
      approaches the DST closed form S sign(lambda) S b as m grows."""
    import scipy.fft as sfft

    SIGN = W.FuncSpec("sign")
    n = 60
    r = np.random.default_rng(41)
    X = np.eye(n) + 0.3 * r.standard_normal((n, n)) / math.sqrt(n)
    d = np.repeat([-2.3, -1.7, -0.45, 0.6, 1.35, 2.85], n // 6)
    Ad = X @ np.diag(d) @ np.linalg.inv(X)
    A = sp.csr_matrix(Ad)
    b = r.standard_normal(n)
    ref = closed_form.dense_fAb(Ad, SIGN, b)
    res = krylov.sign_fAb(A, b, 8, 8, ls="none")   # window k = m: full orthogonalisation
    H = res["Hbar"]
    assert abs(H[6, 5]) < 1e-10 * np.abs(H).max()   # invariant after 6 steps (to rounding)
    assert krylov.relerr(res["f"], ref) < 1e-12
    twice = krylov.sign_fAb(A, res["f"], 8, 8, ls="none")["f"]
    assert krylov.relerr(twice, b) < 1e-11
    # planted slip: A^2 with FP32-rounded values
    A2r = sp.csr_matrix(A @ A)
    A2r.data = A2r.data.astype(np.float32).astype(np.float64)
    f = W.FuncSpec("pow", sigma=0.0, p=-0.5)
    wrong = krylov.nt(A2r, A @ b, f, 8, 8, None, "none")["f"]
    assert krylov.relerr(wrong, ref) > 1e-9
    # planted slip: z^{-1/2} applied to a shifted A^2
    wrong = krylov.nt(A @ A + 0.5 * sp.identity(n), A @ b, f, 8, 8, None, "none")["f"]
    assert krylov.relerr(wrong, ref) > 1e-3
    # shifted Laplacian, non-integer centre 2.7: the exact FP64 square
    N, shift = 8, 1.3
    st = W.Stencil(2, N, N, 1, (4.0 - shift, -1.0, -1.0, -1.0, -1.0, 0.0, 0.0))
    L = operators.as_matrix(st)
    assert np.abs((krylov.square_operator(L) - L @ L).toarray()).max() == 0.0
    bl = W.rhs(st.n, 4)
    lam = closed_form.laplacian_eigs(W.laplacian2d(N)) - shift
    ref = sfft.dstn(sfft.dstn(bl.reshape(N, N), type=1, norm="ortho") * np.sign(lam), type=1, norm="ortho").ravel()
    np.testing.assert_allclose(closed_form.dense_fAb(L.toarray(), SIGN, bl, symmetric=True), ref, atol=1e-12)
    e30 = krylov.relerr(krylov.fm(krylov.square_operator(L), L @ bl, f, 30), ref)
    e45 = krylov.relerr(krylov.fm(krylov.square_operator(L), L @ bl, f, 45), ref)
    assert e45 < 1e-5 and e45 < 1e-2 * e30