"""Krylov approximations of f(A)b (oracle side, test infrastructure).

Plain, slow FP64 implementations of the paper's definitions and algorithms:

* ``arnoldi``            Arnoldi decomposition A U_m = U_{m+1} K_m, eq. (2).
* ``fm``                 f_m = ||b|| U_m f(K_m) e_1, eq. (4) -- the parity target.
* ``truncated_arnoldi``  Algorithm 2 (k-truncated orthogonalisation), giving the
                         Arnoldi-like decomposition A V_m = V_{m+1} H_m, eq. (3).
* ``nt``                 Algorithm 4 (least-squares correction of the last
                         column, eqs. (6)-(7)) and Algorithm 5 (no correction,
                         eq. (8)); the least-squares problem is solved exactly,
                         by sketch-and-solve (Remark 3) or skipped.
* ``sfom``               the sFOM approximation, eq. (9).
* ``sketched_gs_basis``  Algorithm 1; ``sgs`` Algorithm 3 (exact least squares).
* ``whitened_basis``     Algorithm 2 with whitening, continued by Algorithm 1
                         (Section 2.1.2); ``whitened`` its f(A)b.
* ``sign_fAb``           sign(A)b = (A^2)^{-1/2}(A b) (Section 5.1.3).

Readings of the printed Algorithm 2 (typographical slips in the inner loop):
the update subtracts h_{j,i-1} v_j (the coefficient just computed times the
window vector j), and the new column's subdiagonal entry is ||w_i||.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from . import matfun

EPS = np.finfo(np.float64).eps


def _breakdown_tol() -> float:
    return 100.0 * EPS


def arnoldi(A, b: np.ndarray, m: int):
    """Arnoldi decomposition, eq. (2).

    Gram-Schmidt with one full re-orthogonalisation pass, so that the returned
    U is orthonormal to working precision and K = U^T A U (the compression of
    A onto K_m(A, b)).  Stops early on an invariant subspace (h_{j+1,j} below
    100 eps ||A u_j||) and then returns the exact dimension j.

    Returns (U rows u_1..u_{mu+1} as a (mu+1) x n array (mu x n on breakdown),
    Kbar (mu+1) x mu, beta = ||b||, mu).
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    U = np.zeros((m + 1, n))
    K = np.zeros((m + 1, m))
    beta = float(np.linalg.norm(b))
    U[0] = b / beta
    for j in range(m):
        w = A @ U[j]
        wn = np.linalg.norm(w)
        Q = U[: j + 1]
        h = Q @ w
        w = w - Q.T @ h
        h2 = Q @ w
        w = w - Q.T @ h2
        K[: j + 1, j] = h + h2
        K[j + 1, j] = np.linalg.norm(w)
        if K[j + 1, j] <= _breakdown_tol() * wn:
            return U[: j + 1], K[: j + 2, : j + 1], beta, j + 1
        U[j + 1] = w / K[j + 1, j]
    return U, K, beta, m


def fm(A, b: np.ndarray, f, m: int) -> np.ndarray:
    """f_m = ||b||_2 U_m f(K_m) e_1, eq. (4).  Multi-column b is handled column by column."""
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 2:
        return np.stack([fm(A, b[:, r], f, m) for r in range(b.shape[1])], axis=1)
    if not np.any(b):
        return np.zeros_like(b)
    U, K, beta, mu = arnoldi(A, b, m)
    c = matfun.fmat_e1(f, K[:mu, :mu])
    return beta * (U[:mu].T @ c)


def truncated_arnoldi(A, b: np.ndarray, m: int, k: int):
    """Algorithm 2: each new w_i = A v_{i-1} is orthogonalised (modified
    Gram-Schmidt) against the last k basis vectors only, then normalised.

    Returns (V rows v_1..v_{mu+1}, Hbar (mu+1) x mu, beta, mu, breakdown) with
    A V_mu = V_{mu+1} Hbar (eq. (3)).  On an invariant subspace (new norm below
    100 eps ||w_i||) it stops at dimension mu with breakdown=True; then V has
    mu rows and Hbar's last row is zero.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    beta = float(np.linalg.norm(b))
    V[0] = b / beta
    for i in range(1, m + 1):
        w = A @ V[i - 1]
        wn = np.linalg.norm(w)
        for j in range(max(0, i - k), i):
            H[j, i - 1] = V[j] @ w
            w = w - H[j, i - 1] * V[j]
        H[i, i - 1] = np.linalg.norm(w)
        if H[i, i - 1] <= _breakdown_tol() * wn:
            H[i, i - 1] = 0.0
            return V[:i], H[: i + 1, :i], beta, i, True
        V[i] = w / H[i, i - 1]
    return V, H, beta, m, False


def sketched_qr(SV: np.ndarray):
    """Householder QR of the sketched basis (LAPACK via numpy)."""
    Q, R = np.linalg.qr(SV, mode="reduced")
    return Q, R


def nt(A, b: np.ndarray, f, m: int, k: int, sketch=None, ls: str = "sketch"):
    """Algorithms 4 and 5 with every intermediate returned.

    ls = "exact"  : y = argmin ||V_m z - v_{m+1}||_2 (eq. (7)), dense lstsq;
    ls = "sketch" : y = argmin ||Theta (V_m z - v_{m+1})||_2 (sketch-and-solve,
                    Remark 3), via QR of Theta V_m;
    ls = "none"   : y = 0, i.e. Algorithm 5 / eq. (8).
    The compression is H_hat = H_m + h_{m+1,m} y e_m^T (eq. (6)) and the result
    ||b|| V_m f(H_hat) e_1 (Algorithm 4, last line).
    """
    b = np.asarray(b, dtype=np.float64)
    V, Hbar, beta, mu, brk = truncated_arnoldi(A, b, m, k)
    out = {"V": V, "Hbar": Hbar, "beta": beta, "m_used": mu, "breakdown": brk}
    if sketch is not None:
        out["SV"] = sketch.apply(V.T)
    Hm = Hbar[:mu, :mu].copy()
    y = np.zeros(mu)
    if not brk and ls != "none":
        if ls == "exact":
            y = np.linalg.lstsq(V[:mu].T, V[mu], rcond=None)[0]
        elif ls == "sketch":
            SV = out["SV"]
            Q, R = sketched_qr(SV[:, :mu])
            y = sl.solve_triangular(R, Q.T @ SV[:, mu])
            out["R"] = R
        else:
            raise ValueError(ls)
    Hhat = Hm.copy()
    if not brk:
        Hhat[:, mu - 1] += Hbar[mu, mu - 1] * y
    c = matfun.fmat_e1(f, Hhat)
    out.update(y=y, Hhat=Hhat, c=c, f=beta * (V[:mu].T @ c))
    return out


def sketched_gs_basis(A, b: np.ndarray, m: int, sketch, passes: int = 1):
    """Algorithm 1: the basis whose sketch Theta V is kept orthonormal.

    Each new vector w = A v_{i-1} is sketched (p = Theta w), one classical
    Gram-Schmidt step on the sketch gives r = S^T p, s = p - S r and
    r_ii = ||s||, and the same coefficients act on the vectors:
    v_i = (w - V r) / r_ii.  Returns V (rows v_0..v_mu), Hbar (the columns
    2..m+1 of R), r_11 = ||Theta b||, S = Theta V (columns), m_used and the
    breakdown flag (r_ii <= 100 eps ||p||: the subspace is invariant).

    passes = 2 is not in the paper: the Gram-Schmidt step on the sketch is
    repeated once on its own residual (r = r' + r'', s = p - S r' - S r''),
    which leaves exact arithmetic unchanged (S is orthonormal, so r'' = 0)
    but keeps S orthonormal to rounding where one pass loses it (sketches
    with s close to m).  parity unpinned by the paper; pinned by invariants.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    p = sketch.apply(b)
    r11 = float(np.linalg.norm(p))
    V = np.zeros((m + 1, n))
    S = np.zeros((p.size, m + 1))
    H = np.zeros((m + 1, m))
    if r11 == 0.0:
        return V[:1], H[:1, :0], 0.0, S[:, :1], 0, True
    V[0] = b / r11
    S[:, 0] = p / r11
    for i in range(1, m + 1):
        w = A @ V[i - 1]
        p = sketch.apply(w)
        r = S[:, :i].T @ p
        sv = p - S[:, :i] @ r
        for _ in range(passes - 1):
            r2 = S[:, :i].T @ sv
            sv = sv - S[:, :i] @ r2
            r = r + r2
        rii = float(np.linalg.norm(sv))
        H[:i, i - 1] = r
        if rii <= _breakdown_tol() * np.linalg.norm(p):
            return V[:i], H[: i + 1, :i], r11, S[:, :i], i, True
        H[i, i - 1] = rii
        S[:, i] = sv / rii
        V[i] = (w - V[:i].T @ r) / rii
    return V, H, r11, S, m, False


def sketch_condition(SV: np.ndarray) -> float:
    """kappa_1(R) = ||R||_1 ||R^{-1}||_1 of the triangular factor of the
    sketched basis SV (Theta V_i): the quantity the condition estimate of the
    whitening test (Section 5.1.3, threshold 1000) estimates; R has the same
    2-norm condition number as SV."""
    R = np.linalg.qr(SV, mode="r")
    Rinv = sl.solve_triangular(R, np.eye(R.shape[0]))
    return float(np.linalg.norm(R, 1) * np.linalg.norm(Rinv, 1))


def whitened_basis(A, b: np.ndarray, m: int, k: int, sketch, thresh: float = 1000.0, every: int = 5):
    """Algorithm 2 with whitening (Section 2.1.2), continued by Algorithm 1.

    Before step i (i a multiple of ``every``, i >= 2) the sketch of the basis
    built so far, Theta V_i (columns v_0..v_{i-1}), is tested: if
    kappa_1(R) > thresh, with Theta V_i = Q R (R with positive diagonal),
    the basis is whitened, V_i <- V_i R^{-1}, Hbar_{i-1} <- R_i Hbar_{i-1}
    R_{i-1}^{-1}, its sketch becomes Q, and every later step is a step of
    Algorithm 1 on that sketch.  b = beta v_0 becomes beta R_00 v~_0, so the
    scale of the result is beta R_00.  Without a trigger this is Algorithm 2.

    Returns (V, Hbar, scale, S = Theta V, m_used, breakdown, whitened_at),
    whitened_at = 0 when the basis was never whitened.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    beta = float(np.linalg.norm(b))
    p0 = sketch.apply(b)
    S = np.zeros((p0.size, m + 1))
    if beta == 0.0:
        return V[:1], H[:1, :0], 0.0, S[:, :1], 0, True, 0
    V[0] = b / beta
    S[:, 0] = p0 / beta
    white = 0
    for i in range(1, m + 1):
        if not white and i % every == 0 and i >= 2 and sketch_condition(S[:, :i]) > thresh:
            Q, R = np.linalg.qr(S[:, :i], mode="reduced")
            sg = np.sign(np.diag(R))
            sg[sg == 0] = 1.0
            Q, R = Q * sg, R * sg[:, None]
            V[:i] = sl.solve_triangular(R.T, V[:i], lower=True)        # rows of V_i R^{-1}
            H[:i, : i - 1] = R @ H[:i, : i - 1] @ np.linalg.inv(R[: i - 1, : i - 1])
            S[:, :i] = Q
            beta = beta * R[0, 0]
            white = i
        w = A @ V[i - 1]
        if not white:
            wn = np.linalg.norm(w)
            for j in range(max(0, i - k), i):
                H[j, i - 1] = V[j] @ w
                w = w - H[j, i - 1] * V[j]
            H[i, i - 1] = np.linalg.norm(w)
            if H[i, i - 1] <= _breakdown_tol() * wn:
                H[i, i - 1] = 0.0
                return V[:i], H[: i + 1, :i], beta, S[:, :i], i, True, white
            V[i] = w / H[i, i - 1]
            S[:, i] = sketch.apply(V[i])
        else:
            p = sketch.apply(w)
            r = S[:, :i].T @ p
            sv = p - S[:, :i] @ r
            rii = float(np.linalg.norm(sv))
            H[:i, i - 1] = r
            if rii <= _breakdown_tol() * np.linalg.norm(p):
                return V[:i], H[: i + 1, :i], beta, S[:, :i], i, True, white
            H[i, i - 1] = rii
            S[:, i] = sv / rii
            V[i] = (w - V[:i].T @ r) / rii
    return V, H, beta, S, m, False, white


def whitened(A, b: np.ndarray, f, m: int, k: int, sketch, thresh: float = 1000.0, every: int = 5) -> dict:
    """f(A)b from the whitened basis with the exact least-squares solution of
    eq. (7) (the limit of the LSQR iteration the basis is paired with):
    scale V_m f(H_m + h_{m+1,m} y e_m^T) e_1."""
    V, Hbar, scale, S, mu, brk, white = whitened_basis(A, b, m, k, sketch, thresh, every)
    y = np.zeros(mu)
    if not brk and mu > 0:
        y = np.linalg.lstsq(V[:mu].T, V[mu], rcond=None)[0]
    Hhat = Hbar[:mu, :mu].copy()
    if not brk and mu > 0:
        Hhat[:, mu - 1] += Hbar[mu, mu - 1] * y
    c = matfun.fmat_e1(f, Hhat) if mu > 0 else np.zeros(0)
    return {"V": V, "Hbar": Hbar, "scale": scale, "S": S, "m_used": mu, "breakdown": brk, "whitened_at": white,
            "y": y, "Hhat": Hhat, "c": c,
            "f": scale * (V[:mu].T @ c) if mu > 0 else np.zeros_like(np.asarray(b, float))}


def sgs(A, b: np.ndarray, f, m: int, sketch, passes: int = 1) -> dict:
    """Algorithm 3 with the least-squares problem of its second step solved
    exactly (the limit of its LSQR iteration): y = argmin ||V_m z - v_{m+1}||,
    result r_11 V_m f(H_m + h_{m+1,m} y e_m^T) e_1.  ``passes`` as in
    sketched_gs_basis."""
    V, Hbar, r11, S, mu, brk = sketched_gs_basis(A, b, m, sketch, passes)
    y = np.zeros(mu)
    if not brk and mu > 0:
        y = np.linalg.lstsq(V[:mu].T, V[mu], rcond=None)[0]
    Hhat = Hbar[:mu, :mu].copy()
    if not brk and mu > 0:
        Hhat[:, mu - 1] += Hbar[mu, mu - 1] * y
    c = matfun.fmat_e1(f, Hhat) if mu > 0 else np.zeros(0)
    return {"V": V, "Hbar": Hbar, "r11": r11, "S": S, "m_used": mu, "breakdown": brk, "y": y, "Hhat": Hhat,
            "c": c, "f": r11 * (V[:mu].T @ c) if mu > 0 else np.zeros_like(np.asarray(b, float))}


def estimates(res: dict, f, unit_round: float) -> dict:
    """A-posteriori quantities of the dense tail for a result of ``nt``.

    Norms are taken as ||R x||, which approximates ||V_m x|| through the
    sketch (Section 2.1.1); R is the factor of Theta V_m (identity without a
    least-squares solve):

    * ls_gate  = ||R (c - c_0)|| / ||R c||, c_0 = f(H_m) e_1: how far the
      least-squares column of eq. (6) moves the result (eq. (8) vs Algorithm 4);
    * conv_est = ||R (c - [c_d; 0])|| / ||R c||, c_d from the compression at
      order m_d = m - max(5, m // 10), whose sketched least-squares solution
      R_d^{-1} R[:m_d, m_d] comes from the same factor;
    * round_est = u sum_j |c_j| ||R e_j|| / ||R c|| (u: basis unit roundoff),
      the first-order effect of rounding every stored basis vector on V_m c.
    After a breakdown the result is exact and both quantities are 0.
    """
    mu = res["m_used"]
    H = res["Hbar"]
    c = res["c"]
    have_r = "R" in res
    R = res["R"][:mu, :mu] if have_r else np.eye(mu)
    c0 = matfun.fmat_e1(f, H[:mu, :mu])
    md = mu - max(5, mu // 10)
    cd = np.zeros(mu)
    if md >= 1:
        yd = sl.solve_triangular(R[:md, :md], R[:md, md]) if have_r else np.zeros(md)
        Hd = H[:md, :md].copy()
        if not res["breakdown"]:
            Hd[:, md - 1] += H[md, md - 1] * yd
        cd[:md] = matfun.fmat_e1(f, Hd)
    nc = np.linalg.norm(R @ c)
    gate = np.linalg.norm(R @ (c - c0)) / nc
    conv = np.linalg.norm(R @ (c - cd)) / nc if md >= 1 else np.inf
    rnd = unit_round * float(np.abs(c) @ np.linalg.norm(R, axis=0)) / nc
    if res["breakdown"]:
        gate = conv = 0.0
    return {"ls_gate": float(gate), "conv_est": float(conv), "round_est": float(rnd)}


def sfom(A, b: np.ndarray, f, m: int, k: int, sketch) -> np.ndarray:
    """sFOM, eq. (9): V_m R^{-1} f(S^T Theta A V_m R^{-1}) S^T Theta b,
    with Theta V_m = S R and the basis from Algorithm 2."""
    V, Hbar, beta, mu, brk = truncated_arnoldi(A, b, m, k)
    Vm = V[:mu].T
    S, R = sketched_qr(sketch.apply(Vm))
    SAV = sketch.apply(np.column_stack([A @ Vm[:, j] for j in range(mu)]))
    M = S.T @ SAV @ np.linalg.inv(R)
    z = matfun.fmat(f, M) @ (S.T @ sketch.apply(np.asarray(b, dtype=np.float64)))
    return Vm @ sl.solve_triangular(R, z)


def square_operator(A):
    """A^2 as an exact FP64 sparse product (the operator whose inverse square
    root gives the sign function, Section 5.1.3).  Only FP64 rounding of the
    product itself: no value is rounded to a lower precision."""
    import scipy.sparse as sps

    return sps.csr_matrix(A @ A)


def sign_fAb(A, b: np.ndarray, m: int, k: int, sketch=None, ls: str = "sketch") -> dict:
    """sign(A) b = (A^2)^{-1/2} (A b) (Section 5.1.3, after Higham's
    Chapter 5): the method of ``nt`` applied to the operator A^2
    (``square_operator``), the start vector A b and f(z) = z^{-1/2}."""
    from types import SimpleNamespace

    f = SimpleNamespace(kind="pow", sigma=0.0, p=-0.5, alpha=0.0, coef=())
    return nt(square_operator(A), A @ np.asarray(b, dtype=np.float64), f, m, k, sketch, ls)


def relerr(x: np.ndarray, ref: np.ndarray) -> float:
    """Relative 2-norm error, as reported in Section 5."""
    d = float(np.linalg.norm(ref))
    return float(np.linalg.norm(np.asarray(x) - ref)) / (d if d > 0 else 1.0)
