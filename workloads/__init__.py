"""Seeded synthetic inputs for the sketched-Krylov f(A)b path.

This module only *describes* inputs: stencil coefficient sets, a random
geometric graph Laplacian in CSR form, right-hand sides and the scalar
parameters of each workload.  It contains none of the method's arithmetic
(no matvec, no Krylov step, no sketch) so that both the CPU oracle and the
HIP path can take their inputs from here without sharing any computation.

Operators (paper context: Section 5 uses PDE discretisations and graph
Laplacians; the synthetic stand-ins below replace the SuiteSparse / SNAP /
Matrix Market matrices of Sections 5.1.3 and 5.2, which are not available):

* ``laplacian2d(N)``   5-point Dirichlet Laplacian, diag 4, off-diag -1.
* ``laplacian3d(N)``   7-point Dirichlet Laplacian (T_N (x) I (x) I + ...,
                        T_N = tridiag(-1, 2, -1); Section 5.1.4 prints the
                        last off-diagonal sign as +1, read as -1).
* ``convdiff3d(N, Pe)`` upwind 7-point discretisation of -Lap(u) + Pe(1,1,1).grad(u)
                        on the unit cube, h = 1/(N+1), rescaled so that
                        ||A||_inf = ||A||_1 = 1e3 (hence ||A||_2 <= 1e3).
* ``rgg_laplacian(n)``  graph Laplacian D - W of a random geometric graph in
                        the unit square with mean degree ~10, CSR int32/FP32.
* ``convdiff2d_varcoef(N)`` the variable-coefficient convection-diffusion
                        operator of Section 5.1.1 (D_1 = 1000 on [0.25, 0.75]^2,
                        else 1; D_2 = D_1 / 2; v = (x + y, x - y); Pe = 200) on an
                        N x N interior grid, CSR int32/FP32 (construction below).

Grid ordering everywhere: row = x + nx*(y + ny*z), x fastest.
Stencil coefficient order: (centre, x-1, x+1, y-1, y+1, z-1, z+1); a
coefficient multiplies the value at that neighbour; neighbours outside the
grid are zero (homogeneous Dirichlet).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Stencil", "laplacian2d", "laplacian3d", "convdiff3d", "rgg_laplacian", "convdiff2d_varcoef", "sine_rhs",
    "rhs", "FuncSpec", "Workload", "config", "CONFIG_NAMES",
]


@dataclasses.dataclass(frozen=True)
class Stencil:
    """A constant-coefficient 5/7-point stencil on an nx*ny*nz grid."""
    dim: int
    nx: int
    ny: int
    nz: int
    coeff: tuple  # (c, xm, xp, ym, yp, zm, zp)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def laplacian2d(N: int, ny: int | None = None) -> Stencil:
    ny = N if ny is None else ny
    return Stencil(2, N, ny, 1, (4.0, -1.0, -1.0, -1.0, -1.0, 0.0, 0.0))


def laplacian3d(N: int) -> Stencil:
    return Stencil(3, N, N, N, (6.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0))


def convdiff3d(N: int, Pe: float, norm_target: float = 1e3) -> Stencil:
    """Upwind (backward-difference) convection-diffusion, scaled to ||A||_inf = norm_target."""
    h = 1.0 / (N + 1)
    c = 6.0 / h**2 + 3.0 * Pe / h
    up = -1.0 / h**2 - Pe / h        # upstream neighbours x-1, y-1, z-1
    dn = -1.0 / h**2                 # downstream neighbours x+1, y+1, z+1
    row_abs_sum = abs(c) + 3.0 * abs(up) + 3.0 * abs(dn)   # = 12/h^2 + 6 Pe/h
    s = norm_target / row_abs_sum
    return Stencil(3, N, N, N, (c * s, up * s, dn * s, up * s, dn * s, up * s, dn * s))


def rgg_laplacian(n: int, seed: int, mean_degree: float = 10.0):
    """Random geometric graph Laplacian L = D - W in CSR (int32 rowptr/col, float32 val).

    Points are uniform in [0,1]^2 (seeded); radius r = sqrt(mean_degree/(pi (n-1)))
    (boundary deficit ignored); nodes are renumbered by r-cell (row-major cells)
    so that graph neighbours are close in memory.  Values are small integers,
    hence exact in FP32.  Returns (rowptr, col, val) with sorted columns and the
    diagonal included in every row.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = math.sqrt(mean_degree / (math.pi * (n - 1)))
    ncell = max(1, int(1.0 / r))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((pts[:, 0], cx, cy))          # row-major cells, then x
    pts = pts[order]
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i = np.concatenate([pairs[:, 0], pairs[:, 1]])
    j = np.concatenate([pairs[:, 1], pairs[:, 0]])
    deg = np.bincount(i, minlength=n).astype(np.float64)
    rows = np.concatenate([i, np.arange(n)])
    cols = np.concatenate([j, np.arange(n)])
    vals = np.concatenate([-np.ones(i.size), deg])
    perm = np.lexsort((cols, rows))
    rows, cols, vals = rows[perm], cols[perm], vals[perm]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float32)


def convdiff2d_varcoef(N: int, Pe: float = 200.0):
    """CSR (int32 rowptr/col, FP32 val) of
    L[u] = -(D_1 u_x)_x - (D_2 u_y)_y + Pe (1/2 (v . grad u) + 1/2 div(v u))
    on (0, 1)^2, homogeneous Dirichlet, N x N interior points, h = 1/(N+1),
    row = i + N j for the point (x_i, y_j) = ((i+1) h, (j+1) h).
    Diffusion: conservative three-point differences with D at the half
    points; convection: centred differences of the split (skew-symmetric)
    form, so the u_{i+1} entry of row i is Pe (v_1(x_i) + v_1(x_{i+1})) / (4h)
    and the u_{i-1} entry is -Pe (v_1(x_i) + v_1(x_{i-1})) / (4h) (same in y
    with v_2).  The discretisation is not given in the paper (it cites
    Botchev & Knizhnerman 2020); this is a standard choice for that form."""
    h = 1.0 / (N + 1)

    def D1(x, y):
        return np.where((x >= 0.25) & (x <= 0.75) & (y >= 0.25) & (y <= 0.75), 1000.0, 1.0)

    idx = np.arange(N)
    I, J = np.meshgrid(idx, idx, indexing="xy")     # I: x index, J: y index, shape (N, N) with [j, i]
    x, y = (I + 1) * h, (J + 1) * h
    v1 = lambda xx, yy: xx + yy
    v2 = lambda xx, yy: xx - yy
    dxm, dxp = D1(x - h / 2, y), D1(x + h / 2, y)
    dym, dyp = 0.5 * D1(x, y - h / 2), 0.5 * D1(x, y + h / 2)
    centre = (dxm + dxp + dym + dyp) / h**2
    east = -dxp / h**2 + Pe * (v1(x, y) + v1(x + h, y)) / (4 * h)
    west = -dxm / h**2 - Pe * (v1(x, y) + v1(x - h, y)) / (4 * h)
    north = -dyp / h**2 + Pe * (v2(x, y) + v2(x, y + h)) / (4 * h)
    south = -dym / h**2 - Pe * (v2(x, y) + v2(x, y - h)) / (4 * h)
    row = (I + N * J).ravel()
    rows, cols, vals = [row], [row], [centre.ravel()]
    for val, di, dj in ((east, 1, 0), (west, -1, 0), (north, 0, 1), (south, 0, -1)):
        ok = ((I + di >= 0) & (I + di < N) & (J + dj >= 0) & (J + dj < N)).ravel()
        rows.append(row[ok])
        cols.append(((I + di) + N * (J + dj)).ravel()[ok])
        vals.append(val.ravel()[ok])
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(N * N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N * N), out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float32)


def sine_rhs(N: int) -> np.ndarray:
    """sin(pi x) sin(pi y) on the N x N interior grid, normalised (Section 5.1.1)."""
    h = 1.0 / (N + 1)
    t = np.sin(np.pi * (np.arange(N) + 1) * h)
    b = np.outer(t, t).ravel()
    return b / np.linalg.norm(b)


def rhs(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """b ~ N(0,1) from numpy's default_rng(seed); nrhs > 1 gives columns seed..seed+nrhs-1,
    returned interleaved as an (n, nrhs) C-ordered array (layout [n][nrhs])."""
    if nrhs == 1:
        return np.random.default_rng(seed).standard_normal(n)
    return np.stack([np.random.default_rng(seed + r).standard_normal(n) for r in range(nrhs)], axis=1)


@dataclasses.dataclass(frozen=True)
class FuncSpec:
    """f(z) = exp(alpha z)  |  (z + sigma)^p with p = +-1/2  |  sum_j coef[j] z^j  |  sign(z)."""
    kind: str                # "exp" | "pow" | "poly" | "sign"
    alpha: float = 0.0
    sigma: float = 0.0
    p: float = 0.0
    coef: tuple = ()


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    op: object               # Stencil or (rowptr, col, val) tuple
    b_seed: int
    nrhs: int
    f: FuncSpec
    m: int
    k: int
    s: int
    sketch: str              # "srht" | "sparse_sign"
    zeta: int = 8
    sketch_seed: int = 0

    @property
    def n(self) -> int:
        if isinstance(self.op, Stencil):
            return self.op.n
        return len(self.op[0]) - 1


CONFIG_NAMES = ("lap2d_100_exp", "convdiff3d_128_exp", "rgg_2p20_invsqrt", "convdiff3d_256_exp_8rhs",
                "lap3d_80_invsqrt", "convdiff2d_352_exp")


def config(name: str, scale: int | None = None) -> Workload:
    """The named synthetic workloads.  ``scale`` shrinks the grid/graph for
    fast parity cases while keeping the same structure and parameters."""
    if name == "lap2d_100_exp":
        N = 100 if scale is None else scale
        return Workload(name, laplacian2d(N), 0, 1, FuncSpec("exp", alpha=-0.5),
                        m=40, k=2, s=82, sketch="sparse_sign", zeta=8, sketch_seed=1)
    if name == "convdiff3d_128_exp":
        N = 128 if scale is None else scale
        return Workload(name, convdiff3d(N, 50.0), 2, 1, FuncSpec("exp", alpha=-1e-3),
                        m=100, k=4, s=400, sketch="srht", sketch_seed=2)
    if name == "rgg_2p20_invsqrt":
        n = (1 << 20) if scale is None else scale
        return Workload(name, rgg_laplacian(n, seed=3), 3, 1,
                        FuncSpec("pow", sigma=1e-3, p=-0.5),
                        m=150, k=2, s=300, sketch="sparse_sign", zeta=8, sketch_seed=3)
    if name == "convdiff3d_256_exp_8rhs":
        N = 256 if scale is None else scale
        return Workload(name, convdiff3d(N, 100.0), 50, 8, FuncSpec("exp", alpha=-1e-3),
                        m=200, k=4, s=800, sketch="srht", sketch_seed=5)
    if name == "lap3d_80_invsqrt":
        # timing workload of the sketched Gram-Schmidt basis (Section 5.1.4):
        # A^{-1/2} b for the 3D Laplacian with N = 80 (n = 512000), a sketch of
        # floor(1.05 m) rows
        N = 80 if scale is None else scale
        m = 120
        return Workload(name, laplacian3d(N), 8, 1, FuncSpec("pow", sigma=0.0, p=-0.5),
                        m=m, k=2, s=int(math.floor(1.05 * m)), sketch="srht", sketch_seed=8)
    if name == "convdiff2d_352_exp":
        # Section 5.1.1: 352 x 352 mesh, Pe = 200, exp(-t A) with the time scale
        # t = 100 / ||A||_inf (the paper does not state t); b = sin(pi x) sin(pi y)
        # normalised (b_seed -1 marks it: not a random vector)
        N = 352 if scale is None else scale
        op = convdiff2d_varcoef(N)
        rp, _, va = op
        rowsum = np.add.reduceat(np.abs(va.astype(np.float64)), rp[:-1].astype(np.int64))
        t = 100.0 / float(rowsum.max())
        return Workload(name, op, -1, 1, FuncSpec("exp", alpha=-t), m=100, k=2, s=200, sketch="srht",
                        sketch_seed=11)
    raise KeyError(name)


def laplacian_norm2(st: Stencil) -> float:
    """||A||_2 of a Dirichlet Laplacian stencil: the largest eigenvalue,
    sum over the grid directions of 2 + 2 cos(pi / (N + 1))."""
    sides = (st.nx, st.ny) if st.dim == 2 else (st.nx, st.ny, st.nz)
    return float(sum(2.0 + 2.0 * math.cos(math.pi / (N + 1)) for N in sides))


@dataclasses.dataclass(frozen=True)
class ServedRequest:
    rid: int                 # request id (b seed 10^6 + rid)
    event: int               # arrival event (a burst of shared-matrix requests shares one)
    op: Stencil
    pool: int                # index of the shared resident matrix, -1 for a fresh matrix
    f: FuncSpec
    m: int
    k: int
    s: int
    sketch_seed: int


def serving_mix(nreq: int = 4096, seed: int = 4, shared_frac: float = 0.3, pool_size: int = 4):
    """The serving mix: nreq single-rhs requests on 2D 5-point / 3D 7-point
    Dirichlet Laplacians with n log-uniform in [2^14, 2^21] (rounded to a
    square or cube grid), f uniform over {exp(-tA) with ||tA||_2 log-uniform
    in [1, 50], A^{1/2}, (A + 1e-3 I)^{-1/2}}, m uniform in [30, 200], k
    uniform in {2, 3, 4}, a sketch of s = 2m rows (its kind is the server's
    choice).

    A fraction shared_frac of the requests use one of pool_size resident
    matrices, each with its own fixed f, m, k, s and sketch seed, and arrive
    in bursts of 8..32 requests (one arrival event per burst) that a server
    can run as one block solve; every other request has a fresh matrix and
    its own sketch seed and arrives alone.  Returns (requests in arrival
    order, unit-rate exponential gaps between the arrival events)."""
    rng = np.random.default_rng(seed)

    def draw_op():
        dim = int(rng.integers(2, 4))
        n = math.exp(rng.uniform(math.log(2 ** 14), math.log(2 ** 21)))
        side = max(4, int(round(n ** (1.0 / dim))))
        return laplacian2d(side) if dim == 2 else laplacian3d(side)

    def draw_f(op):
        kind = int(rng.integers(0, 3))
        if kind == 0:
            tnorm = math.exp(rng.uniform(0.0, math.log(50.0)))
            return FuncSpec("exp", alpha=-tnorm / laplacian_norm2(op))
        if kind == 1:
            return FuncSpec("pow", sigma=0.0, p=0.5)
        return FuncSpec("pow", sigma=1e-3, p=-0.5)

    def draw_mk():
        m = int(rng.integers(30, 201))
        return m, int(rng.integers(2, 5)), 2 * m

    pool = []
    for j in range(pool_size):
        op = draw_op()
        m, k, s = draw_mk()
        pool.append((op, draw_f(op), m, k, s, 7_000_000 + j))
    n_shared = int(round(shared_frac * nreq))
    events = []   # list of ('fresh', None) or ('burst', (pool index, count))
    left = n_shared
    while left > 0:
        c = min(left, int(rng.integers(8, 33)))
        events.append(("burst", (int(rng.integers(0, pool_size)), c)))
        left -= c
    events += [("fresh", None)] * (nreq - n_shared)
    order = rng.permutation(len(events))
    gaps = rng.exponential(1.0, size=len(events))
    reqs = []
    rid = 0
    for e, idx in enumerate(order):
        kind, val = events[idx]
        if kind == "fresh":
            op = draw_op()
            m, k, s = draw_mk()
            reqs.append(ServedRequest(rid, e, op, -1, draw_f(op), m, k, s, 5_000_000 + rid))
            rid += 1
        else:
            pj, c = val
            op, f, m, k, s, sseed = pool[pj]
            for _ in range(c):
                reqs.append(ServedRequest(rid, e, op, pj, f, m, k, s, sseed))
                rid += 1
    return reqs, gaps
