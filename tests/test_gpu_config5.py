"""Parity at the full size of the largest single-GPU workload, in the launch
configuration the benchmark times: 3D upwind convection-diffusion on a 256^3
grid (n = 16,777,216), Pe = 100, scaled to ||A||_inf = 1e3, exp(-1e-3 A) B for
a block of 8 right-hand sides interleaved row by row (2^27 elements per basis
vector: 65,536 tiles of 2048 elements on 512 blocks), m = 200, k = 4, SRHT
sketch with s = 800 rows (6400 sketch accumulators per block).

Oracles:
* every output against the converged exp(-tA) B of the Kronecker-sum closed
  form, which equals f_m at this m (pinned on the CPU: at ||tA||_inf = 1 full
  Arnoldi agrees with it to 1e-13);
* the first column of Theta V (the sketch of b_q / ||b_q||, Section 2.1.1)
  against the oracle's SRHT for two right-hand sides, which checks the tile
  transform, the cross-tile signs and the row sampling at the padded length
  2^24.
Tolerances: 1e-6 for the FP32-basis result, 1e-10 for the FP64 basis.
"""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form, krylov, sketch as osk

pytestmark = pytest.mark.gpu

NAME = "convdiff3d_256_exp_8rhs"


@pytest.fixture(scope="module")
def setup():
    import torch

    from paper_2212_12758_amd import Context

    assert torch.cuda.is_available()
    w = W.config(NAME)
    n, nrhs = w.n, w.nrhs
    B = W.rhs(n, w.b_seed, nrhs)
    # workspace for an FP64 basis of the block (216 GB) plus 2 GiB
    ldv = (n * nrhs + 63) // 64 * 64
    ctx = Context(0, arena_bytes=(w.m + 1) * ldv * 8 + 2 * n * nrhs * 8 + (2 << 30))
    A = ctx.matrix(w.op)
    Bd = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    print("config5: closed form", flush=True)
    ref = closed_form.kronecker_exp_fAb(w.op, w.f.alpha, B)
    yield w, ctx, A, B, Bd, ref
    A.destroy()
    ctx.close()
    del Bd
    torch.cuda.empty_cache()


def _params(w, prec, ls, tol):
    from paper_2212_12758_amd import make_params

    return make_params(w.m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, prec, ls, tol)


def _first_sketch_column(w, B, dg, atol):
    sk = osk.Sketch(w.sketch, w.n, w.s, w.sketch_seed, w.zeta)
    for q in (0, w.nrhs - 1):
        bq = np.ascontiguousarray(B[:, q])
        ref = sk.apply(bq / np.linalg.norm(bq))
        np.testing.assert_allclose(dg["sv"][q][:, 0], ref, rtol=0, atol=atol, err_msg=f"rhs {q}")


def test_config5_fp32_basis_auto_policies(setup):
    w, ctx, A, B, Bd, ref = setup
    print("config5: fp32 basis, auto policies", flush=True)
    out, info, dg = ctx.solve(A, Bd, w.f, _params(w, "auto", "auto", 1e-6), diag=True)
    out = out.cpu().numpy()
    for q in range(w.nrhs):
        assert info[q]["m_used"] == w.m
        err = krylov.relerr(out[:, q], ref[:, q])
        print(f"  rhs {q}: relerr {err:.3e} err_est {info[q]['err_est']:.2e} prec_used {info[q]['prec_used']}",
              flush=True)
        assert err < 1e-6, q
    # the FP32 basis stores fl(b); its sketch differs from Theta b / ||b|| by ~1e-8
    _first_sketch_column(w, B, dg, 1e-6)


def test_config5_fp64_basis(setup):
    w, ctx, A, B, Bd, ref = setup
    print("config5: fp64 basis", flush=True)
    out, info, dg = ctx.solve(A, Bd, w.f, _params(w, "fp64", "auto", 1e-10), diag=True)
    out = out.cpu().numpy()
    for q in range(w.nrhs):
        err = krylov.relerr(out[:, q], ref[:, q])
        print(f"  rhs {q}: relerr {err:.3e}", flush=True)
        assert err < 1e-10, q
    _first_sketch_column(w, B, dg, 1e-12)
