"""The variable-coefficient convection-diffusion workload of Section 5.1.1
(CSR operator, exp, b = sin(pi x) sin(pi y)) on the HIP path against the
oracle, scaled to a 64 x 64 grid and at its full 352 x 352 size."""
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


@pytest.mark.parametrize("N,m", [(64, 40), (352, 100)])
def test_convdiff2d_varcoef_exp(ctx, N, m):
    from paper_2212_12758_amd import make_params

    w = W.config("convdiff2d_352_exp", scale=N)
    Aor = operators.as_matrix(w.op)
    b = W.sine_rhs(N)
    sk = osk.Sketch(w.sketch, w.n, w.s, w.sketch_seed, w.zeta)
    ref = krylov.nt(Aor, b, w.f, m, w.k, sk, "sketch")
    fm = krylov.fm(Aor, b, w.f, m)
    A = ctx.matrix(w.op)
    print(f"case convdiff2d N={N} fp64", flush=True)
    out, info, dg = ctx.solve(A, _dev(b), w.f, make_params(m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "fp64",
                                                           "sketch"), diag=True)
    out = out.cpu().numpy()
    H = ref["Hbar"]
    assert np.abs(dg["hbar"][:11, :10] - H[:11, :10]).max() <= 1e-10 * np.abs(H).max()
    assert krylov.relerr(out, ref["f"]) < 1e-9
    assert krylov.relerr(out, fm) < 1e-9
    print(f"case convdiff2d N={N} auto", flush=True)
    out_a, info_a = ctx.solve(A, _dev(b), w.f, make_params(m, w.k, w.s, w.sketch, w.zeta, w.sketch_seed, "auto",
                                                           "auto", 1e-6))
    assert krylov.relerr(out_a.cpu().numpy(), fm) < 1e-6
    A.destroy()
