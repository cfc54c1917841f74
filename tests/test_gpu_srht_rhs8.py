"""The SRHT of Section 2.1.1 on blocks of exactly 8 right-hand sides, the
layout where k_update keeps the sums of the first sampled rows in registers
(how many depends on the window length the kernel is instantiated for:
k <= 2, k <= 4, k > 4 keep 1, 2 and 0 rows per thread) and the rest in LDS,
with two tile buffers for the transform.  Every column of Theta V, Hbar and
the result of each rhs against the oracle's Algorithm 2 run on that rhs
alone, on both tile sizes (512-element tiles below 2^20 elements, 2048
above), with s larger than the rows held in registers so that both kinds of
sums are exercised, a ragged last tile, FP64 (1e-11 / 1e-10) and FP32 (the
result within 1e-6 of the oracle)."""
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


# N = 21: 9261 rows x 8 (512-element tiles, 64-thread blocks, ragged);
# N = 52: 140608 rows x 8 >= 2^20 (2048-element tiles, 256-thread blocks)
@pytest.mark.parametrize("N,k,s", [(21, 2, 150), (21, 4, 200), (21, 6, 150), (52, 2, 300), (52, 4, 600)])
def test_srht_eight_rhs_sums(ctx, N, k, s):
    from paper_2212_12758_amd import make_params

    st = W.convdiff3d(N, 50.0)
    nrhs, m, seed = 8, 20, 23
    f = W.FuncSpec("exp", alpha=-1e-3)
    Aor = operators.as_matrix(st)
    B = W.rhs(st.n, 80 + k, nrhs)
    A = ctx.matrix(st)
    print(f"case srht 8 rhs N={N} k={k} s={s}", flush=True)
    out, info, dg = ctx.solve(A, _dev(B), f, make_params(m, k, s, "srht", 8, seed, "fp64", "sketch"), diag=True)
    out = out.cpu().numpy()
    out32, _ = ctx.solve(A, _dev(B), f, make_params(m, k, s, "srht", 8, seed, "fp32", "sketch"))
    out32 = out32.cpu().numpy()
    sk = osk.Sketch("srht", st.n, s, seed, 8)
    for q in range(nrhs):
        ref = krylov.nt(Aor, np.ascontiguousarray(B[:, q]), f, m, k, sk, "sketch")
        H = ref["Hbar"]
        assert np.abs(dg["hbar"][q] - H).max() <= 1e-12 * np.abs(H).max(), q
        np.testing.assert_allclose(dg["sv"][q], ref["SV"], rtol=0, atol=1e-11, err_msg=f"rhs {q}")
        assert krylov.relerr(out[:, q], ref["f"]) < 1e-10, q
        assert krylov.relerr(out32[:, q], ref["f"]) < 1e-6, q
    A.destroy()
