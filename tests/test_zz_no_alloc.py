"""gn_residual_noalloc (the entry point that allocates nothing) against
gn_residual through the C ABI -- needs a GPU.

Both run the same residual kernels with the same fixed-order reduction; one keeps
the per-tile partial sums in a caller workspace, the other in the library's
device array.  Two calls in a row on the same array (the second on a smaller
problem, so stale partials of the first stay in the array past the second's
tiles) must each equal gn_residual bit for bit, for FP32 and bfloat16 (with
block scales) matrices; sizes beyond the array are refused before any launch.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import gn as OG  # noqa: E402
from paper_2009_11392_amd import _capi as C  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    return gn


def _inputs(m, n, k, seed, dtype):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randn(m, n, generator=g, device="cuda", dtype=torch.float32)
    F = torch.randn(m, k, generator=g, device="cuda", dtype=torch.float64)
    Gm = torch.randn(k, n, generator=g, device="cuda", dtype=torch.float64) * 0.1
    return A, F, Gm


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_noalloc_equals_workspace_entry_point(G, dtype):
    outs = []
    for (m, n, k, seed) in ((3000, 2100, 20, 1), (700, 500, 7, 2)):
        print(f"\n[noalloc] {dtype} m={m} n={n} k={k}", flush=True)
        A, F, Gm = _inputs(m, n, k, seed, dtype)
        scales = None
        if dtype == "bf16":
            A, scales = G.gn_quantize_bf16_bs(A)
        ref = G.gn_residual(A, F, Gm, scales=scales)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        got = G.gn_residual_noalloc(A, F, Gm, scales=scales, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), (float(got.item()), float(ref.item()))
        # and the value itself against the oracle's block-row residual in FP64
        if dtype == "bf16":
            bits = A.view(torch.int16).cpu().numpy().view(np.uint16)
            Ah = OG.block_dequantize_bf16(bits, scales.cpu().numpy())
        else:
            Ah = A.cpu().double().numpy()
        e = OG.residual_fro(Ah, F.cpu().numpy(), Gm.cpu().numpy()) ** 2
        assert abs(float(got.item()) - e) <= 1e-12 * e
        outs.append(float(got.item()))
    assert outs[0] != outs[1]


def test_noalloc_rejects_sizes_beyond_the_array(G):
    lib = C.lib()
    A = torch.zeros(8, 8, dtype=torch.float32, device="cuda")
    F = torch.zeros(8, 1, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    # 32769 x 32768 needs 513 x 512 > 262144 tiles: refused before anything runs
    code = lib.gn_residual_noalloc(32769, 32768, 1, A.data_ptr(), 32768, C.GN_DT_F32, None,
                                   F.data_ptr(), 1, F.data_ptr(), 32768, out.data_ptr(), None)
    assert code == C.GN_ERR_UNSUPPORTED
    code = lib.gn_residual_noalloc(8, 8, 1, None, 8, C.GN_DT_F32, None, F.data_ptr(), 1,
                                   F.data_ptr(), 8, out.data_ptr(), None)
    assert code == C.GN_ERR_ARG
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0
