"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances:
  * sketches: Philox words feed both sides identically; FP64 normals agree to a
    few ulp (libm differences in log/cos/sin), rounded FP32/BF16 sketches are
    equal except at rounding ties (counted, each one unit in the last place);
    SRHT signs and sample indices are bit-exact.
  * FP64 pass: relative Frobenius error <= 1e-13; FP64 approximant <= 1e-10.
  * FP32 / BF16 pass (FP32 accumulation): every entry within the inner-product
    bound gamma_K * (|A| |X|)_ij with gamma_K = K u / (1 - K u), u = 2^-24,
    which holds for any summation order.
"""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gn as OG, philox as OP  # noqa: E402
from paper_2009_11392_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    return gn


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().double().numpy() if t.dtype != torch.bfloat16 else \
        t.detach().cpu().float().double().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def ulp_diff(a, b):
    ai = np.asarray(a, np.float64).view(np.int64)
    bi = np.asarray(b, np.float64).view(np.int64)
    ai = np.where(ai < 0, np.int64(-(1 << 63)) - ai, ai)
    bi = np.where(bi < 0, np.int64(-(1 << 63)) - bi, bi)
    return np.abs(ai - bi)


def gamma(K, u=U32):
    return K * u / (1 - K * u)


def tau_of(p, n=None):
    nx = OG.nu_srht(p.n) if p.kind_x == "srht" else OG.nu_gaussian(p.n, p.r)
    ny = OG.nu_gaussian(p.m, p.rl)
    return OG.threshold(p.eps, nx, ny) if p.eps > 0 else 0.0


# ----------------------------------------------------------------------------- sketches
@pytest.mark.parametrize("layout", [0, 1])
def test_gaussian_f64_matches_oracle(G, layout):
    rows, cols, r0, c0 = 301, 77, 5, 3
    t = G.gn_generate_gaussian(11, 2, rows, cols, torch.float64, layout=layout, row0=r0, col0=c0)
    got = host(t)
    if layout == 1:
        got = got.T
    ref = OP.gaussian(11, 2, rows, cols, row0=r0, col0=c0)
    # Both sides take the same 53-bit uniforms and the same rounded 2 pi u2; they
    # differ only in the libraries' log, sqrt, cos and sin (each within about one
    # ulp, the cosine and sine relative to their result), so z = sqrt(-2 ln u1) *
    # cos(2 pi u2) may differ by a few ulp; 8 ulp is that sum with a margin.
    d = ulp_diff(got, ref)
    print(f"FP64 Gaussian: max {int(np.max(d))} ulp, {float(np.mean(d > 0)):.3f} not bit-equal")
    assert np.max(d) <= 8


def test_gaussian_f64_large_block_within_ulps(G):
    """4M FP64 sketch values (both Box-Muller outputs, u1 down to its smallest
    values and angles in every quadrant) against the oracle's NumPy log, cos and
    sin: the device's Box-Muller steps stay within a few ulp of the library
    functions everywhere, not only on a small block."""
    rows, cols = 4096, 1024
    got = host(G.gn_generate_gaussian(23, 2, rows, cols, torch.float64))
    ref = OP.gaussian(23, 2, rows, cols, workers=8)
    d = ulp_diff(got, ref)
    print(f"FP64 Gaussian, 4M values: max {int(np.max(d))} ulp, {float(np.mean(d > 0)):.3f} not bit-equal")
    assert np.max(d) <= 8


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_gaussian_rounded_equal_except_ties(G, dtype):
    rows, cols = 1000, 333
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    got = host(G.gn_generate_gaussian(5, 1, rows, cols, tdt))
    z = OP.gaussian(5, 1, rows, cols)
    ref = OG.round_mode(z, dtype)
    bad = got != ref
    assert bad.mean() <= 1e-5
    if bad.any():   # only rounding ties: neighbours in the target format
        ulp = np.spacing(np.abs(ref[bad]).astype(np.float32)).astype(np.float64)
        if dtype == "bf16":
            ulp = ulp * 2.0 ** 16
        elif dtype == "f16":
            ulp = np.spacing(np.abs(ref[bad]).astype(np.float16)).astype(np.float64)
        assert np.all(np.abs(got[bad] - ref[bad]) <= ulp * 1.0001)


def test_gaussian_f16_subnormals_and_ties(G):
    """binary16 rounding of the sketch values straight from FP64: a large block so
    that values below 2^-14 (subnormal in binary16) occur, each compared with the
    oracle's direct double-to-half rounding."""
    rows, cols = 4096, 1024
    got = host(G.gn_generate_gaussian(23, 2, rows, cols, torch.float16))
    z = OP.gaussian(23, 2, rows, cols, workers=8)
    ref = OG.round_mode(z, "f16")
    sub = np.abs(z) < 2.0 ** -14
    print(f"binary16 sketch: {int(sub.sum())} subnormal values")
    assert sub.sum() > 0
    assert np.array_equal(got[sub], ref[sub])
    assert np.mean(got != ref) <= 1e-5


@pytest.mark.parametrize("n,r", [(1000, 10), (4096, 1000), (100, 64), (1, 1), (32768, 1000)])
def test_srht_parameters_bit_exact(G, n, r):
    signs, idx = G.gn_srht_generate(77, n, r)
    npad = OP.next_pow2(n)
    assert np.array_equal(signs.cpu().numpy(), OP.srht_signs(77, npad))
    assert np.array_equal(idx.cpu().numpy(), OP.srht_sample(77, npad, r))


# ----------------------------------------------------------------------------- FP64 pipeline
@pytest.fixture(scope="module")
def small(G):
    w = W.SMALL
    A = W.host_matrix(w)
    p = G.Problem(w.m, w.n, w.r, w.l, seed=w.seed, mode="f64", eps=w.eps)
    X, Y = OG.gaussian_sketches(w.seed, w.m, w.n, w.r, w.l)
    ref = OG.gn(A, X, Y, tau_of(p))
    return w, A, p, X, Y, ref


def test_small_pass_f64(G, small):
    w, A, p, X, Y, ref = small
    AX, YtA, _, _ = G.gn_sketch(p, dev(A))
    assert relerr(host(AX), ref.AX) <= 1e-13
    assert relerr(host(YtA), ref.YA) <= 1e-13


def test_small_core_and_approximant_f64(G, small):
    w, A, p, X, Y, ref = small
    Ad = dev(A)
    AX, YtA, core = G.solve(p, Ad)
    assert core.rank() == ref.core.k == w.r
    assert core.flags() == 0
    assert relerr(host(core.R), ref.core.R) <= 1e-12
    assert relerr(host(core.Q1), ref.core.Q) <= 1e-12
    F, Gm = G.gn_factors(p, AX, YtA, core)
    Ahat = host(F) @ host(Gm)
    assert relerr(Ahat, ref.approx) <= 1e-10
    # error measured on the device, tile by tile
    ss = float(G.gn_residual(Ad, F, Gm).item())
    e_ref = OG.residual_fro(A, ref.F, ref.G)
    assert math.isclose(math.sqrt(ss), e_ref, rel_tol=1e-9)


def test_small_apply_both_sides(G, small):
    w, A, p, X, Y, ref = small
    AX, YtA, core = G.solve(p, dev(A))
    Wr = W.host_gaussian(w.n, 7, 21)
    Wl = W.host_gaussian(5, w.m, 22)
    outr = host(G.gn_apply(p, 0, AX, YtA, core, dev(Wr)))
    outl = host(G.gn_apply(p, 1, AX, YtA, core, dev(Wl)))
    assert relerr(outr, OG.apply_right(ref.AX, ref.YA, ref.core, Wr)) <= 1e-10
    assert relerr(outl, OG.apply_left(ref.AX, ref.YA, ref.core, Wl)) <= 1e-10


def test_exact_recovery_on_gpu(G, small):
    w, _, p, X, Y, _ = small
    A = W.spectrum_matrix(w.m, w.n, w.sigma()[:w.r], seed=7)
    AX, YtA, core = G.solve(p, dev(A))
    assert core.rank() == w.r
    F, Gm = G.gn_factors(p, AX, YtA, core)
    assert math.sqrt(float(G.gn_residual(dev(A), F, Gm).item())) / np.linalg.norm(A) <= 1e-12


def test_truncation_rank_on_gpu(G, small):
    w, _, p, X, Y, _ = small
    A = W.spectrum_matrix(w.m, w.n, w.sigma()[:40], seed=8)
    ref = OG.gn(A, X, Y, tau_of(p))
    AX, YtA, core = G.solve(p, dev(A))
    assert core.rank() == ref.core.k == 40
    assert (core.flags() & 3) == 0
    F, Gm = G.gn_factors(p, AX, YtA, core)
    Fh, Gh = host(F), host(Gm)
    assert np.all(Fh[:, 40:] == 0) and np.all(Gh[40:] == 0)
    assert relerr(Fh[:, :40] @ Gh[:40], ref.approx) <= 1e-10
    Wr = W.host_gaussian(w.n, 3, 5)
    Wl = W.host_gaussian(4, w.m, 6)
    assert relerr(host(G.gn_apply(p, 0, AX, YtA, core, dev(Wr))), ref.approx @ Wr) <= 1e-10
    assert relerr(host(G.gn_apply(p, 1, AX, YtA, core, dev(Wl))), Wl @ ref.approx) <= 1e-10


# gn_core runs the kept-rank scan and the second QR on a per-device side stream
# (joined before it returns) and gn_apply prepares its solve there.  Two solves
# enqueued back to back on two streams -- one truncated, so the second QR does
# real work -- give bit for bit the results of the same solves one at a time
# (every kernel sums in a fixed order).
def test_solves_on_two_streams(G, small):
    w, _, p, _, _, _ = small
    mats = [W.spectrum_matrix(w.m, w.n, w.sigma()[:40], seed=8),
            W.spectrum_matrix(w.m, w.n, w.sigma(), seed=9)]
    Wr = W.host_gaussian(w.n, 5, 77)
    serial = []
    for A in mats:
        AX, YtA, core = G.solve(p, dev(A))
        serial.append((core, host(G.gn_apply(p, 0, AX, YtA, core, dev(Wr)))))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    both = []
    for A, st in zip(mats, streams):
        with torch.cuda.stream(st):
            AX, YtA, core = G.solve(p, dev(A))
            both.append((core, G.gn_apply(p, 0, AX, YtA, core, dev(Wr))))
    torch.cuda.synchronize()
    assert serial[0][0].rank() == 40 and serial[1][0].rank() == w.r
    for (c0, o0), (c1, o1) in zip(serial, both):
        k = c0.rank()
        assert c1.rank() == k and c1.flags() == c0.flags()
        for name in ("R", "Q1"):
            assert np.array_equal(host(getattr(c0, name)), host(getattr(c1, name))), name
        if k < w.r:
            assert np.array_equal(host(c0.Q2)[:, :k], host(c1.Q2)[:, :k])
            assert np.array_equal(host(c0.R2)[:k, :k], host(c1.R2)[:k, :k])
        assert np.array_equal(o0, host(o1))


# ----------------------------------------------------------------------------- FP32 / BF16 pass
def test_pass_f32_gaussian_ragged(G):
    m, n, r, l = 777, 1234, 37, 19
    A = W.spectrum_matrix(m, n, 0.95 ** np.arange(1, 301), seed=31).astype(np.float32)
    p = G.Problem(m, n, r, l, seed=9, mode="f32")
    AX, YtA, _, _ = G.gn_sketch(p, dev(A, torch.float32))
    X, Y = OG.gaussian_sketches(9, m, n, r, l, mode="f32")
    A64 = A.astype(np.float64)
    ax, ya = host(AX), host(YtA)
    assert np.all(np.abs(ax - A64 @ X) <= gamma(n) * (np.abs(A64) @ np.abs(X)))
    assert np.all(np.abs(ya - Y.T @ A64) <= gamma(m) * (np.abs(Y.T) @ np.abs(A64)))
    assert relerr(ax, A64 @ X) <= 1e-5 and relerr(ya, Y.T @ A64) <= 1e-5


# r up to 512 and r + l up to 768 on wide or tall matrices: tiles of 64 sketch
# rows (Y^T A) or columns (AX) by 256, so the narrow side is padded to 64 instead
# of 256, with K split into slices summed in order where the tiles are few.
# Ragged m and n, vector (r, r + l, lda multiples of 4) and scalar loads, r and
# r + l not multiples of 64, and the limits r = 512, r + l = 768.
@pytest.mark.parametrize("m,n,r,l", [(3001, 33024, 16, 8), (4196, 30000, 20, 10),
                                     (5000, 8200, 128, 64), (2500, 32770, 4, 2),
                                     (3000, 8192, 256, 128), (1500, 5001, 449, 223),
                                     (1030, 4100, 512, 256), (8192, 4100, 300, 150)])
def test_pass_f32_gaussian_narrow_tiles(G, m, n, r, l):
    A = np.random.default_rng(m + n).standard_normal((m, n)).astype(np.float32)
    p = G.Problem(m, n, r, l, seed=11, mode="f32")
    AX, YtA, _, _ = G.gn_sketch(p, dev(A, torch.float32))
    X, Y = OG.gaussian_sketches(11, m, n, r, l, mode="f32")
    A64 = A.astype(np.float64)
    ax, ya = host(AX), host(YtA)
    ref_ax, ref_ya = A64 @ X, Y.T @ A64
    Aa = np.abs(A64)
    assert np.all(np.abs(ax - ref_ax) <= gamma(n) * (Aa @ np.abs(X)))
    assert np.all(np.abs(ya - ref_ya) <= gamma(m) * (np.abs(Y.T) @ Aa))
    assert relerr(ax, ref_ax) <= 1e-5 and relerr(ya, ref_ya) <= 1e-5


# r + l <= 16 with a Gaussian X: the single-read narrow pass (one 256-column chunk
# per wave; Y^T A from the loaded registers, AX from the same values staged in LDS
# 16 rows at a time, both on the matrix cores; partials added in order).  Ragged
# rows (not a multiple of 16), a ragged last chunk, padding chunks past n (n =
# 1236: 5 chunks rounded up to 8), r + l = 1 and 16; and just past the limit (r +
# l = 17, 24, 32), where the narrow tiles take over.
@pytest.mark.parametrize("m,n,r,l", [(1001, 3000, 7, 5), (4096, 4096, 10, 6), (37, 1024, 1, 0),
                                     (2050, 8192, 16, 0), (300, 1236, 5, 3), (1001, 3000, 12, 5),
                                     (700, 1024, 16, 8), (2050, 8192, 21, 11), (517, 2000, 4, 13)])
def test_pass_f32_gaussian_single_read(G, m, n, r, l):
    A = np.random.default_rng(m * n).standard_normal((m, n)).astype(np.float32)
    p = G.Problem(m, n, r, l, seed=12, mode="f32")
    AX, YtA, _, _ = G.gn_sketch(p, dev(A, torch.float32))
    X, Y = OG.gaussian_sketches(12, m, n, r, l, mode="f32")
    A64 = A.astype(np.float64)
    ax, ya = host(AX), host(YtA)
    ref_ax, ref_ya = A64 @ X, Y.T @ A64
    Aa = np.abs(A64)
    assert np.all(np.abs(ax - ref_ax) <= gamma(n) * (Aa @ np.abs(X)))
    assert np.all(np.abs(ya - ref_ya) <= gamma(m) * (np.abs(Y.T) @ Aa))
    assert relerr(ax, ref_ax) <= 1e-5 and relerr(ya, ref_ya) <= 1e-5


def test_pass_srht_integer_inputs_exact(G):
    m, n, r = 170, 1000, 100         # n' = 1024: two 512-column chunks, ragged tail
    A = W.integer_matrix(m, n, 41).astype(np.float32)
    p = G.Problem(m, n, r, 50, kind_x="srht", seed=4, mode="f32")
    AX, YtA, signs, idx = G.gn_sketch(p, dev(A, torch.float32), want_srht=True)
    npad = OP.next_pow2(n)
    assert np.array_equal(signs.cpu().numpy(), OP.srht_signs(4, npad))
    assert np.array_equal(idx.cpu().numpy(), OP.srht_sample(4, npad, r))
    X = OP.srht_matrix(4, n, r)
    A64 = A.astype(np.float64)
    assert np.array_equal(host(AX), A64 @ X)   # integers: exact
    # Y^T A with the FP32 Gaussian Y: every entry within the inner-product bound
    _, Y = OG.gaussian_sketches(4, m, n, r, 50, mode="f32")
    ya = host(YtA)
    assert np.all(np.abs(ya - Y.T @ A64) <= gamma(m) * (np.abs(Y.T) @ np.abs(A64)))
    assert relerr(ya, Y.T @ A64) <= 1e-5


# r + l <= 16 with an SRHT X: the single-read narrow pass (one 256-column chunk per
# wave, the Walsh-Hadamard transform and the Y^T A product from the same registers,
# partial sums added in a fixed order).  Integer A: AX exact; Y^T A within gamma_m.
# Ragged row counts, n not a power of two (chunks past n), r + l = 1 and 16, and
# n % 4 != 0 (which takes the fused 256 x 256 kernel instead).
@pytest.mark.parametrize("m,n,r,l", [(1001, 3000, 7, 5), (4096, 4096, 10, 6), (37, 1024, 1, 0),
                                     (2050, 8192, 16, 0), (500, 2048, 3, 2), (300, 1234, 5, 3)])
def test_pass_srht_narrow(G, m, n, r, l):
    A = W.integer_matrix(m, n, 43).astype(np.float32)
    p = G.Problem(m, n, r, l, kind_x="srht", seed=8, mode="f32")
    AX, YtA, signs, idx = G.gn_sketch(p, dev(A, torch.float32), want_srht=True)
    npad = OP.next_pow2(n)
    assert np.array_equal(signs.cpu().numpy(), OP.srht_signs(8, npad))
    assert np.array_equal(idx.cpu().numpy(), OP.srht_sample(8, npad, r))
    A64 = A.astype(np.float64)
    assert np.array_equal(host(AX), A64 @ OP.srht_matrix(8, n, r))   # integers: exact
    Y = OG.round_mode(OP.gaussian(8, OP.STREAM_Y, m, r + l), "f32")
    ya, ref = host(YtA), Y.T @ A64
    assert np.all(np.abs(ya - ref) <= gamma(m) * (np.abs(Y.T) @ np.abs(A64)))
    assert relerr(ya, ref) <= 5e-6


def test_pass_srht_f64_matches_oracle(G):
    m, n, r = 300, 700, 90
    A = W.spectrum_matrix(m, n, 0.9 ** np.arange(1, 301), seed=12)
    p = G.Problem(m, n, r, 45, kind_x="srht", seed=6, mode="f64")
    AX, _, _, _ = G.gn_sketch(p, dev(A))
    assert relerr(host(AX), A @ OP.srht_matrix(6, n, r)) <= 1e-13


SKETCH_DT = {"bf16": torch.bfloat16, "f16": torch.float16}


def quantize(G, mode, A):
    return G.gn_quantize_f16_bs(A) if mode == "f16" else G.gn_quantize_bf16_bs(A)


def quantize_oracle(mode, A):
    if mode == "f16":
        rb, rs = OG.block_quantize_f16(A)
        return rb, rs, OG.block_dequantize_f16(rb, rs)
    rb, rs = OG.block_quantize_bf16(A)
    return rb, rs, OG.block_dequantize_bf16(rb, rs)


@pytest.mark.parametrize("mode", ["bf16", "f16"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_quantize_bit_exact(G, mode, dtype):
    A = W.spectrum_matrix(300, 260, 0.9 ** np.arange(1, 261), seed=9)
    A[:128, :128] = 0.0
    A[130:140, 200:210] *= 1e-4       # tiny entries: binary16 subnormals after scaling
    A = A.astype(np.float32).astype(np.float64) if dtype == torch.float32 else A
    bits, scales = quantize(G, mode, dev(A, dtype))
    rb, rs, _ = quantize_oracle(mode, A)
    assert np.array_equal(bits.view(torch.int16).cpu().numpy().view(np.uint16), rb)
    assert np.array_equal(scales.cpu().numpy(), rs)


@pytest.mark.parametrize("mode", ["bf16", "f16"])
def test_pass_h16_block_scaled(G, mode):
    m, n, r, l = 300, 260, 40, 20
    A = W.spectrum_matrix(m, n, 0.9 ** np.arange(1, 261), seed=13)
    bits, scales = quantize(G, mode, dev(A))
    p = G.Problem(m, n, r, l, seed=3, mode=mode)
    AX, YtA, _, _ = G.gn_sketch(p, bits, scales=scales)
    _, _, Aq = quantize_oracle(mode, A)
    X, Y = OG.gaussian_sketches(3, m, n, r, l, mode=mode)
    ax, ya = host(AX), host(YtA)
    assert np.all(np.abs(ax - Aq @ X) <= gamma(n) * (np.abs(Aq) @ np.abs(X)))
    assert np.all(np.abs(ya - Y.T @ Aq) <= gamma(m) * (np.abs(Y.T) @ np.abs(Aq)))


# The large 16-bit tile (256 x 256 per workgroup, direct-to-LDS staging; taken
# when m and n are multiples of 8): ragged output tiles in both families, K not
# a multiple of the 32-deep stage, a tiny r, and three kinds of block scales --
# uniform along each 128-row / 128-column stripe, mixed (some blocks 2^-3 or 2^-6
# smaller: the non-matrix fragments are scaled by powers of two), and wide (one
# block 2^-12 smaller for binary16, 2^-40 for bfloat16: beyond the scaled range,
# so those tiles take the general tile).  Every entry within the FP32
# inner-product bound of the oracle's product of the dequantized matrix and the
# sketches' 16-bit values.
@pytest.mark.parametrize("mode", ["bf16", "f16"])
@pytest.mark.parametrize("scales_kind", ["uniform", "mixed", "wide"])
@pytest.mark.parametrize("m,n,r,l", [(1000, 1032, 300, 150), (776, 1000, 8, 4)])
def test_pass_h16_large_tile(G, mode, scales_kind, m, n, r, l):
    A = W.spectrum_matrix(m, n, np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.0, seed=31)
    if scales_kind != "uniform":
        A[128:256, 256:384] *= 2.0 ** -3
        A[512:640, 0:128] *= 2.0 ** -6
    if scales_kind == "wide":
        A[0:128, 640:768] *= 2.0 ** (-12 if mode == "f16" else -40)
    bits, scales = quantize(G, mode, dev(A))
    p = G.Problem(m, n, r, l, seed=8, mode=mode)
    AX, YtA, _, _ = G.gn_sketch(p, bits, scales=scales)
    _, _, Aq = quantize_oracle(mode, A)
    X, Y = OG.gaussian_sketches(8, m, n, r, l, mode=mode)
    ax, ya = host(AX), host(YtA)
    ref_ax, ref_ya = Aq @ X, Y.T @ Aq
    bad_ax = np.abs(ax - ref_ax) > gamma(n) * (np.abs(Aq) @ np.abs(X))
    bad_ya = np.abs(ya - ref_ya) > gamma(m) * (np.abs(Y.T) @ np.abs(Aq))
    print(f"{mode} {scales_kind} {m}x{n} r={r}: AX rel err {relerr(ax, ref_ax):.2e}, "
          f"Y^T A rel err {relerr(ya, ref_ya):.2e}, outside bound {int(bad_ax.sum())}, "
          f"{int(bad_ya.sum())}")
    assert not bad_ax.any() and not bad_ya.any()


# Small r (at most 64) and r + l (at most 96) in the 16-bit modes: the general
# 16-bit tile with 64 sketch rows / columns by 256, K split into slices that
# start on block-scale boundaries.  Block scales mixed (some 128 x 128 blocks
# 2^-5 smaller), ragged m and n, m not a multiple of 8 (scalar loads of Y^T), and
# the limits r = 64, r + l = 96.
@pytest.mark.parametrize("mode", ["bf16", "f16"])
@pytest.mark.parametrize("m,n,r,l", [(3000, 30000, 16, 8), (2999, 33000, 5, 3),
                                     (4104, 16384, 64, 32)])
def test_pass_h16_narrow_tiles(G, mode, m, n, r, l):
    A = np.random.default_rng(m + n + r).standard_normal((m, n))
    A[128:256, 256:384] *= 2.0 ** -5
    A[512:640, 0:128] *= 2.0 ** -5
    bits, scales = quantize(G, mode, dev(A))
    p = G.Problem(m, n, r, l, seed=8, mode=mode)
    AX, YtA, _, _ = G.gn_sketch(p, bits, scales=scales)
    _, _, Aq = quantize_oracle(mode, A)
    X, Y = OG.gaussian_sketches(8, m, n, r, l, mode=mode)
    ax, ya = host(AX), host(YtA)
    ref_ax, ref_ya = Aq @ X, Y.T @ Aq
    Aa = np.abs(Aq)
    assert np.all(np.abs(ax - ref_ax) <= gamma(n) * (Aa @ np.abs(X)))
    assert np.all(np.abs(ya - ref_ya) <= gamma(m) * (np.abs(Y.T) @ Aa))


# ----------------------------------------------------------------------------- edge cases
def test_nonfinite_input_sets_status(G):
    m, n, r = 200, 150, 10
    A = W.spectrum_matrix(m, n, 0.9 ** np.arange(1, 151), seed=1)
    A[3, 4] = np.nan
    p = G.Problem(m, n, r, 5, seed=1, mode="f64", eps=1e-15)
    _, _, core = G.solve(p, dev(A))
    assert core.flags() & 1


# ----------------------------------------------------------------------------- FP32 / BF16 solves
def _noisy(m, n, seed):
    sig = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -2.0
    return W.spectrum_matrix(m, n, sig[:512], seed=seed, noise=1e-5)


@pytest.mark.parametrize("mode,kind_x", [("f32", "gaussian"), ("f32", "srht"),
                                         ("bf16", "gaussian"), ("bf16", "srht"),
                                         ("f16", "gaussian"), ("f16", "srht")])
def test_low_precision_solve_within_5pct_of_oracle(G, mode, kind_x):
    """FP32 / BF16 pass + FP64 core: ||A - A_hat||_F <= 1.05 x the FP64 oracle's
    error with the same sketches (the error is measured against the FP64 A)."""
    m, n, r, l = 3000, 2000, 200, 100
    A = _noisy(m, n, 21)
    eps = 10 * U32
    p = G.Problem(m, n, r, l, kind_x=kind_x, seed=17, mode=mode, eps=eps)
    if mode == "f32":
        Ad, sc = dev(A, torch.float32), None
    else:
        Ad, sc = quantize(G, mode, dev(A))
    AX, YtA, _, _ = G.gn_sketch(p, Ad, scales=sc)
    core = G.gn_core(p, AX)
    assert (core.flags() & 3) == 0
    F, Gm = G.gn_factors(p, AX, YtA, core)
    e_gpu = math.sqrt(float(G.gn_residual(dev(A), F, Gm).item()))
    # oracle: FP64 GN on the FP64 A with the working-precision sketch values
    if kind_x == "srht":
        X = OP.srht_matrix(17, n, r)
        Y = OG.round_mode(OP.gaussian(17, OP.STREAM_Y, m, r + l), mode)
        nx = OG.nu_srht(n)
    else:
        X, Y = OG.gaussian_sketches(17, m, n, r, l, mode=mode)
        nx = OG.nu_gaussian(n, r)
    ref = OG.gn(A, X, Y, OG.threshold(eps, nx, OG.nu_gaussian(m, r + l)))
    e_ref = OG.residual_fro(A, ref.F, ref.G)
    assert e_gpu <= 1.05 * e_ref, (e_gpu, e_ref)


# BF16 mode: the core matrix on the BF16 matrix cores (Y's bfloat16 values, AX in
# two bfloat16 terms, FP32 accumulation) against the oracle's FP64 Y^T (AX) on the
# same sketch values, next to the FP32-matrix-core product the mode uses for a user
# Y (the same Y given as user values).  Both carry FP32 accumulation error; the
# two-term split adds at most 2^-17 relative per entry of AX, so the BF16 product
# may not be more than a few times further from the oracle than the FP32 one.
@pytest.mark.parametrize("mode", ["bf16", "f16"])
def test_core_bf16_product(G, mode):
    m, n, r, l = 3000, 2000, 200, 100
    A = _noisy(m, n, 21)
    p = G.Problem(m, n, r, l, seed=17, mode=mode, eps=10 * U32)
    Ad, sc = quantize(G, mode, dev(A))
    AX, YtA, _, _ = G.gn_sketch(p, Ad, scales=sc)
    core = G.gn_core(p, AX)
    Yb = G.gn_generate_gaussian(17, 2, m, p.rl, dtype=SKETCH_DT[mode])
    pu = dataclasses.replace(p, kind_y="user", nu_y=OG.nu_gaussian(m, p.rl))
    core32 = G.gn_core(pu, AX, Y_user=Yb)
    Y = OG.round_mode(OP.gaussian(17, OP.STREAM_Y, m, p.rl), mode)
    assert np.array_equal(Yb.float().cpu().numpy().astype(np.float64), Y)
    ref = OG.core(host(AX), Y, 0.0)
    e16, e32 = relerr(host(core.R), ref.R), relerr(host(core32.R), ref.R)
    assert e16 <= 1e-5 and e32 <= 1e-5, (e16, e32)
    assert core.rank() == core32.rank()


# The FP16 core product divides each column of AX by a power of two before the
# two-term binary16 split: columns spread over 10^-8 .. 10^8 (far outside
# binary16's range unscaled) must each come out of the product to FP32-like
# relative accuracy.  Householder QR is columnwise backward stable, so Q1 R
# reproduces every column of C = Y^T (AX) to that accuracy.
def test_core_f16_product_wide_columns(G):
    m, r, l = 2048, 64, 32
    rng = np.random.default_rng(5)
    AXh = (rng.standard_normal((m, r)) * 10.0 ** rng.uniform(-8, 8, r)).astype(np.float32)
    p = G.Problem(m, 4 * r, r, l, seed=23, mode="f16")
    core = G.gn_core(p, dev(AXh, torch.float32))
    Y = OG.round_mode(OP.gaussian(23, OP.STREAM_Y, m, p.rl), "f16")
    C = Y.T @ AXh.astype(np.float64)
    QR = host(core.Q1) @ host(core.R)
    err = np.linalg.norm(QR - C, axis=0) / np.linalg.norm(C, axis=0)
    print(f"FP16 core product, wide columns: worst column rel err {err.max():.2e}")
    assert core.rank() == r and err.max() <= 1e-5


# ----------------------------------------------------------------------------- products, several blocks
# r = 300: five 64-row blocks of the triangular solve, the last ragged.  16
# right-hand sides take the few-right-hand-side solver, 40 the blocked one; both
# against the oracle's products, untruncated (k = r) and truncated (k = 220).
@pytest.mark.parametrize("rank", [300, 220])
def test_apply_multiblock(G, rank):
    m, n, r = 900, 700, 300
    A = W.spectrum_matrix(m, n, 0.97 ** np.arange(rank), seed=31)
    p = G.Problem(m, n, r, seed=19, mode="f64", eps=1e-12)
    X = OP.gaussian(p.seed, OP.STREAM_X, n, r)
    Y = OP.gaussian(p.seed, OP.STREAM_Y, m, p.rl)
    ref = OG.gn(A, X, Y, tau_of(p))
    AX, YtA, core = G.solve(p, dev(A))
    assert core.rank() == ref.core.k == min(rank, r)
    for kc in (16, 40):
        Wr = W.host_gaussian(n, kc, 30 + kc)
        Wl = W.host_gaussian(kc, m, 31 + kc)
        outr = host(G.gn_apply(p, 0, AX, YtA, core, dev(Wr)))
        outl = host(G.gn_apply(p, 1, AX, YtA, core, dev(Wl)))
        assert relerr(outr, OG.apply_right(ref.AX, ref.YA, ref.core, Wr)) <= 1e-10
        assert relerr(outl, OG.apply_left(ref.AX, ref.YA, ref.core, Wl)) <= 1e-10


# ----------------------------------------------------------------------------- core as (Y^T A) X
# FP32 pass with an SRHT X: gn_core given Y^T A forms the core matrix as
# (Y^T A) X by the FP64 transform of Y^T A's rows; against the oracle's QR of
# (Y^T A) X on the same FP32 sketch (widened), and products with both cores.
def test_core_right_srht_f32(G):
    m, n, r, l = 1500, 1200, 100, 50     # n' = 2048: four 512-column chunks, ragged
    A = W.spectrum_matrix(m, n, 0.97 ** np.arange(300), seed=35).astype(np.float32)
    p = G.Problem(m, n, r, l, kind_x="srht", seed=27, mode="f32", eps=1e-7)
    AX, YtA, _, _ = G.gn_sketch(p, dev(A, torch.float32))
    core = G.gn_core(p, AX, YtA=YtA)
    ya = host(YtA)
    ref = OG.core_right(ya, OP.srht_matrix(27, n, r), tau_of(p))
    assert core.rank() == ref.k
    assert relerr(host(core.R), ref.R) <= 1e-12
    Wr = W.host_gaussian(n, 8, 61)
    out = host(G.gn_apply(p, 0, AX, YtA, core, dev(Wr)))
    assert relerr(out, OG.apply_right(host(AX), ya, ref, Wr)) <= 1e-10


# ----------------------------------------------------------------------------- few-column products
# FP32 factors (AX, Y^T A as the FP32 pass stores them): products with 1, 7 and 16
# columns (rows) take the narrow-factor kernels -- K-contiguous and M-contiguous
# left factors, several K slices with ragged ends -- and 17 the tiled kernel.  All
# are checked against the materialized factors F, G (gn_factors: a separate path)
# multiplied on the host in FP64.
def test_apply_few_columns_f32(G):
    m, n, r, l = 3000, 2500, 200, 100
    A = W.spectrum_matrix(m, n, 0.97 ** np.arange(300), seed=33).astype(np.float32)
    p = G.Problem(m, n, r, l, seed=23, mode="f32", eps=1e-6)
    AX, YtA, core = G.solve(p, dev(A, torch.float32))
    assert AX.dtype == torch.float32 and YtA.dtype == torch.float32
    F, Gm = G.gn_factors(p, AX, YtA, core)
    Fh, Gh = host(F), host(Gm)
    for kc in (1, 7, 16, 17):
        Wr = W.host_gaussian(n, kc, 50 + kc)
        Wl = W.host_gaussian(kc, m, 51 + kc)
        outr = host(G.gn_apply(p, 0, AX, YtA, core, dev(Wr)))
        outl = host(G.gn_apply(p, 1, AX, YtA, core, dev(Wl)))
        assert relerr(outr, Fh @ (Gh @ Wr)) <= 1e-10, kc
        assert relerr(outl, (Wl @ Fh) @ Gh) <= 1e-10, kc


# ----------------------------------------------------------------------------- larger cores
# Core shapes that exercise every panel configuration of the QR (1 to 8 rows per
# thread, panel widths 16 and 8) and the second QR of a truncated core.
@pytest.mark.parametrize("m,r,l,drop", [(2048, 1000, 500, 0), (2048, 1200, 600, 0),
                                        (3072, 2000, 1000, 0), (4096, 2700, 1350, 0),
                                        (2048, 900, 450, 60)])
def test_core_large_f64(G, m, r, l, drop):
    rng = np.random.default_rng(r + drop)
    AX = rng.standard_normal((m, r))
    if drop:   # the last `drop` columns are combinations of the others: rank r - drop
        AX[:, r - drop:] = AX[:, :r - drop] @ rng.standard_normal((r - drop, drop))
    eps = 1e-9 if drop else 0.0
    p = G.Problem(m, m, r, l, seed=11, mode="f64", eps=eps)
    Y = OP.gaussian(p.seed, OP.STREAM_Y, m, p.rl)
    ref = OG.core(AX, Y, tau_of(p))
    core = G.gn_core(p, dev(AX))
    k = ref.k
    assert core.rank() == k == r - drop
    assert (core.flags() & 3) == 0
    assert relerr(host(core.R)[:k], ref.R[:k]) <= 1e-12
    assert relerr(host(core.Q1)[:, :k], ref.Q[:, :k]) <= 1e-12
    if drop:
        assert relerr(host(core.Q2)[:, :k], ref.Q2) <= 1e-11
        assert relerr(np.triu(host(core.R2)[:k, :k]), ref.R2) <= 1e-11
