"""Full-size GPU parity: the 32768 x 32768 FP32 solve with an SRHT X (r = 1000)
and a Gaussian Y (l = 500), called exactly as the benchmark times it
(prepare, fused pass, core from (Y^T A) X, right apply), checked on outputs the
oracle can compute one by one and on properties that hold at any size.

  * pass: sampled rows of AX (A's rows times the oracle's explicit SRHT matrix,
    Sections 1 and 3.5.1) and sampled rows of Y^T A (the oracle's Philox columns of Y times
    A, summed over row blocks of A on the host), each entry within the
    inner-product bound gamma_K (|.| |.|)_ij and the rows within a relative
    Frobenius error 2e-5 (sequential FP32 accumulation over K = 32768 gives
    about 2.4e-6 on Gaussian data);
  * SRHT signs and sample: bit-exact;
  * core (Section 5.1, 5.1.1): Q orthonormal, R upper triangular with a
    non-negative diagonal, Q R equal to sampled columns of (Y^T A) X, the kept
    rank the first diagonal below the threshold, and R_1^T = Q_2 R_2 when
    truncated;
  * apply (Section 2): sampled rows of A_hat W equal the factored form
    AX R^-1 Q^T (Y^T A W) (or its truncated form) evaluated on the host from the
    library's own factors;
  * the core against the oracle's core_right on the library's own Y^T A (R and
    Q to 1e-12, the kept rank equal);
  * accuracy (eq. (4)): the solve's ||A - A_hat||_F within 1.05 times the FP64
    oracle's on the same matrix and the same sketch values, at this size (and
    for the BF16 variant below, against the unquantized matrix).
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")

from oracle import gn as OG, philox as OP  # noqa: E402
from paper_2009_11392_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def gamma(K, u=U32):
    return K * u / (1 - K * u)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def host_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def near_ties(d, tau):
    """Diagonal entries (or singular values) where two correct implementations may
    keep a different rank: within a factor 2 of the threshold."""
    d = np.abs(np.asarray(d))
    return int(np.sum((d >= 0.5 * tau) & (d <= 2.0 * tau)))


def check_rank(k_gpu, k_ref, d_ref, tau):
    """The kept rank equals the oracle's unless the oracle's diagonal has near-ties
    at the threshold; then it may differ by at most their number."""
    nt = near_ties(d_ref, tau)
    if nt == 0:
        assert k_gpu == k_ref, (k_gpu, k_ref)
    else:
        print(f"  {nt} near-tie(s) at tau: kept ranks {k_gpu} (GPU) and {k_ref} (oracle)")
        assert abs(k_gpu - k_ref) <= nt, (k_gpu, k_ref, nt)


def oracle_error(A64, X, Y, tau):
    """The FP64 oracle's GN (Algorithm 2.1 with the Section 5.1.1 truncation) on
    the host and its ||A - A_hat||_F (formed block row by block row)."""
    ref = OG.gn(A64, X, Y, tau)
    return OG.residual_fro(A64, ref.F, ref.G), ref


def host(t):
    return t.detach().cpu().double().numpy()


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    w = W.SRHT32K
    print(f"\n[full-size] {w.name}: generating A on the device", flush=True)
    A = W.device_matrix(w)
    p = gn.Problem(w.m, w.n, w.r, w.l, kind_x=w.kind_x, kind_y=w.kind_y, seed=w.seed,
                   mode=w.mode, eps=w.eps)
    ws = gn.workspace(p, gn.C.GN_OP_SKETCH)
    ws_core = gn.workspace(p, gn.C.GN_OP_CORE)
    AX = torch.empty(w.m, w.r, dtype=torch.float32, device="cuda")
    YtA = torch.empty(p.rl, w.n, dtype=torch.float32, device="cuda")
    core = gn.new_core(p)
    Wr = W.host_gaussian(w.n, 16, 99)
    Wd = torch.from_numpy(Wr).cuda()
    out = torch.empty(w.m, 16, dtype=torch.float64, device="cuda")
    print("[full-size] prepare, pass, core, apply", flush=True)
    signs, idx = gn.gn_sketch_prepare(p, ws, want_srht=True)
    gn.gn_sketch_pass(p, A, ws, AX=AX, YtA=YtA)
    gn.gn_core(p, AX, out=core, ws=ws_core, YtA=YtA)
    gn.gn_apply(p, 0, AX, YtA, core, Wd, out=out)
    torch.cuda.synchronize()
    npad = OP.next_pow2(w.n)
    print("[full-size] oracle SRHT matrix", flush=True)
    X = OP.srht_matrix(w.seed, w.n, w.r)
    return dict(gn=gn, w=w, p=p, A=A, AX=AX, YtA=YtA, core=core, Wr=Wr, out=out,
                signs=signs.cpu().numpy(), idx=idx.cpu().numpy(), npad=npad, X=X)


def test_full_srht_parameters_bit_exact(full):
    w, npad = full["w"], full["npad"]
    assert np.array_equal(full["signs"], OP.srht_signs(w.seed, npad))
    assert np.array_equal(full["idx"], OP.srht_sample(w.seed, npad, w.r))


def test_full_pass_ax_sampled_rows(full):
    w, A, X = full["w"], full["A"], full["X"]
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([[0, 1, 255, 256, 16383, 16384, w.m - 2, w.m - 1],
                                     rng.integers(0, w.m, 24)]))
    rt = torch.from_numpy(rows).cuda()
    Ar = host(A.index_select(0, rt))
    ref = Ar @ X
    got = host(full["AX"].index_select(0, rt))
    bound = gamma(w.n) * (np.abs(Ar) @ np.abs(X))
    assert np.all(np.abs(got - ref) <= bound)
    e = relerr(got, ref)
    print(f"AX sampled rows: rel err {e:.3e}")
    assert e <= 2e-5


def test_full_pass_yta_sampled_rows(full):
    w, p, A = full["w"], full["p"], full["A"]
    rng = np.random.default_rng(8)
    sel = np.unique(np.concatenate([[0, 1, 255, 256, 999, 1000, 1279, 1280, p.rl - 1],
                                    rng.integers(0, p.rl, 7)]))
    # the oracle's Y columns (Philox stream of Y), rounded to the working precision
    Ys = np.concatenate([OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, 1, col0=int(a)), "f32")
                         for a in sel], axis=1)
    ref = np.zeros((len(sel), w.n))
    mag = np.zeros((len(sel), w.n))
    step = 2048
    for i0 in range(0, w.m, step):
        Ab = host(A[i0:i0 + step])
        yb = Ys[i0:i0 + step]
        ref += yb.T @ Ab
        mag += np.abs(yb).T @ np.abs(Ab)
    got = host(full["YtA"].index_select(0, torch.from_numpy(sel).cuda()))
    assert np.all(np.abs(got - ref) <= gamma(w.m) * mag)
    e = relerr(got, ref)
    print(f"Y^T A sampled rows: rel err {e:.3e}")
    assert e <= 2e-5


@pytest.fixture(scope="module")
def full_r10(full):
    """The same resident matrix at r = 10, l = 5: the single-read narrow pass
    (SRHT X with r + l <= 16), launched as the benchmark's small-r entry is."""
    gn, A = full["gn"], full["A"]
    w = W.SRHT32K_R10
    p = gn.Problem(w.m, w.n, w.r, w.l, kind_x=w.kind_x, kind_y=w.kind_y, seed=w.seed,
                   mode=w.mode, eps=w.eps)
    ws = gn.workspace(p, gn.C.GN_OP_SKETCH)
    AX = torch.empty(w.m, w.r, dtype=torch.float32, device="cuda")
    YtA = torch.empty(p.rl, w.n, dtype=torch.float32, device="cuda")
    print("\n[full-size] r = 10 narrow pass", flush=True)
    gn.gn_sketch_prepare(p, ws, want_srht=True)
    gn.gn_sketch_pass(p, A, ws, AX=AX, YtA=YtA)
    torch.cuda.synchronize()
    return dict(w=w, p=p, A=A, AX=AX, YtA=YtA, X=OP.srht_matrix(w.seed, w.n, w.r))


def test_full_r10_narrow_pass(full_r10):
    w, p, A, X = full_r10["w"], full_r10["p"], full_r10["A"], full_r10["X"]
    rng = np.random.default_rng(9)
    rows = np.unique(np.concatenate([[0, 3, 4, 1023, 1024, w.m - 5, w.m - 1],
                                     rng.integers(0, w.m, 25)]))
    Ar = host(A.index_select(0, torch.from_numpy(rows).cuda()))
    ref = Ar @ X
    got = host(full_r10["AX"].index_select(0, torch.from_numpy(rows).cuda()))
    assert np.all(np.abs(got - ref) <= gamma(w.n) * (np.abs(Ar) @ np.abs(X)))
    e_ax = relerr(got, ref)
    # every row of Y^T A (all r + l = 15), summed over row blocks of A on the host
    Y = OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, p.rl), "f32")
    ref = np.zeros((p.rl, w.n))
    mag = np.zeros((p.rl, w.n))
    step = 2048
    for i0 in range(0, w.m, step):
        Ab = host(A[i0:i0 + step])
        yb = Y[i0:i0 + step]
        ref += yb.T @ Ab
        mag += np.abs(yb).T @ np.abs(Ab)
    got = host(full_r10["YtA"])
    assert np.all(np.abs(got - ref) <= gamma(w.m) * mag)
    e_ya = relerr(got, ref)
    print(f"r = 10 narrow pass: AX sampled rows rel err {e_ax:.3e}, Y^T A rel err {e_ya:.3e}")
    assert e_ax <= 2e-5 and e_ya <= 2e-5


def test_full_core_properties(full):
    w, p, core, X = full["w"], full["p"], full["core"], full["X"]
    k, r = core.rank(), w.r
    assert (core.flags() & 3) == 0
    Q, R = host(core.Q1), host(core.R)
    assert Q.shape == (p.rl, r)
    assert np.all(np.tril(R, -1) == 0)
    d = np.diag(R)
    assert np.all(d >= 0)
    assert np.max(np.abs(Q.T @ Q - np.eye(r))) <= 1e-12
    # Q R against sampled columns of the core matrix (Y^T A) X
    rng = np.random.default_rng(9)
    cols = np.unique(np.concatenate([[0, 1, r - 1], rng.integers(0, r, 13)]))
    YA = host(full["YtA"])
    Cs = YA @ X[:, cols]
    assert relerr(Q @ R[:, cols], Cs) <= 1e-11
    # kept rank: the first diagonal entry below the threshold (Section 5.1.1)
    nx, ny = OG.nu_srht(p.n), OG.nu_gaussian(p.m, p.rl)
    tau = OG.threshold(p.eps, nx, ny)
    assert np.all(d[:k] >= tau)
    assert k == r or d[k] < tau
    print(f"core: kept rank {k} of {r}, tau {tau:.3e}, R diagonal {d[0]:.3e} .. {d[-1]:.3e}")
    if k < r:
        Q2, R2 = host(core.Q2)[:, :k], host(core.R2)[:k, :k]
        assert np.max(np.abs(Q2.T @ Q2 - np.eye(k))) <= 1e-12
        assert np.all(np.tril(R2, -1) == 0)
        assert relerr(Q2 @ R2, R[:k, :].T) <= 1e-12


def test_full_core_vs_oracle_core_right(full):
    """The whole core against the oracle's: C = (Y^T A) X formed by the oracle from
    the library's own Y^T A and the explicit SRHT matrix, its Householder QR with
    R_ii >= 0 and the truncation (Section 5.1.1)."""
    w, p, core, X = full["w"], full["p"], full["core"], full["X"]
    tau = OG.threshold(p.eps, OG.nu_srht(p.n), OG.nu_gaussian(p.m, p.rl))
    ref = OG.core_right(host(full["YtA"]), X, tau)
    R, Q = host(core.R), host(core.Q1)
    eR, eQ = relerr(R, ref.R), relerr(Q, ref.Q)
    print(f"core vs oracle core_right: R rel err {eR:.3e}, Q rel err {eQ:.3e}, "
          f"k {core.rank()} / {ref.k}")
    check_rank(core.rank(), ref.k, np.diag(ref.R), tau)
    assert eR <= 1e-12 and eQ <= 1e-12


@pytest.mark.timeout(900)
def test_full_error_vs_oracle(full):
    """eq. (4) at the benchmark's size: the FP32-pass solve's error is within 1.05x
    the FP64 oracle's on the same matrix (FP32 values), the same SRHT X and the
    same FP32-valued Y."""
    gn, w, p, core = full["gn"], full["w"], full["p"], full["core"]
    F, Gm = gn.gn_factors(p, full["AX"], full["YtA"], core)
    e_gpu = math.sqrt(float(gn.gn_residual(full["A"], F, Gm).item()))
    del F, Gm
    torch.cuda.empty_cache()
    print("\n[full-size] FP64 oracle solve on the host", flush=True)
    A64 = full["A"].cpu().numpy().astype(np.float64)
    Y = OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, p.rl, workers=host_threads()), "f32")
    tau = OG.threshold(p.eps, OG.nu_srht(p.n), OG.nu_gaussian(p.m, p.rl))
    e_ref, ref = oracle_error(A64, full["X"], Y, tau)
    na = float(np.linalg.norm(A64))
    print(f"error: GPU {e_gpu / na:.6e}, oracle {e_ref / na:.6e}, ratio {e_gpu / e_ref:.6f}, "
          f"k {core.rank()} / {ref.core.k}")
    check_rank(core.rank(), ref.core.k, np.diag(ref.core.R), tau)
    assert e_gpu <= 1.05 * e_ref


def test_full_apply_sampled_rows(full):
    p, core = full["p"], full["core"]
    k, r = core.rank(), p.r
    Q, R = host(core.Q1), host(core.R)
    YA, Wr = host(full["YtA"]), full["Wr"]
    t = Q[:, :k].T @ (YA @ Wr)                   # Q_1^T (Y^T A W), k x 16
    rng = np.random.default_rng(10)
    rows = np.unique(np.concatenate([[0, p.m - 1], rng.integers(0, p.m, 30)]))
    rt = torch.from_numpy(rows).cuda()
    AXr = host(full["AX"].index_select(0, rt))
    if k == r:
        ref = AXr @ sla.solve_triangular(R, t, lower=False)
    else:
        Q2, R2 = host(core.Q2)[:, :k], host(core.R2)[:k, :k]
        ref = (AXr @ Q2) @ sla.solve_triangular(R2, t, trans="T", lower=False)
    got = host(full["out"].index_select(0, rt))
    e = relerr(got, ref)
    print(f"apply sampled rows: rel err {e:.3e}")
    assert e <= 1e-12


# ----------------------------------------------------------------------------- BF16 precision variant
# The same spectrum-controlled 32768 x 32768 matrix stored in bfloat16 with
# power-of-two scales per 128 x 128 block, Gaussian X and Y in bfloat16
# (r = 2000, l = 1000), FP32 accumulation, the core product on the BF16 matrix
# cores, as the benchmark's BF16 solve runs it.  Products of bfloat16 values are
# exact in FP32 and the block scales are powers of two, so every entry of AX and
# Y^T A obeys the FP32 inner-product bound against the dequantized matrix.  The
# core matrix Y^T (AX) takes AX in two bfloat16 terms (at most 2^-17 relative per
# entry) with FP32 accumulation: rows of Q R within 5e-5 of Y^T AX in FP64.
@pytest.fixture(scope="module")
def full_bf16():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    w = W.BF16_32K
    print(f"\n[full-size] {w.name}: generating A on the device", flush=True)
    A32 = W.device_matrix(W.F32_32K)
    bits, scales = gn.gn_quantize_bf16_bs(A32)
    p = gn.Problem(w.m, w.n, w.r, w.l, kind_x=w.kind_x, kind_y=w.kind_y, seed=w.seed,
                   mode=w.mode, eps=w.eps)
    ws = gn.workspace(p, gn.C.GN_OP_SKETCH)
    ws_core = gn.workspace(p, gn.C.GN_OP_CORE)
    AX = torch.empty(w.m, w.r, dtype=torch.float32, device="cuda")
    YtA = torch.empty(p.rl, w.n, dtype=torch.float32, device="cuda")
    core = gn.new_core(p)
    Wr = W.host_gaussian(w.n, 16, 98)
    out = torch.empty(w.m, 16, dtype=torch.float64, device="cuda")
    print("[full-size] BF16 prepare, pass, core, apply", flush=True)
    gn.gn_sketch_prepare(p, ws)
    gn.gn_sketch_pass(p, bits, ws, scales=scales, AX=AX, YtA=YtA)
    gn.gn_core(p, AX, out=core, ws=ws_core, YtA=YtA)
    gn.gn_apply(p, 0, AX, YtA, core, torch.from_numpy(Wr).cuda(), out=out)
    torch.cuda.synchronize()
    return dict(w=w, p=p, A32=A32, bits=bits, scales=scales, AX=AX, YtA=YtA, core=core,
                Wr=Wr, out=out)


def _bits_host(t):
    return t.view(torch.int16).cpu().numpy().view(np.uint16)


def test_full_bf16_quantization_sampled_blocks(full_bf16):
    A32, bits, scales = full_bf16["A32"], full_bf16["bits"], full_bf16["scales"]
    nb = scales.shape[0]
    sc = scales.cpu().numpy()
    for bi, bj in ((0, 0), (nb - 1, nb - 1), (17, 200), (255, 3), (100, 100)):
        blk = host(A32[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128])
        rb, rs = OG.block_quantize_bf16(blk)
        got = _bits_host(bits[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128])
        assert np.array_equal(got, rb), (bi, bj)
        assert sc[bi, bj] == rs[0, 0], (bi, bj)


def test_full_bf16_pass_sampled(full_bf16):
    w, p = full_bf16["w"], full_bf16["p"]
    rng = np.random.default_rng(11)
    cols = np.unique(np.concatenate([[0, 1, 255, 256, w.r - 1], rng.integers(0, w.r, 11)]))
    sel = np.unique(np.concatenate([[0, 1, 255, 256, 2047, 2048, p.rl - 1],
                                    rng.integers(0, p.rl, 9)]))
    Xs = np.concatenate([OG.round_mode(OP.gaussian(w.seed, OP.STREAM_X, w.n, 1, col0=int(c)), "bf16")
                         for c in cols], axis=1)
    Ys = np.concatenate([OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, 1, col0=int(a)), "bf16")
                         for a in sel], axis=1)
    sc = full_bf16["scales"].cpu().numpy()
    ax_ref = np.zeros((w.m, len(cols)))
    ax_mag = np.zeros((w.m, len(cols)))
    ya_ref = np.zeros((len(sel), w.n))
    ya_mag = np.zeros((len(sel), w.n))
    step = 2048
    for i0 in range(0, w.m, step):
        Ab = OG.block_dequantize_bf16(_bits_host(full_bf16["bits"][i0:i0 + step]),
                                      sc[i0 // 128:(i0 + step) // 128])
        ax_ref[i0:i0 + step] = Ab @ Xs
        ax_mag[i0:i0 + step] = np.abs(Ab) @ np.abs(Xs)
        yb = Ys[i0:i0 + step]
        ya_ref += yb.T @ Ab
        ya_mag += np.abs(yb).T @ np.abs(Ab)
    ax = host(full_bf16["AX"].index_select(1, torch.from_numpy(cols).cuda()))
    ya = host(full_bf16["YtA"].index_select(0, torch.from_numpy(sel).cuda()))
    assert np.all(np.abs(ax - ax_ref) <= gamma(w.n) * ax_mag)
    assert np.all(np.abs(ya - ya_ref) <= gamma(w.m) * ya_mag)
    e_ax, e_ya = relerr(ax, ax_ref), relerr(ya, ya_ref)
    print(f"BF16 AX sampled columns: rel err {e_ax:.3e}; Y^T A sampled rows: rel err {e_ya:.3e}")
    assert e_ax <= 2e-5 and e_ya <= 2e-5


def test_full_bf16_core_and_apply(full_bf16):
    w, p, core = full_bf16["w"], full_bf16["p"], full_bf16["core"]
    k, r = core.rank(), w.r
    assert (core.flags() & 3) == 0
    Q, R = host(core.Q1), host(core.R)
    assert np.all(np.tril(R, -1) == 0)
    d = np.diag(R)
    assert np.all(d >= 0)
    assert np.max(np.abs(Q.T @ Q - np.eye(r))) <= 1e-12
    rng = np.random.default_rng(12)
    sel = np.unique(np.concatenate([[0, p.rl - 1], rng.integers(0, p.rl, 14)]))
    Ys = np.concatenate([OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, 1, col0=int(a)), "bf16")
                         for a in sel], axis=1)
    AXh = host(full_bf16["AX"])
    e_c = relerr(Q[sel] @ R, Ys.T @ AXh)
    tau = OG.threshold(p.eps, OG.nu_gaussian(p.n, p.r), OG.nu_gaussian(p.m, p.rl))
    print(f"BF16 core: rows of QR vs Y^T AX rel err {e_c:.3e}; kept rank {k} of {r}, "
          f"tau {tau:.3e}, R diagonal {d[0]:.3e} .. {d[-1]:.3e}")
    assert e_c <= 5e-5
    assert np.all(d[:k] >= tau)
    assert k == r or d[k] < tau
    YA, Wr = host(full_bf16["YtA"]), full_bf16["Wr"]
    t = Q[:, :k].T @ (YA @ Wr)
    rows = np.unique(np.concatenate([[0, p.m - 1], rng.integers(0, p.m, 30)]))
    AXr = AXh[rows]
    if k == r:
        ref = AXr @ sla.solve_triangular(R, t, lower=False)
    else:
        Q2, R2 = host(core.Q2)[:, :k], host(core.R2)[:k, :k]
        assert relerr(Q2 @ R2, R[:k, :].T) <= 1e-12
        ref = (AXr @ Q2) @ sla.solve_triangular(R2, t, trans="T", lower=False)
    e = relerr(host(full_bf16["out"].index_select(0, torch.from_numpy(rows).cuda())), ref)
    print(f"BF16 apply sampled rows: rel err {e:.3e}")
    assert e <= 1e-12


@pytest.mark.timeout(900)
def test_full_bf16_error_vs_oracle(full_bf16):
    """eq. (4) for the BF16 variant, measured against the unquantized matrix: the
    FP64 oracle runs GN on the FP32 matrix with the same bfloat16-valued X and Y
    (the storage error of A is then part of the BF16 solve's error only), and the
    BF16 solve's ||A - A_hat||_F is within 1.05x the oracle's."""
    from paper_2009_11392_amd import gn
    w, p, core = full_bf16["w"], full_bf16["p"], full_bf16["core"]
    F, Gm = gn.gn_factors(p, full_bf16["AX"], full_bf16["YtA"], core)
    e_gpu = math.sqrt(float(gn.gn_residual(full_bf16["A32"], F, Gm).item()))
    del F, Gm
    torch.cuda.empty_cache()
    print("\n[full-size] FP64 oracle solve (bfloat16 sketch values) on the host", flush=True)
    A64 = full_bf16["A32"].cpu().numpy().astype(np.float64)
    X, Y = OG.gaussian_sketches(w.seed, w.m, w.n, w.r, w.l, mode="bf16", workers=host_threads())
    tau = OG.threshold(p.eps, OG.nu_gaussian(p.n, p.r), OG.nu_gaussian(p.m, p.rl))
    e_ref, ref = oracle_error(A64, X, Y, tau)
    na = float(np.linalg.norm(A64))
    print(f"BF16 error: GPU {e_gpu / na:.6e}, oracle {e_ref / na:.6e}, ratio {e_gpu / e_ref:.6f}, "
          f"k {core.rank()} / {ref.core.k}")
    check_rank(core.rank(), ref.core.k, np.diag(ref.core.R), tau)
    assert e_gpu <= 1.05 * e_ref


# ----------------------------------------------------------------------------- binary16 variant
# The same matrix stored as IEEE binary16 with the same power-of-two 128 x 128
# block scales (which keep the small entries out of the binary16 subnormal range),
# Gaussian X and Y in binary16 (r = 2000, l = 1000), FP32 accumulation; the core
# product on the FP32 matrix cores with Y's binary16 values.
@pytest.fixture(scope="module")
def full_f16(full_bf16):
    from paper_2009_11392_amd import gn
    w = W.F16_32K
    A32 = full_bf16["A32"]
    bits, scales = gn.gn_quantize_f16_bs(A32)
    p = gn.Problem(w.m, w.n, w.r, w.l, kind_x=w.kind_x, kind_y=w.kind_y, seed=w.seed,
                   mode=w.mode, eps=w.eps)
    ws = gn.workspace(p, gn.C.GN_OP_SKETCH)
    ws_core = gn.workspace(p, gn.C.GN_OP_CORE)
    AX = torch.empty(w.m, w.r, dtype=torch.float32, device="cuda")
    YtA = torch.empty(p.rl, w.n, dtype=torch.float32, device="cuda")
    core = gn.new_core(p)
    print("\n[full-size] binary16 prepare, pass, core", flush=True)
    gn.gn_sketch_prepare(p, ws)
    gn.gn_sketch_pass(p, bits, ws, scales=scales, AX=AX, YtA=YtA)
    gn.gn_core(p, AX, out=core, ws=ws_core, YtA=YtA)
    torch.cuda.synchronize()
    return dict(w=w, p=p, A32=A32, bits=bits, scales=scales, AX=AX, YtA=YtA, core=core)


def test_full_f16_quantization_sampled_blocks(full_f16):
    A32, bits, scales = full_f16["A32"], full_f16["bits"], full_f16["scales"]
    nb = scales.shape[0]
    sc = scales.cpu().numpy()
    for bi, bj in ((0, 0), (nb - 1, nb - 1), (17, 200), (255, 3), (100, 100)):
        blk = host(A32[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128])
        rb, rs = OG.block_quantize_f16(blk)
        got = _bits_host(bits[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128])
        assert np.array_equal(got, rb), (bi, bj)
        assert sc[bi, bj] == rs[0, 0], (bi, bj)


def test_full_f16_pass_sampled(full_f16):
    w, p = full_f16["w"], full_f16["p"]
    rng = np.random.default_rng(13)
    cols = np.unique(np.concatenate([[0, 1, 255, 256, w.r - 1], rng.integers(0, w.r, 11)]))
    sel = np.unique(np.concatenate([[0, 1, 255, 256, 2047, 2048, p.rl - 1],
                                    rng.integers(0, p.rl, 9)]))
    Xs = np.concatenate([OG.round_mode(OP.gaussian(w.seed, OP.STREAM_X, w.n, 1, col0=int(c)), "f16")
                         for c in cols], axis=1)
    Ys = np.concatenate([OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, 1, col0=int(a)), "f16")
                         for a in sel], axis=1)
    sc = full_f16["scales"].cpu().numpy()
    ax_ref = np.zeros((w.m, len(cols)))
    ax_mag = np.zeros((w.m, len(cols)))
    ya_ref = np.zeros((len(sel), w.n))
    ya_mag = np.zeros((len(sel), w.n))
    step = 2048
    for i0 in range(0, w.m, step):
        Ab = OG.block_dequantize_f16(_bits_host(full_f16["bits"][i0:i0 + step]),
                                     sc[i0 // 128:(i0 + step) // 128])
        ax_ref[i0:i0 + step] = Ab @ Xs
        ax_mag[i0:i0 + step] = np.abs(Ab) @ np.abs(Xs)
        yb = Ys[i0:i0 + step]
        ya_ref += yb.T @ Ab
        ya_mag += np.abs(yb).T @ np.abs(Ab)
    ax = host(full_f16["AX"].index_select(1, torch.from_numpy(cols).cuda()))
    ya = host(full_f16["YtA"].index_select(0, torch.from_numpy(sel).cuda()))
    assert np.all(np.abs(ax - ax_ref) <= gamma(w.n) * ax_mag)
    assert np.all(np.abs(ya - ya_ref) <= gamma(w.m) * ya_mag)
    e_ax, e_ya = relerr(ax, ax_ref), relerr(ya, ya_ref)
    print(f"binary16 AX sampled columns: rel err {e_ax:.3e}; Y^T A sampled rows: rel err {e_ya:.3e}")
    assert e_ax <= 2e-5 and e_ya <= 2e-5


@pytest.mark.timeout(900)
def test_full_f16_error_vs_oracle(full_f16):
    """eq. (4) for the binary16 variant, against the unquantized matrix: the FP64
    oracle runs GN on the FP32 matrix with the same binary16-valued X and Y."""
    from paper_2009_11392_amd import gn
    w, p, core = full_f16["w"], full_f16["p"], full_f16["core"]
    assert (core.flags() & 3) == 0
    F, Gm = gn.gn_factors(p, full_f16["AX"], full_f16["YtA"], core)
    e_gpu = math.sqrt(float(gn.gn_residual(full_f16["A32"], F, Gm).item()))
    del F, Gm
    torch.cuda.empty_cache()
    print("\n[full-size] FP64 oracle solve (binary16 sketch values) on the host", flush=True)
    A64 = full_f16["A32"].cpu().numpy().astype(np.float64)
    X, Y = OG.gaussian_sketches(w.seed, w.m, w.n, w.r, w.l, mode="f16", workers=host_threads())
    tau = OG.threshold(p.eps, OG.nu_gaussian(p.n, p.r), OG.nu_gaussian(p.m, p.rl))
    e_ref, ref = oracle_error(A64, X, Y, tau)
    na = float(np.linalg.norm(A64))
    print(f"binary16 error: GPU {e_gpu / na:.6e}, oracle {e_ref / na:.6e}, "
          f"ratio {e_gpu / e_ref:.6f}, k {core.rank()} / {ref.core.k}")
    check_rank(core.rank(), ref.core.k, np.diag(ref.core.R), tau)
    assert e_gpu <= 1.05 * e_ref
