"""Section 6 updates on the GPU (gn_sketch_extend / _append / _update) -- needs a GPU.

Each updated AX and Y^T A is compared with the oracle's update formula and with a
fresh gn_sketch of the enlarged (or perturbed) problem; FP64 to 1e-13 relative,
FP32 entrywise within gamma_K of the magnitudes.  After an append, the full solve
from the updated sketches matches the oracle's approximant of the enlarged matrix.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import gn as OG, philox as OP, update as OU  # noqa: E402
from paper_2009_11392_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
SEED = 23


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    return gn


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().double().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _mat(m, n, seed):
    sig = np.arange(1, min(m, n) + 1, dtype=float) ** -1.0
    return W.spectrum_matrix(m, n, sig, seed=seed)


def _sketch(G, p, A):
    AX, YtA, _, _ = G.gn_sketch(p, A)
    return AX, YtA


def _X(p, rows=None, row0=0):
    if p.kind_x == "srht":
        return OP.srht_matrix(p.seed, p.n, p.r)
    return OP.gaussian(p.seed, OP.STREAM_X, rows or p.n, p.r, row0=row0)


@pytest.mark.parametrize("kind_x", ["gaussian", "srht"])
def test_extend_rank_f64(G, kind_x):
    m, n, r, dr = 300, 200, 20, 9
    A = _mat(m, n, 1)
    po = G.Problem(m, n, r, kind_x=kind_x, seed=SEED, mode="f64")
    pn = G.Problem(m, n, r + dr, kind_x=kind_x, seed=SEED, mode="f64")
    Ad = dev(A)
    AXo, YAo = _sketch(G, po, Ad)
    AX = torch.zeros(m, pn.r, dtype=torch.float64, device="cuda")
    YtA = torch.zeros(pn.rl, n, dtype=torch.float64, device="cuda")
    AX[:, :r] = AXo
    YtA[:po.rl] = YAo
    G.gn_sketch_extend(po, pn, Ad, AX, YtA)
    Xn = _X(pn)[:, r:]
    Yn = OP.gaussian(SEED, OP.STREAM_Y, m, pn.rl - po.rl, col0=po.rl)
    ref_ax, ref_ya = OU.extend_rank(A, host(AXo), host(YAo), Xn, Yn)
    assert relerr(host(AX), ref_ax) <= 1e-13 and relerr(host(YtA), ref_ya) <= 1e-13
    AXf, YAf = _sketch(G, pn, Ad)
    assert relerr(host(AX), host(AXf)) <= 1e-13 and relerr(host(YtA), host(YAf)) <= 1e-13


@pytest.mark.parametrize("kind_x", ["gaussian", "srht"])
def test_append_rows_then_solve_f64(G, kind_x):
    m, mb, n, r = 300, 57, 200, 16
    Afull = _mat(m + mb, n, 2)
    A, B = Afull[:m], Afull[m:]
    po = G.Problem(m, n, r, kind_x=kind_x, seed=SEED, mode="f64")
    pn = G.Problem(m + mb, n, r, kind_x=kind_x, seed=SEED, mode="f64")
    AXo, YAo = _sketch(G, po, dev(A))
    AX = torch.zeros(m + mb, r, dtype=torch.float64, device="cuda")
    AX[:m] = AXo
    YtA = YAo.clone()
    G.gn_sketch_append(pn, 0, m, dev(B), AX, YtA)
    X = _X(po)
    Yb = OP.gaussian(SEED, OP.STREAM_Y, mb, pn.rl, row0=m)
    ref_ax, ref_ya = OU.append_rows(host(AXo), host(YAo), B, X, Yb)
    assert relerr(host(AX), ref_ax) <= 1e-13 and relerr(host(YtA), ref_ya) <= 1e-13
    # the solve from the updated sketches is the solve of the enlarged matrix
    core = G.gn_core(pn, AX)
    Y2 = OP.gaussian(SEED, OP.STREAM_Y, m + mb, pn.rl)
    ref = OG.gn(Afull, _X(pn), Y2, 0.0)
    assert core.rank() == ref.core.k == r
    F, Gm = G.gn_factors(pn, AX, YtA, core)
    assert relerr(host(F) @ host(Gm), ref.approx) <= 1e-10


def test_append_cols_f64(G):
    m, n, nb, r = 260, 180, 45, 14
    Afull = _mat(m, n + nb, 3)
    A, B = Afull[:, :n], Afull[:, n:]
    po = G.Problem(m, n, r, seed=SEED, mode="f64")
    pn = G.Problem(m, n + nb, r, seed=SEED, mode="f64")
    AXo, YAo = _sketch(G, po, dev(A))
    AX = AXo.clone()
    YtA = torch.zeros(pn.rl, n + nb, dtype=torch.float64, device="cuda")
    YtA[:, :n] = YAo
    G.gn_sketch_append(pn, 1, n, dev(B), AX, YtA)
    Xb = OP.gaussian(SEED, OP.STREAM_X, nb, r, row0=n)
    Y = OP.gaussian(SEED, OP.STREAM_Y, m, pn.rl)
    ref_ax, ref_ya = OU.append_cols(host(AXo), host(YAo), B, Xb, Y)
    assert relerr(host(AX), ref_ax) <= 1e-13 and relerr(host(YtA), ref_ya) <= 1e-13
    AXf, YAf = _sketch(G, pn, dev(Afull))
    assert relerr(host(AX), host(AXf)) <= 1e-13 and relerr(host(YtA), host(YAf)) <= 1e-13


# the last two cases run the single-read narrow passes (FP32, r + l <= 16,
# n >= 1024; SRHT and Gaussian X) over E
@pytest.mark.parametrize("mode,kind_x,m,n,r", [("f64", "gaussian", 333, 250, 24),
                                               ("f64", "srht", 333, 250, 24),
                                               ("f32", "gaussian", 333, 250, 24),
                                               ("f32", "srht", 333, 250, 24),
                                               ("f32", "srht", 700, 2048, 10),
                                               ("f32", "gaussian", 700, 2048, 10)])
def test_perturbation_update(G, mode, kind_x, m, n, r):
    A = _mat(m, n, 4)
    E = 1e-3 * np.random.default_rng(5).standard_normal((m, n))
    dt = torch.float64 if mode == "f64" else torch.float32
    p = G.Problem(m, n, r, kind_x=kind_x, seed=SEED, mode=mode)
    AX, YtA = _sketch(G, p, dev(A, dt))
    G.gn_sketch_update(p, dev(E, dt), AX, YtA)
    if mode == "f64":
        AXf, YAf = _sketch(G, p, dev(A + E))
        assert relerr(host(AX), host(AXf)) <= 1e-13 and relerr(host(YtA), host(YAf)) <= 1e-13
    else:
        A32 = A.astype(np.float32).astype(np.float64)
        E32 = E.astype(np.float32).astype(np.float64)
        X = OG.round_mode(_X(p), "f32")
        Y = OG.round_mode(OP.gaussian(SEED, OP.STREAM_Y, m, p.rl), "f32")
        g = lambda K: 2 * K * U32 / (1 - 2 * K * U32)   # two accumulations and one add
        bax = g(n) * ((np.abs(A32) + np.abs(E32)) @ np.abs(X))
        bya = g(m) * (np.abs(Y.T) @ (np.abs(A32) + np.abs(E32)))
        assert np.all(np.abs(host(AX) - (A32 + E32) @ X) <= bax + 1e-30)
        assert np.all(np.abs(host(YtA) - Y.T @ (A32 + E32)) <= bya + 1e-30)


def _check_f32(AX, YtA, A32, X, Y, adds=1):
    """FP32 sketches against the exact products of the FP32-rounded operands:
    entrywise within the bound of `adds` + 1 accumulations."""
    g = lambda K: (adds + 1) * K * U32 / (1 - (adds + 1) * K * U32)
    m, n = A32.shape
    assert np.all(np.abs(host(AX) - A32 @ X) <= g(n) * (np.abs(A32) @ np.abs(X)) + 1e-30)
    assert np.all(np.abs(host(YtA) - Y.T @ A32) <= g(m) * (np.abs(Y.T) @ np.abs(A32)) + 1e-30)


def test_extend_rank_narrow_f32(G):
    """Section 6 rank extension through the narrow pass: r = 6 -> 10 (r + l = 9 -> 15)
    with an SRHT X on 2048 columns; the new columns and rows come from a pass of
    r = 4, r + l = 6 with the sample offset by the old r."""
    m, n, r, dr = 700, 2048, 6, 4
    A = _mat(m, n, 6)
    A32 = A.astype(np.float32).astype(np.float64)
    po = G.Problem(m, n, r, 3, kind_x="srht", seed=SEED, mode="f32")
    pn = G.Problem(m, n, r + dr, 5, kind_x="srht", seed=SEED, mode="f32")
    Ad = dev(A, torch.float32)
    AXo, YAo = _sketch(G, po, Ad)
    AX = torch.zeros(m, pn.r, dtype=torch.float32, device="cuda")
    YtA = torch.zeros(pn.rl, n, dtype=torch.float32, device="cuda")
    AX[:, :r] = AXo
    YtA[:po.rl] = YAo
    G.gn_sketch_extend(po, pn, Ad, AX, YtA)
    X = OG.round_mode(_X(pn), "f32")
    Y = OG.round_mode(OP.gaussian(SEED, OP.STREAM_Y, m, pn.rl), "f32")
    _check_f32(AX, YtA, A32, X, Y, adds=0)


def test_append_rows_narrow_f32(G):
    """Section 6 row append through the narrow pass: the new rows' AX and their
    Y^T B added to Y^T A (r = 10, l = 5, SRHT X on 2048 columns)."""
    m, mb, n, r = 600, 100, 2048, 10
    Afull = _mat(m + mb, n, 7)
    A32 = Afull.astype(np.float32).astype(np.float64)
    po = G.Problem(m, n, r, 5, kind_x="srht", seed=SEED, mode="f32")
    pn = G.Problem(m + mb, n, r, 5, kind_x="srht", seed=SEED, mode="f32")
    AXo, YAo = _sketch(G, po, dev(Afull[:m], torch.float32))
    AX = torch.zeros(m + mb, r, dtype=torch.float32, device="cuda")
    AX[:m] = AXo
    YtA = YAo.clone()
    G.gn_sketch_append(pn, 0, m, dev(Afull[m:], torch.float32), AX, YtA)
    X = OG.round_mode(_X(pn), "f32")
    Y = OG.round_mode(OP.gaussian(SEED, OP.STREAM_Y, m + mb, pn.rl), "f32")
    _check_f32(AX, YtA, A32, X, Y, adds=1)
