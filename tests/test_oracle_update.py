"""Pins of the Section 6 updates (oracle/update.py) -- CPU only.

Each update of the sketch products is compared with a fresh sketch pass over the
enlarged or perturbed matrix with the enlarged sketches (drawn directly at the
enlarged size); the sketches themselves are checked to be prefix-stable in rows
and columns (Gaussian) and in the sample size (SRHT), which is what makes the
updates exact.
"""
import numpy as np

from oracle import gn as OG, philox as OP, update as OU

SEED = 31


def _A(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


def test_gaussian_sketches_are_prefix_stable():
    big = OP.gaussian(SEED, OP.STREAM_X, 70, 40)
    assert np.array_equal(OP.gaussian(SEED, OP.STREAM_X, 50, 23), big[:50, :23])
    assert np.array_equal(OP.gaussian(SEED, OP.STREAM_X, 20, 17, row0=50, col0=23),
                          big[50:, 23:])


def test_srht_sample_is_prefix_stable():
    assert np.array_equal(OP.srht_sample(SEED, 256, 40), OP.srht_sample(SEED, 256, 64)[:40])


def test_extend_rank_equals_fresh_pass():
    m, n, r, l, dr = 90, 70, 8, 4, 5
    A = _A(m, n, 1)
    l2 = (r + dr + 1) // 2
    X, Y = OP.gaussian(SEED, OP.STREAM_X, n, r), OP.gaussian(SEED, OP.STREAM_Y, m, r + l)
    AX, YA = OG.sketch_pass(A, X, Y)
    Xn = OP.gaussian(SEED, OP.STREAM_X, n, dr, col0=r)
    Yn = OP.gaussian(SEED, OP.STREAM_Y, m, r + dr + l2 - (r + l), col0=r + l)
    AX2, YA2 = OU.extend_rank(A, AX, YA, Xn, Yn)
    X2, Y2 = OP.gaussian(SEED, OP.STREAM_X, n, r + dr), OP.gaussian(SEED, OP.STREAM_Y, m, r + dr + l2)
    ref_ax, ref_ya = OG.sketch_pass(A, X2, Y2)
    assert np.allclose(AX2, ref_ax, rtol=0, atol=1e-12) and np.allclose(YA2, ref_ya, rtol=0, atol=1e-12)


def test_extend_rank_srht():
    m, n, r, dr = 60, 100, 6, 4
    A = _A(m, n, 2)
    X = OP.srht_matrix(SEED, n, r)
    X2 = OP.srht_matrix(SEED, n, r + dr)
    assert np.array_equal(X2[:, :r], X)
    Y = OP.gaussian(SEED, OP.STREAM_Y, m, r + 3)
    AX, _ = OG.sketch_pass(A, X, Y)
    AX2, _ = OU.extend_rank(A, AX, Y.T @ A, X2[:, r:], np.zeros((m, 0)))
    assert np.allclose(AX2, A @ X2, rtol=0, atol=1e-11)


def test_append_rows_equals_fresh_pass():
    m, mb, n, r, l = 80, 25, 60, 7, 4
    A, B = _A(m, n, 3), _A(mb, n, 4)
    X = OP.gaussian(SEED, OP.STREAM_X, n, r)
    Y = OP.gaussian(SEED, OP.STREAM_Y, m, r + l)
    Yb = OP.gaussian(SEED, OP.STREAM_Y, mb, r + l, row0=m)
    AX2, YA2 = OU.append_rows(A @ X, Y.T @ A, B, X, Yb)
    Y2 = OP.gaussian(SEED, OP.STREAM_Y, m + mb, r + l)
    ref_ax, ref_ya = OG.sketch_pass(np.vstack([A, B]), X, Y2)
    assert np.allclose(AX2, ref_ax, rtol=0, atol=1e-12) and np.allclose(YA2, ref_ya, rtol=0, atol=1e-12)
    # the core of the enlarged problem: Y^T A X + Y_B^T B X
    assert np.allclose(Y2.T @ AX2, Y.T @ (A @ X) + Yb.T @ (B @ X), rtol=0, atol=1e-11)


def test_append_cols_equals_fresh_pass():
    m, n, nb, r, l = 70, 50, 30, 6, 3
    A, B = _A(m, n, 5), _A(m, nb, 6)
    X = OP.gaussian(SEED, OP.STREAM_X, n, r)
    Xb = OP.gaussian(SEED, OP.STREAM_X, nb, r, row0=n)
    Y = OP.gaussian(SEED, OP.STREAM_Y, m, r + l)
    AX2, YA2 = OU.append_cols(A @ X, Y.T @ A, B, Xb, Y)
    ref_ax, ref_ya = OG.sketch_pass(np.hstack([A, B]), OP.gaussian(SEED, OP.STREAM_X, n + nb, r), Y)
    assert np.allclose(AX2, ref_ax, rtol=0, atol=1e-12) and np.allclose(YA2, ref_ya, rtol=0, atol=1e-12)


def test_perturbation_equals_fresh_pass():
    m, n, r, l = 64, 48, 5, 3
    A, E = _A(m, n, 7), 1e-3 * _A(m, n, 8)
    X = OP.gaussian(SEED, OP.STREAM_X, n, r)
    Y = OP.gaussian(SEED, OP.STREAM_Y, m, r + l)
    AX2, YA2 = OU.perturb(A @ X, Y.T @ A, E, X, Y)
    ref_ax, ref_ya = OG.sketch_pass(A + E, X, Y)
    assert np.allclose(AX2, ref_ax, rtol=0, atol=1e-12) and np.allclose(YA2, ref_ya, rtol=0, atol=1e-12)


def test_updated_approximant_recovers_appended_low_rank_matrix():
    """Exact recovery survives an append: rank([A; B]) = r gives A_hat = [A; B]."""
    rng = np.random.default_rng(9)
    m, mb, n, r, l = 60, 20, 40, 6, 3
    U = rng.standard_normal((m + mb, r))
    V = rng.standard_normal((n, r))
    Afull = U @ V.T
    A, B = Afull[:m], Afull[m:]
    X = OP.gaussian(SEED, OP.STREAM_X, n, r)
    Y = OP.gaussian(SEED, OP.STREAM_Y, m, r + l)
    Yb = OP.gaussian(SEED, OP.STREAM_Y, mb, r + l, row0=m)
    AX2, YA2 = OU.append_rows(A @ X, Y.T @ A, B, X, Yb)
    Y2 = np.vstack([Y, Yb])
    c = OG.core(AX2, Y2, 0.0)
    F, G = OG.factors(AX2, YA2, c)
    assert np.linalg.norm(F @ G - Afull) <= 1e-10 * np.linalg.norm(Afull)
