"""Pins of the alternative core stabilizations and the plain-GN check
(oracle/stabilize.py, Sections 5.1.1 and 5.1.2) -- CPU only.

Cores are built from chosen factors (C = U diag(s) V^T, or C = Q R with a chosen
upper triangular R) through an orthonormal Y and AX = Y C, so that Y^T AX = C and
the expected approximant is written from the chosen factors, not from the
oracle's factorizations:
  S1  SVD route: kept rank and A_hat against the chosen singular triplets
  S2  SVD route = plain GN when no singular value is below tau; = the truncated
      QR route and exact recovery when rank(A) < r
  S3  perturbation (a): singular values raised to tau (closed form); inverse
      bounded by 1/tau
  S4  column-pivoted QR: C P = Q R, Q orthonormal, the pivoting inequalities; (b)
      equals plain GN when nothing is lifted and bounds the inverse after lifting
  S5  perturbation (c) against a chosen R; on Kahan's matrix (c) lifts nothing
      and leaves ||R^{-1}|| >> 1/tau while (a) gives exactly 1/tau
  S6  power method: never above ||T^{-1}||_2, converges with a gap
  S7  the check flags rank-deficient plain GN and not the well-conditioned
      workload; the checked solve then equals SGN
"""
import math

import numpy as np
import scipy.linalg as sla

from oracle import gn as G, philox, stabilize as S
from paper_2009_11392_amd import workloads as W


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _orth(rng, rows, cols):
    q, rr = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q * np.sign(np.diag(rr))


def _designed(C, m=90, n=70, seed=0):
    """AX, Y^T A, Y with Y^T AX = C (Y orthonormal) and a random Y^T A."""
    rng = np.random.default_rng(seed)
    rl, r = C.shape
    Y = _orth(rng, m, rl)
    AX = Y @ C
    YA = rng.standard_normal((rl, n))
    return AX, YA, Y


def _svd_core(r=12, rl=18, s=None, seed=1):
    rng = np.random.default_rng(seed)
    U = _orth(rng, rl, r)
    V = _orth(rng, r, r)
    return U, s, V, (U * s) @ V.T


TAU = 1e-6
S_VALUES = np.array([3.0, 1.0, 0.5, 0.2, 1e-2, 1e-3, 1e-4, 1e-5, 5e-7, 1e-8, 1e-10, 0.0])


# ----------------------------------------------------------------------------- S1
def test_s1_svd_route_closed_form():
    U, s, V, C = _svd_core(s=S_VALUES)
    AX, YA, Y = _designed(C)
    f = S.core_svd(AX, YA, Y, TAU)
    assert f.k == 8                                  # s >= 1e-6: the first eight
    ref = AX @ (V[:, :8] / s[:8]) @ U[:, :8].T @ YA
    assert relerr(f.approx, ref) <= 1e-10
    assert np.allclose(f.values[:8], s[:8], rtol=0, atol=1e-14 * s[0])   # absolute u ||C||


# ----------------------------------------------------------------------------- S2
def test_s2_svd_route_plain_when_nothing_small():
    w = W.SMALL
    A = W.host_matrix(w)
    X, Y = G.gaussian_sketches(1, w.m, w.n, w.r, w.l)
    AX, YA = A @ X, Y.T @ A
    f = S.core_svd(AX, YA, Y, 0.0)
    plain = G.gn(A, X, Y, 0.0)
    assert f.k == w.r == plain.core.k
    assert relerr(f.approx, plain.approx) <= 1e-9


def test_s2_svd_route_rank_deficient_recovery():
    w = W.SMALL
    X, Y = G.gaussian_sketches(1, w.m, w.n, w.r, w.l)
    A = W.spectrum_matrix(w.m, w.n, w.sigma()[:20], seed=8)
    tau = G.threshold(w.eps, G.nu_gaussian(w.n, w.r), G.nu_gaussian(w.m, w.r + w.l))
    f = S.core_svd(A @ X, Y.T @ A, Y, tau)
    q = G.gn(A, X, Y, tau)
    assert f.k == q.core.k == 20
    assert relerr(f.approx, A) <= 1e-10
    assert relerr(f.approx, q.approx) <= 1e-10


# ----------------------------------------------------------------------------- S3
def test_s3_lift_svd_closed_form():
    U, s, V, C = _svd_core(s=S_VALUES)
    AX, YA, Y = _designed(C)
    f = S.lift_svd(AX, YA, Y, TAU)
    sl = np.maximum(s, TAU)
    assert f.k == 12 and f.lifted == 4
    # the lifted directions enter with weight 1/tau: compare the exact factors
    ref = AX @ (V / sl) @ U.T @ YA
    assert relerr(f.approx, ref) <= 1e-8
    # ||(C')^+|| = 1 / max(s_min, tau) = 1 / tau
    Cl = (U * sl) @ V.T
    assert math.isclose(np.linalg.norm(np.linalg.pinv(Cl), 2), 1 / TAU, rel_tol=1e-6)


# ----------------------------------------------------------------------------- S4
def _scaled_cols(seed=3, rl=30, r=20, rank=None):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((rl, r))
    if rank is not None:
        B = rng.standard_normal((rl, rank)) @ rng.standard_normal((rank, r))
    return B * (3.0 ** -np.arange(r)[::-1])[None, :]   # last column largest


def test_s4_pivoted_qr_properties():
    C = _scaled_cols()
    Q, R, p = S.qr_pivoted(C)
    r = C.shape[1]
    assert sorted(p.tolist()) == list(range(r)) and p[0] == r - 1
    assert np.linalg.norm(C[:, p] - Q @ R) <= 1e-14 * np.linalg.norm(C)
    assert np.linalg.norm(Q.T @ Q - np.eye(r)) <= 1e-13
    assert np.allclose(np.tril(R, -1), 0)
    # each pivot dominates every trailing column at its stage
    for j in range(r):
        tails = np.linalg.norm(R[j:, j:], axis=0)
        assert abs(R[j, j]) >= tails.max() * (1 - 1e-12)


def test_s4_lift_rrqr_plain_and_bounded():
    C = _scaled_cols(r=12, rl=18)
    AX, YA, Y = _designed(C)
    f = S.lift_rrqr(AX, YA, Y, 1e-30)
    assert f.lifted == 0
    assert relerr(f.approx, AX @ np.linalg.pinv(C) @ YA) <= 1e-10
    # a rank-5 core: QRCP puts the five pivots first, the rest is lifted to tau
    Cd = _scaled_cols(seed=4, r=12, rl=18, rank=5)
    AXd, YAd, Yd = _designed(Cd)
    tau = 1e-9 * np.linalg.norm(Cd, 2)
    fd = S.lift_rrqr(AXd, YAd, Yd, tau)
    assert fd.lifted == 7
    _, R, _ = S.qr_pivoted(Cd)
    Rl, _ = S._lift_diagonal(R, tau)
    assert np.linalg.norm(sla.solve_triangular(Rl, np.eye(12)), 2) <= 12 / tau


# ----------------------------------------------------------------------------- S5
def test_s5_lift_diag_closed_form():
    rng = np.random.default_rng(5)
    rl, r = 18, 12
    Q = _orth(rng, rl, r)
    d = np.array([2.0, 1.5, 1.0, 0.7, 0.5, 0.3, 0.2, 1e-5, 1e-7, 1e-9, 1e-8, 3e-9])
    # rows graded with their diagonal, so the trailing rows are small as a whole
    R = np.triu(0.3 * d[:, None] * rng.standard_normal((r, r)), 1)
    R[np.diag_indices(r)] = d
    C = Q @ R
    AX, YA, Y = _designed(C)
    f = S.lift_diag(AX, YA, Y, TAU)
    assert f.lifted == 4
    Rl = R.copy()
    Rl[np.diag_indices(r)] = np.maximum(d, TAU)
    ref = AX @ np.linalg.inv(Rl) @ Q.T @ YA
    assert relerr(f.approx, ref) <= 1e-8
    assert np.allclose(f.values, d, rtol=1e-6, atol=1e-15)


def _kahan(r, theta):
    s, c = math.sin(theta), math.cos(theta)
    K = np.eye(r) - c * np.triu(np.ones((r, r)), 1)
    return (s ** np.arange(r))[:, None] * K


def test_s5_kahan_c_fails_a_holds():
    r, rl = 40, 50
    K = _kahan(r, 1.2)
    smin = np.linalg.svd(K, compute_uv=False)[-1]
    dmin = np.min(np.abs(np.diag(K)))
    tau = math.sqrt(smin * dmin)                     # between sigma_min and min |K_ii|
    assert smin * 100 < tau < dmin / 100
    rng = np.random.default_rng(6)
    C = _orth(rng, rl, r) @ K
    AX, YA, Y = _designed(C, m=120, n=60)
    fc = S.lift_diag(AX, YA, Y, tau)
    assert fc.lifted == 0                            # every |R_ii| >= tau: nothing changes
    Q, R = G._qr_nonneg(C)
    assert np.linalg.norm(sla.solve_triangular(R, np.eye(r)), 2) > 100 / tau
    fa = S.lift_svd(AX, YA, Y, tau)
    assert fa.lifted >= 1
    U, s, Vt = np.linalg.svd(C, full_matrices=False)
    Cl = (U * np.maximum(s, tau)) @ Vt
    assert math.isclose(np.linalg.norm(np.linalg.pinv(Cl), 2), 1 / tau, rel_tol=1e-6)


# ----------------------------------------------------------------------------- S6
def test_s6_power_method_bound_and_convergence():
    rng = np.random.default_rng(7)
    r = 60
    s = np.concatenate([np.logspace(0, -6, r - 1), [1e-8]])   # gap 100 at the bottom
    M = _orth(rng, 80, r) @ np.diag(s) @ _orth(rng, r, r).T
    _, T = G._qr_nonneg(M)
    true = 1.0 / s[-1]
    V0 = S.power_start(11, 8, r)
    for it in range(1, 6):
        est = S.inv_norm_power(T, V0, it)
        assert est <= true * (1 + 1e-9)
    assert S.inv_norm_power(T, V0, 3) >= 0.999 * true
    # no gap: random triangular factor, still a lower bound and within 2x
    T2 = np.triu(rng.standard_normal((r, r))) + 4 * np.eye(r)
    true2 = np.linalg.norm(np.linalg.inv(T2), 2)
    e2 = S.inv_norm_power(T2, V0, 6)
    assert true2 / 2 <= e2 <= true2 * (1 + 1e-9)
    # a diagonal factor: 1 / min |T_ii| once the iterates align
    D = np.diag(np.linspace(1.0, 2.0, r))
    D[5, 5] = 1e-3
    assert math.isclose(S.inv_norm_power(D, V0, 4), 1e3, rel_tol=1e-9)
    # a lower triangular factor: the same norm as its transpose
    assert math.isclose(S.inv_norm_power(T.T.copy(), V0, 3, lower=True), true, rel_tol=1e-3)
    assert S.power_start(11, 8, r).shape == (8, r)
    assert np.array_equal(S.power_start(11, 8, r), philox.gaussian(11, 6, 8, r))


# ----------------------------------------------------------------------------- S7
def test_s7_check_decides_on_both_sides():
    w = W.SMALL
    X, Y = G.gaussian_sketches(1, w.m, w.n, w.r, w.l)
    nx, ny = G.nu_gaussian(w.n, w.r), G.nu_gaussian(w.m, w.r + w.l)
    delta = w.eps
    # well conditioned: sigma_i = 0.9^i, r = 50
    A = W.host_matrix(w)
    res, est, flag = S.gn_checked(A, X, Y, delta, nx, ny, seed=3)
    assert not flag and est * delta * nx * ny < 1e-3
    assert res.core.k == w.r
    # rank 20 < r: plain GN's R has a noise-level tail
    Ad = W.spectrum_matrix(w.m, w.n, w.sigma()[:20], seed=8)
    plain = G.gn(Ad, X, Y, 0.0)
    est_d, flag_d = S.check(plain.core, delta, nx, ny, seed=3)
    assert flag_d and est_d * delta * nx * ny > 10
    # on the truncated core the applied factor R_2^T is bounded: no flag
    sgn = G.gn(Ad, X, Y, G.threshold(delta, nx, ny))
    est_t, flag_t = S.check(sgn.core, delta, nx, ny, seed=3)
    assert sgn.core.k == 20 and not flag_t and est_t * delta * nx * ny < 1
    res_d, _, flagged = S.gn_checked(Ad, X, Y, delta, nx, ny, seed=3)
    assert flagged and res_d.core.k == 20
    assert relerr(res_d.approx, Ad) <= 1e-10
