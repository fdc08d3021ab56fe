"""Pins of the oracle's reverse mode (oracle/grad.py) -- CPU only.

The gradient of L = <Gbar, A_hat> with the kept rank k held at its forward value
is checked against
  * central finite differences of the oracle's own forward map in FP64, in random
    directions and entry by entry, for k = r and for two kinds of truncation
    (rank-deficient A, and full-rank A with a spectral gap below the threshold);
  * torch's FP64 autograd through an independent torch forward of the same map
    (torch's QR and linear-solve adjoints; the pseudoinverse of R_1 written as
    R_1^T (R_1 R_1^T)^-1), on the FD sizes and on a gradient-workload-shaped
    problem (sigma_i = i^-1.5, Gaussian X and Y).
"""
import numpy as np
import pytest
import torch

from oracle import gn as OG, grad as OGR

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _problem(m, n, r, l, sig, seed):
    rng = np.random.default_rng(seed)
    k = len(sig)
    U, _ = np.linalg.qr(rng.standard_normal((m, k)))
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    A = (U * np.asarray(sig)) @ V.T
    X = rng.standard_normal((n, r))
    Y = rng.standard_normal((m, r + l))
    Gb = rng.standard_normal((m, n))
    return A, X, Y, Gb, rng


CASES = {
    # name: (m, n, r, l, sigma, tau, expected k)
    "full_rank": (64, 32, 4, 2, np.linspace(1.0, 0.3, 32), 0.0, 4),
    "rank_deficient": (64, 32, 4, 2, np.linspace(1.0, 0.3, 3), 4e-5, 3),
    "gap": (64, 32, 6, 3, np.r_[1.0, 0.8, 0.6, 0.5, 1e-4 * np.ones(28)], 1e-2, 4),
}


@pytest.fixture(params=sorted(CASES))
def case(request):
    m, n, r, l, sig, tau, kexp = CASES[request.param]
    A, X, Y, Gb, rng = _problem(m, n, r, l, sig, seed=sorted(CASES).index(request.param) + 11)
    c = OG.gn(A, X, Y, tau).core
    assert c.k == kexp
    return A, X, Y, Gb, c, rng


def _fd(A, X, Y, k, Gb, E, h=1e-6):
    return (OGR.loss_fixed_rank(A + h * E, X, Y, k, Gb)
            - OGR.loss_fixed_rank(A - h * E, X, Y, k, Gb)) / (2 * h)


def test_directional_finite_differences(case):
    A, X, Y, Gb, c, rng = case
    dA = OGR.gn_backward(A, X, Y, c, Gb)
    for _ in range(4):
        E = rng.standard_normal(A.shape)
        fd = _fd(A, X, Y, c.k, Gb, E)
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * np.linalg.norm(dA))


def test_entrywise_finite_differences(case):
    A, X, Y, Gb, c, rng = case
    dA = OGR.gn_backward(A, X, Y, c, Gb)
    scale = np.abs(dA).max()
    for _ in range(6):
        i, j = rng.integers(A.shape[0]), rng.integers(A.shape[1])
        E = np.zeros_like(A)
        E[i, j] = 1.0
        assert abs(_fd(A, X, Y, c.k, Gb, E) - dA[i, j]) <= 1e-6 * scale


def _torch_grad(A, X, Y, k, Gb):
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    Xt, Yt, Gt = (torch.tensor(v, dtype=torch.float64) for v in (X, Y, Gb))
    P = At @ Xt
    S = Yt.T @ At
    C = Yt.T @ P
    Q1, _ = torch.linalg.qr(C[:, :k])
    R1 = Q1.T @ C
    M = R1.T @ torch.linalg.solve(R1 @ R1.T, Q1.T)
    L = (Gt * (P @ M @ S)).sum()
    L.backward()
    return At.grad.numpy()


def test_matches_torch_autograd(case):
    A, X, Y, Gb, c, _ = case
    dA = OGR.gn_backward(A, X, Y, c, Gb)
    ref = _torch_grad(A, X, Y, c.k, Gb)
    assert np.linalg.norm(dA - ref) <= 1e-9 * np.linalg.norm(ref)


def test_matches_torch_autograd_gradient_workload_shape():
    """sigma_i = i^-1.5, Gaussian sketches, r = 20, l = 10 (the gradient workload's
    recipe at a size the CPU handles in well under a second)."""
    sig = np.arange(1, 101, dtype=float) ** -1.5
    A, X, Y, Gb, _ = _problem(200, 100, 20, 10, sig, seed=5)
    c = OG.gn(A, X, Y, 10 * 2.0 ** -53 * OG.nu_gaussian(100, 20) * OG.nu_gaussian(200, 30)).core
    assert c.k == 20
    dA = OGR.gn_backward(A, X, Y, c, Gb)
    ref = _torch_grad(A, X, Y, c.k, Gb)
    assert np.linalg.norm(dA - ref) <= 1e-9 * np.linalg.norm(ref)


def test_stored_sketch_products_give_the_same_gradient(case):
    A, X, Y, Gb, c, _ = case
    d1 = OGR.gn_backward(A, X, Y, c, Gb)
    d2 = OGR.gn_backward(A, X, Y, c, Gb, AX=A @ X, YA=Y.T @ A)
    assert np.array_equal(d1, d2)


def test_truncated_core_pinv_matches_svd_definition():
    """M = R_1^+ Q_1^T equals the pseudoinverse of the rank-k matrix Q_1 R_1."""
    A, X, Y, Gb, rng = _problem(64, 32, 6, 3, np.r_[1.0, 0.8, 0.6, 0.5, 1e-4 * np.ones(28)], 7)
    c = OG.gn(A, X, Y, 1e-2).core
    assert c.k == 4
    B = c.Q[:, :c.k] @ c.R[:c.k, :]
    assert np.linalg.norm(OGR.core_pinv(c) - np.linalg.pinv(B, rcond=1e-10)) <= \
        1e-10 * np.linalg.norm(np.linalg.pinv(B, rcond=1e-10))


def test_all_entries_finite_differences_64x32():
    """Every entry of dL/dA at 64 x 32, r = 4, l = 2 against central differences
    with h = u^(1/3) ||A||_2 (the finite-difference check of the gradient
    workload's recipe at its test size)."""
    A, X, Y, Gb, _ = _problem(64, 32, 4, 2, np.arange(1, 33, dtype=float) ** -1.5, seed=21)
    c = OG.gn(A, X, Y, 0.0).core
    assert c.k == 4
    dA = OGR.gn_backward(A, X, Y, c, Gb)
    h = (2.0 ** -53) ** (1.0 / 3.0) * np.linalg.norm(A, 2)
    fd = np.empty_like(A)
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            E = np.zeros_like(A)
            E[i, j] = h
            fd[i, j] = (OGR.loss_fixed_rank(A + E, X, Y, 4, Gb)
                        - OGR.loss_fixed_rank(A - E, X, Y, 4, Gb)) / (2 * h)
    assert np.linalg.norm(fd - dA) <= 1e-7 * np.linalg.norm(dA)
