"""CPU pins for the oracle's random sketches (no GPU).

The paper only requires i.i.d. zero-mean unit-variance Gaussian sketches
(Section 3.1) or an SRHT (Section 1); these tests check exactly those properties
of the oracle's generator, plus the closed form of the Sylvester-Hadamard matrix
against scipy.linalg.hadamard and the bfloat16 rounding against torch.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as st

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_known_answer_vectors():
    """The raw Philox4x32-10 words against the generator's published known-answer
    vectors (Random123, SC'11): a wrong multiplier, Weyl constant, word order or
    round count changes every output word."""
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for case in kat["cases"]:
        c = [int(x, 16) for x in case["counter"]]
        k0, k1 = (int(x, 16) for x in case["key"])
        got = philox.philox4x32_10(c[0], c[1], c[2], c[3], (k1 << 32) | k0)
        assert [int(w) for w in got] == [int(x, 16) for x in case["output"]], case
    # vectorized: the same blocks in one call, in a different order
    cs = np.array([[int(x, 16) for x in c["counter"]] for c in kat["cases"]][::-1], dtype=np.uint64)
    for i, case in enumerate(kat["cases"][::-1]):
        k0, k1 = (int(x, 16) for x in case["key"])
        got = philox.philox4x32_10(cs[i:i + 1, 0], cs[i:i + 1, 1], cs[i:i + 1, 2], cs[i:i + 1, 3],
                                   (k1 << 32) | k0)
        assert [int(w[0]) for w in got] == [int(x, 16) for x in case["output"]]


def test_gaussian_moments_and_ks():
    z = philox.gaussian(12345, philox.STREAM_Y, 1000, 1000).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    # third and fourth moments of N(0,1): 0 and 3
    assert abs(np.mean(z ** 3)) < 5 * np.sqrt(15.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 5 * np.sqrt(96.0 / n)
    assert st.kstest(z, "norm").pvalue > 1e-4


def test_gaussian_pairs_and_neighbours_uncorrelated():
    Z = philox.gaussian(7, philox.STREAM_X, 2000, 256)
    n = Z[:, 0::2].size
    for a, b in ((Z[:, 0::2], Z[:, 1::2]),          # z0 vs z1 of the same block
                 (Z[:-1], Z[1:]),                      # adjacent rows
                 (Z[:, :-2], Z[:, 2:])):               # adjacent blocks
        c = np.corrcoef(a.ravel(), b.ravel())[0, 1]
        assert abs(c) < 5 / np.sqrt(n)


def test_streams_and_seeds_differ():
    a = philox.gaussian(1, 1, 64, 64)
    assert not np.array_equal(a, philox.gaussian(1, 2, 64, 64))
    assert not np.array_equal(a, philox.gaussian(2, 1, 64, 64))
    assert not np.array_equal(a, philox.gaussian(1 + (1 << 32), 1, 64, 64))


def test_gaussian_prefix_stable_and_offsets():
    big = philox.gaussian(99, philox.STREAM_Y, 300, 77)
    assert np.array_equal(philox.gaussian(99, philox.STREAM_Y, 100, 50), big[:100, :50])
    assert np.array_equal(philox.gaussian(99, philox.STREAM_Y, 40, 31, row0=17, col0=5),
                          big[17:57, 5:36])


def test_philox_avalanche_and_distinct():
    c = np.arange(1 << 16, dtype=np.uint64)
    w = np.stack(philox.philox4x32_10(c, 0, 0, 0, 42), -1)
    flat = w.view(np.uint8).reshape(len(c), -1)
    assert len(np.unique(flat, axis=0)) == len(c)
    # flipping one counter bit changes about half of the 128 output bits
    w2 = np.stack(philox.philox4x32_10(c ^ np.uint64(1 << 7), 0, 0, 0, 42), -1)
    diff = np.unpackbits((w ^ w2).view(np.uint8)).reshape(len(c), -1).sum(1)
    assert abs(diff.mean() - 64) < 1.0
    bits = np.unpackbits(w.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 5 * 0.5 / np.sqrt(bits.size)


def test_uniforms_in_range():
    i = np.arange(4096, dtype=np.uint64)
    w = philox.philox4x32_10(i, 3, 1, 0, 5)
    z0, z1 = philox.box_muller(*w)
    assert np.all(np.isfinite(z0)) and np.all(np.isfinite(z1))
    # radius^2 = z0^2 + z1^2 is Exp(1/2)-distributed: mean 2
    assert abs(np.mean(z0 ** 2 + z1 ** 2) - 2.0) < 0.2


def test_bf16_rounding_ties_and_torch():
    one = 1.0
    ties = np.array([one + 2 ** -8, one + 3 * 2 ** -8, -(one + 2 ** -8), 3.0 + 2 ** -7])
    expect = np.array([1.0, one + 2 ** -6, -1.0, 3.0])
    assert np.array_equal(philox.round_bf16(ties), expect)
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x32 = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-8, 3, 100000)).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(philox.round_bf16_bits(x32.astype(np.float64)), ref)


def test_srht_signs_balanced():
    d = philox.srht_signs(3, 1 << 16)
    assert set(np.unique(d)) == {-1, 1}
    assert abs(d.astype(np.float64).mean()) < 5 / np.sqrt(d.size)
    assert np.array_equal(philox.srht_signs(3, 1000), d[:1000])


def test_srht_sample_distinct_sorted_prefix():
    npad, r = 4096, 1000
    idx = philox.srht_sample(11, npad, r)
    assert len(np.unique(idx)) == r and idx.min() >= 0 and idx.max() < npad
    keys = philox.srht_keys(11, npad)
    assert np.all(np.diff(keys[idx].astype(np.float64)) >= 0)
    assert np.all(keys[idx].max() <= np.delete(keys, idx).min())
    assert np.array_equal(philox.srht_sample(11, npad, 300), idx[:300])


def test_srht_matches_scipy_hadamard():
    for n, r in ((64, 10), (100, 17), (512, 512)):
        npad = philox.next_pow2(n)
        H = sla.hadamard(npad).astype(np.float64)
        d = philox.srht_signs(5, npad)[:n].astype(np.float64)
        idx = philox.srht_sample(5, npad, r)
        X = philox.srht_matrix(5, n, r)
        assert np.array_equal(X, d[:, None] * H[:n, idx])
    X = philox.srht_matrix(9, 256, 256)
    assert np.array_equal(X.T @ X, 256.0 * np.eye(256))


def _half_values():
    """Every finite non-negative binary16 value, exactly, built from its
    definition: (m / 1024) 2^-14 for the subnormals, (1 + m / 1024) 2^(e-15)
    for biased exponents e = 1..30."""
    from fractions import Fraction
    vals = [Fraction(m, 1024) * Fraction(1, 2 ** 14) for m in range(1024)]
    for e in range(1, 31):
        vals += [(1 + Fraction(m, 1024)) * Fraction(2) ** (e - 15) for m in range(1024)]
    return vals


def test_f16_rounding_brute_force():
    """round_f16 (one-step double -> binary16, nearest-even) against a brute-force
    search over every binary16 value in exact rational arithmetic: random doubles
    across the normal and subnormal ranges, exact ties (half-way points), points
    one double away from a tie, and the overflow threshold."""
    from fractions import Fraction
    vals = _half_values()
    rng = np.random.default_rng(5)
    xs = list(rng.standard_normal(300) * 10.0 ** rng.uniform(-9, 4.5, 300))
    for k in (3, 517, 1023, 1024, 1500, 20000, 30000):            # ties between neighbours
        a, b = vals[k], vals[k + 1]
        mid = float((a + b) / 2)
        xs += [mid, np.nextafter(mid, np.inf), np.nextafter(mid, -np.inf)]
    xs += [65504.0, 65519.99, 2.0 ** -24 * 0.5, 2.0 ** -24 * 1.5, 2.0 ** -25 + 2.0 ** -60]
    import bisect
    got = philox.round_f16(np.array(xs))
    for x, g in zip(xs, got):
        ax = Fraction(abs(float(x)))
        if ax >= 65520:          # half-way from 65504 to the next (absent) value: infinity
            assert np.isinf(g)
            continue
        # nearest value; on a tie the one with an even last significand bit (the
        # index of a value in the list has the parity of its significand)
        j = bisect.bisect_left(vals, ax)
        cand = [t for t in (j - 1, j) if 0 <= t < len(vals)]
        i = min(cand, key=lambda t: (abs(vals[t] - ax), t % 2))
        want = float(vals[i]) * (1 if x >= 0 else -1)
        assert g == want, (x, g, want)
