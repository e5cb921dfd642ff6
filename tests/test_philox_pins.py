"""Pins of the oracle's Philox4x32-10 twin: the generator's published
known-answer vectors, and statistical checks of the derived uniforms, normals
and signs (the GPU generator is compared with the twin bit for bit in the GPU
tests)."""
import os

import numpy as np

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_known_answer_vectors():
    """Counter (c0, c1, c2, c3) = (block lo, block hi, stream lo, stream hi),
    key (k0, k1) = (seed lo, seed hi): the published outputs, word for word."""
    rows = [line.split() for line in open(GOLDEN) if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        c0, c1, c2, c3, k0, k1, *out = (int(v, 16) for v in row)
        q = np.array([c0 | (c1 << 32)], dtype=np.uint64)
        got = philox.philox4x32_10(q, seed=k0 | (k1 << 32), stream=c2 | (c3 << 32))[0]
        assert [int(v) for v in got] == out


def test_uniform_words_chi_square():
    w = philox.philox4x32_10(np.arange(1 << 16, dtype=np.uint64), seed=12345, stream=7)
    u = w.astype(np.float64).ravel() / 2.0 ** 32
    counts, _ = np.histogram(u, bins=64, range=(0.0, 1.0))
    expected = u.size / 64
    chi2 = np.sum((counts - expected) ** 2 / expected)
    # 63 degrees of freedom: mean 63, sd ~11.2; 63 + 6 sd
    assert chi2 < 63 + 6 * np.sqrt(2 * 63)
    assert abs(u.mean() - 0.5) < 6 * np.sqrt(1 / 12 / u.size)


def test_normals_moments():
    z = philox.normal(seed=99, stream=1, n=1_000_001)
    n = z.size
    assert abs(z.mean()) < 6 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 6 * np.sqrt(2.0 / n)
    tail = np.mean(np.abs(z) > 1.959963984540054)
    assert abs(tail - 0.05) < 6 * np.sqrt(0.05 * 0.95 / n)
    kurt = np.mean(z ** 4)
    assert abs(kurt - 3.0) < 6 * np.sqrt(96.0 / n)
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.mean(z[0:-1:2] * z[1::2])) < 6 / np.sqrt(n / 2)


def test_rademacher_balanced_and_independent():
    a = philox.rademacher(seed=5, stream=3, n=200_003).astype(np.float64)
    b = philox.rademacher(seed=5, stream=4, n=200_003).astype(np.float64)
    c = philox.rademacher(seed=6, stream=3, n=200_003).astype(np.float64)
    n = a.size
    assert set(np.unique(a)) == {-1.0, 1.0}
    for v in (a, b, c):
        assert abs(v.mean()) < 6 / np.sqrt(n)
    assert abs(np.mean(a * b)) < 6 / np.sqrt(n)
    assert abs(np.mean(a * c)) < 6 / np.sqrt(n)
    assert abs(np.mean(a[:-1] * a[1:])) < 6 / np.sqrt(n)


def test_counter_avalanche():
    """Flipping one counter bit changes about half of the 128 output bits."""
    q = np.arange(4096, dtype=np.uint64) * np.uint64(2654435761)
    base = philox.philox4x32_10(q, seed=1, stream=0)
    for bit in (0, 13, 31, 40):
        flip = philox.philox4x32_10(q ^ np.uint64(1 << bit), seed=1, stream=0)
        diff = np.unpackbits((base ^ flip).view(np.uint8), axis=None).reshape(q.size, -1).sum(axis=1)
        assert abs(diff.mean() - 64.0) < 6 * np.sqrt(32.0 / q.size)


def test_layout_prefix_consistency():
    """A shorter request is a prefix of a longer one (element layout)."""
    z = philox.normal(3, 2, 1001)
    assert np.array_equal(philox.normal(3, 2, 10), z[:10])
    r = philox.rademacher(3, 2, 1000)
    assert np.array_equal(philox.rademacher(3, 2, 129), r[:129])
