"""Pins of the oracle's counter-based Rademacher probes (Sec. 3.1; Alg. 2 probe sampling)."""

import os

import numpy as np

from oracle import probes


def test_splitmix64_published_outputs(golden_dir):
    vals = [int(l, 16) for l in open(os.path.join(golden_dir, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = probes.splitmix64(0, np.arange(1, 5, dtype=np.uint64))
    assert [int(v) for v in got] == vals


def _spec_scalar(seed, it, C, K, D, t, c, k, d):
    """The probe definition evaluated with Python integers, one entry at a time."""
    M = (1 << 64) - 1
    G = 0x9E3779B97F4A7C15

    def out(s, i):
        z = (s + i * G) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    key = out(seed, it + 1)
    W = (D + 63) // 64
    word = out(key, ((t * C + c) * K + k) * W + d // 64 + 1)
    return -1.0 if (word >> (d % 64)) & 1 else 1.0


def test_layout_matches_scalar_definition():
    seed, it, T, C, K, D = 7, 3, 3, 2, 4, 150          # ragged last word (150 = 2*64 + 22)
    P = probes.rademacher(seed, it, T, C, K, D)
    rng = np.random.default_rng(0)
    for _ in range(300):
        t, c, k, d = (int(v) for v in (rng.integers(T), rng.integers(C), rng.integers(K), rng.integers(D)))
        assert P[t, c, k, d] == _spec_scalar(seed, it, C, K, D, t, c, k, d)


def test_task_subset_equals_full():
    P = probes.rademacher(1, 0, 5, 2, 3, 70)
    Q = probes.rademacher(1, 0, 5, 2, 3, 70, t_sel=[4, 1])
    assert np.array_equal(Q, P[[4, 1]])


def test_rademacher_statistics():
    # entries are +-1, balanced, and distinct probes are uncorrelated (i.i.d. Rademacher)
    P = probes.rademacher(1, 0, 8, 4, 32, 1024)
    assert set(np.unique(P)) == {-1.0, 1.0}
    n = P.size
    assert abs(P.mean()) < 4.0 / np.sqrt(n)
    flat = P.reshape(-1, 1024)
    G = flat @ flat.T / 1024.0
    off = G[~np.eye(len(G), dtype=bool)]
    assert np.all(np.diag(G) == 1.0)
    assert abs(off.mean()) < 4.0 / np.sqrt(off.size * 1024)
    assert abs(off.std() - 1.0 / np.sqrt(1024)) < 0.05 / np.sqrt(1024) * 10


def test_fresh_per_iteration_and_pair():
    a = probes.rademacher(1, 0, 2, 2, 2, 256)
    b = probes.rademacher(1, 1, 2, 2, 2, 256)
    assert not np.array_equal(a, b)
    assert not np.array_equal(a[0, 0, 0], a[0, 1, 0])
    assert not np.array_equal(a[0, 0, 0], a[1, 0, 0])
