"""Counter-based Rademacher probes (oracle side).  TEST INFRASTRUCTURE ONLY.

The method draws K fresh Rademacher probes (entries +1 or -1 with probability 1/2 each) for every
task t and cluster c in every EM iteration (Sec. 3.1; Alg. 2, "sample Rademacher probes").  Both the
oracle and the GPU library must see the same probes, so the draw is a pure function of
(seed, it, t, c, k, d).  Each side implements it independently from this definition:

* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
  the i-th output (i >= 1) of the generator seeded with s is mix(s + i * G mod 2^64) with
  G = 0x9E3779B97F4A7C15 and
      mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
              z ^= z >> 31      (all mod 2^64).
* The stream key of EM iteration ``it`` (0-based) is s_it = output(seed, it + 1).
* Probe k (0-based, k < K) of pair (t, c) over a signal of length D uses W = ceil(D / 64) words;
  word m is output(s_it, i + 1) with i = ((t * C + c) * K + k) * W + m.
* Entry d is +1 when bit (d mod 64) of word floor(d / 64) is 0, and -1 when it is 1.
"""

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _mix(z):
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def splitmix64(seed, i):
    """i-th output (i >= 1, scalar or array) of SplitMix64 seeded with ``seed``."""
    with np.errstate(over="ignore"):
        i = np.asarray(i, dtype=np.uint64)
        return _mix(np.uint64(seed % 2**64) + i * np.uint64(GOLDEN))


def stream_key(seed, it):
    """Key of the probe stream for EM iteration ``it``."""
    return int(splitmix64(seed, np.uint64(it + 1)))


def rademacher(seed, it, T, C, K, D, t_sel=None):
    """Probes as float64 array [T][C][K][D] of +-1 (or [len(t_sel)][C][K][D] for a task subset)."""
    key = stream_key(seed, it)
    W = (D + 63) // 64
    tasks = np.arange(T) if t_sel is None else np.asarray(t_sel)
    out = np.empty((len(tasks), C, K, D), dtype=np.float64)
    bits = np.arange(64, dtype=np.uint64)
    for a, t in enumerate(tasks):
        idx = ((int(t) * C + np.arange(C)[:, None, None]) * K + np.arange(K)[None, :, None]) * W \
            + np.arange(W)[None, None, :]
        words = splitmix64(key, idx.astype(np.uint64) + np.uint64(1))          # [C][K][W]
        b = (words[..., None] >> bits) & np.uint64(1)                           # [C][K][W][64]
        b = b.reshape(C, K, W * 64)[..., :D]
        out[a] = 1.0 - 2.0 * b.astype(np.float64)
    return out
