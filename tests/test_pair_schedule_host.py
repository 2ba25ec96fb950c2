"""Host checks of the index arithmetic of the unique-pair FP64 evaluation
(pairs_fp64_up): the ring order p = (k - 1) n + i, decoded on the GPU with an
FP32 product and a truncation, enumerates every unordered pair of an n-atom
cluster exactly once, for every n the evaluation serves (n <= 64)."""
import numpy as np


def decode(p, n):
    """The kernel's decoding, step by step in FP32 (no fused operations)."""
    inv_n = np.float32(1.0) / np.float32(n)
    prod = (np.float32(p) + np.float32(0.5)) * inv_n
    k1 = int(prod)  # truncation toward zero, as the float-to-int conversion
    i = p - k1 * n
    j = i + k1 + 1
    return k1, i, j - n if j >= n else j


def test_fp32_decoding_is_exact_division():
    for n in range(2, 65):
        for p in range(n * (n - 1) // 2):
            k1, i, _ = decode(p, n)
            assert (k1, i) == divmod(p, n), (n, p)


def test_ring_order_covers_every_pair_once():
    for n in range(2, 65):
        P = n * (n - 1) // 2
        seen = set()
        for p in range(P):
            _, i, j = decode(p, n)
            assert 0 <= i < n and 0 <= j < n and i != j, (n, p)
            key = (min(i, j), max(i, j))
            assert key not in seen, (n, p, key)
            seen.add(key)
        assert len(seen) == P
