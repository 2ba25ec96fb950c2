"""Host checks of the pair schedules of the one-wavefront kernels.

The unique-pair FP64 Morse evaluation (pairs_morse64_up): the ring order
p = (k - 1) n + i, decoded on the GPU with an FP32 product and a truncation,
enumerates every unordered pair of an n-atom cluster exactly once, for every
n <= 64.

The FP32 ring (pairs_ring): 64 lanes, lane l holding atom l mod n, staged
coordinates pos[j] = atom j mod n, distances k = 1 .. n/2 (for even n the last
one on the lanes whose atom is below n/2), a reaction register that every lane
passes to the lane below before each step (lane 63 takes lane 0's), and the
readout "lane l holds the reaction on atom (l + n/2) mod n": emulated here lane
by lane, it gives every atom's full pair sum for every n the ring serves
(20 <= n <= 43), and the admission rule n/2 <= 64 - n is exactly where it
stops doing so."""
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


def ring_emulation(x, n):
    """Per-atom sums of the pair vectors d / |d|^2 (any pair term would do)
    through the ring's schedule: own terms plus the rotated reactions."""
    K = n // 2
    lanes = np.arange(64)
    upper = (n % 2 == 0) & (lanes % n >= K)
    pos = np.array([x[j % n] for j in range(64 + K)])
    own = np.zeros((64, 3))
    react = np.zeros((64, 3))
    for k in range(1, K + 1):
        d = pos[lanes] - pos[lanes + k]
        f = 1.0 / (d * d).sum(axis=1)
        if k == K:
            f = np.where(upper, 0.0, f)
        own += f[:, None] * d
        react = np.roll(react, -1, axis=0)  # lane l receives lane l + 1's sum
        react -= f[:, None] * d
    g = own[:n].copy()
    for lane in range(n):
        g[(lane + K) % n] += react[lane]
    return g


def direct_sums(x):
    d = x[:, None, :] - x[None, :, :]
    r2 = (d * d).sum(axis=2)
    np.fill_diagonal(r2, np.inf)
    return (d / r2[:, :, None]).sum(axis=1)


def test_ring_schedule_gives_every_pair_sum():
    rng = np.random.default_rng(20)
    for n in range(20, 47):
        x = rng.standard_normal((n, 3)) * 3.0
        ok = np.allclose(ring_emulation(x, n), direct_sums(x), rtol=1e-12, atol=1e-12)
        assert ok == (n // 2 <= 64 - n), n
