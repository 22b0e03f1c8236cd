"""Pins of the CPU reference of the serving motion (oracle/walk.py).

The motion is the serving workload's, not the paper's method; its reference
is pinned by the published known-answer vectors of Philox4x32-10
(tests/golden/philox4x32_10_kat.json), by a second, deliberately plain
implementation of the same definition (scalar Python integers, one round at a
time) and by distribution properties of the Irwin-Hall normal it feeds."""
import json
import os

import numpy as np
import pytest

from oracle import walk


def philox_scalar(c, k):
    """Philox4x32-10 on Python ints: ten rounds of two 32x32->64 products,
    the key bumped by the two Weyl constants after each round."""
    c = list(c)
    k0, k1 = k
    mask = 0xFFFFFFFF
    for _ in range(10):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & mask, p1 & mask, ((p0 >> 32) ^ c[3] ^ k1) & mask,
             p0 & mask]
        k0 = (k0 + 0x9E3779B9) & mask
        k1 = (k1 + 0xBB67AE85) & mask
    return c


def test_known_answer_vectors():
    """The generator against the known-answer vectors published with the
    Philox definition (counter, key, output), including all-zero and
    all-ones inputs."""
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")
    cases = json.load(open(path))["cases"]
    assert len(cases) == 3
    for c in cases:
        ctr = np.array([[int(w, 16) for w in c["ctr"]]], dtype=np.uint32)
        k0, k1 = (int(w, 16) for w in c["key"])
        want = [int(w, 16) for w in c["out"]]
        assert [int(v) for v in walk.philox4x32_10(ctr, k0, k1)[0]] == want
        assert philox_scalar([int(w, 16) for w in c["ctr"]], (k0, k1)) == want


def test_vectorised_equals_scalar():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, size=(300, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    for key in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (12345, 678910), (0xDEADBEEF, 1)]:
        got = walk.philox4x32_10(ctr, *key)
        for i in range(ctr.shape[0]):
            assert [int(v) for v in got[i]] == philox_scalar([int(v) for v in ctr[i]], key)


def test_avalanche():
    """Flipping one counter bit flips about half of the 128 output bits."""
    rng = np.random.default_rng(4)
    ctr = rng.integers(0, 2 ** 32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    base = walk.philox4x32_10(ctr, 7, 9)
    flipped = ctr.copy()
    flipped[:, 2] ^= np.uint32(1 << 5)
    out = walk.philox4x32_10(flipped, 7, 9)
    bits = np.unpackbits((base ^ out).view(np.uint8)).reshape(2000, -1).sum(axis=1)
    assert abs(bits.mean() - 64.0) < 1.0


def test_irwin_hall_distribution():
    z = walk.normal_z(np.arange(400_000), 1, 3, 99).astype(np.float64)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert z.min() >= -6.0 and z.max() <= 6.0
    # fourth moment of the sum of 12 uniforms: 3 - 1.2/12 = 2.9
    assert abs((z ** 4).mean() - 2.9) < 0.05


def test_walk_step_definition():
    """hi = lo + side after every step, counters depend on region, axis and
    step, and the motion is reproducible."""
    rng = np.random.default_rng(5)
    lo = (rng.random((500, 2)) * 1e6).astype(np.float32)
    a_lo, a_hi = walk.walk_step(lo, 0, 50.0, 5.0, 17, 1)
    b_lo, b_hi = walk.walk_step(lo, 0, 50.0, 5.0, 17, 1)
    assert np.array_equal(a_lo, b_lo) and np.array_equal(a_hi, b_hi)
    assert np.array_equal(a_hi, (a_lo + np.float32(50.0)).astype(np.float32))
    c_lo, _ = walk.walk_step(lo, 0, 50.0, 5.0, 17, 2)
    assert not np.array_equal(a_lo, c_lo)
    d_lo, _ = walk.walk_step(lo, 1, 50.0, 5.0, 17, 1)  # shifted region numbering
    assert not np.array_equal(d_lo, a_lo)
    # the displacement is sigma * z exactly
    z0 = walk.normal_z(np.arange(500), 0, 1, 17)
    assert np.array_equal(a_lo[:, 0], lo[:, 0] + np.float32(5.0) * z0)


@pytest.mark.parametrize("steps", [1, 3])
def test_walk_generator_matches_steps(steps):
    rng = np.random.default_rng(6)
    ul = (rng.random((40, 2)) * 100).astype(np.float32)
    sl = (rng.random((30, 2)) * 100).astype(np.float32)
    last = None
    for st, a, ah, b, bh in walk.walk(ul, sl, 2.0, 0.2, 5, steps):
        last = (st, a, b)
    u, s = ul, sl
    for st in range(1, steps + 1):
        u, _ = walk.walk_step(u, 0, 2.0, 0.2, 5, st)
        s, _ = walk.walk_step(s, 40, 2.0, 0.2, 5, st)
    assert last[0] == steps and np.array_equal(last[1], u) and np.array_equal(last[2], s)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_c_walk_equals_numpy_walk(d):
    """The C replay used for full-size checks gives the numpy reference's
    bits: ordinary coordinates, large ones (where lo + side rounds back to
    lo), negative and huge sigmas, several steps and a 64-bit seed."""
    rng = np.random.default_rng(100 + d)
    lo = (rng.random((3000, d)) * 1e6).astype(np.float32)
    lo[:50] = np.float32(3.0e10)
    lo[50:60] = np.float32(-1.0e38)
    for side, sigma, seed in ((0.25, 0.025, 7), (400.0, -2.0e5, 0xDEADBEEF12345678),
                              (0.0, 1.0e30, 2**63 + 5)):
        fast = list(walk.walk_fast(lo, lo[::-1], side, sigma, seed, 3, first_step=4))
        ref = list(walk.walk(lo, lo[::-1], side, sigma, seed, 3, first_step=4))
        for a, b in zip(fast, ref):
            assert a[0] == b[0]
            for x, y in zip(a[1:], b[1:]):
                assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
