"""Pin the oracle's Philox4x32-10 against rocRAND's independent implementation of the same bijection.

The model's random deviation (section 5.2: a user-set amount of random variation from the optimal path)
is drawn from Philox4x32-10 (Salmon et al., SC'11). rocRAND ships its own Philox4x32-10; its ten-round
block function is called here on the host, so a mistake in the oracle's multipliers, Weyl key
increments, word shuffle or round count fails this test.
"""
import numpy as np
import pytest

import oracle
from tests.support.philox_ref import philox_blocks


def _vectors():
    rng = np.random.default_rng(2025)
    rows = [np.zeros(6, np.uint32), np.full(6, 0xFFFFFFFF, np.uint32),
            np.array([1, 0, 0, 0, 0, 0], np.uint32), np.array([0, 0, 0, 0, 1, 0], np.uint32),
            np.array([0, 0, 0, 0, 0, 1], np.uint32), np.array([0, 0, 0, 1, 0, 0], np.uint32)]
    rows += list(rng.integers(0, 2**32, size=(250, 6), dtype=np.uint64).astype(np.uint32))
    # counters of the shape the model uses: (step/2, replica, cell, run) with a 64-bit seed as the key
    for n in range(0, 40, 7):
        for j in (0, 1, 255):
            rows.append(np.array([n, j, 123457, 3, 0x89ABCDEF, 0x01234567], np.uint32))
    return np.stack(rows)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_philox_matches_rocrand(prec):
    vec = _vectors()
    ref = philox_blocks(vec)
    got = np.stack([oracle.philox(v[:4], v[4:], prec) for v in vec])
    assert np.array_equal(got, ref)


def test_philox_uniform_bits():
    # Output words are uniform: each of the 32 bit positions is set about half the time.
    out = np.stack([oracle.philox([n, 0, 0, 0], [1, 2]) for n in range(4096)])
    bits = ((out[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1, 32)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 0.02)
