"""Pins of the oracle's overlay mipmap (section 3: a mipmap of the full-resolution overlay).

* a 3 x 5 example summed by hand;
* an independent reduction (pad to even with zeros, reshape into 2 x 2 blocks, numpy sum / max) on
  ragged sizes;
* invariants: every level holds the total count and the global maximum speed; the last level is 1 x 1;
  the number of levels is 1 + ceil(log2(max(H, W)));
* degenerate grids (1 x 1, one row, one column).
"""
import math

import numpy as np
import pytest

import oracle


def test_hand_example():
    c = np.arange(15, dtype=np.uint32).reshape(3, 5)
    v = np.array([[1, 0, 0, 0, 2], [0, 3, 0, 0, 0], [0, 0, 5, 0, 4]], np.float32)
    (c1, v1), (c2, v2), (c3, v3) = oracle.mipmap(c, v)
    assert c1.tolist() == [[12, 20, 13], [21, 25, 14]]
    assert v1.tolist() == [[3, 0, 2], [0, 5, 4]]
    assert c2.tolist() == [[78, 27]] and v2.tolist() == [[5, 4]]
    assert c3.tolist() == [[105]] and v3.tolist() == [[5]]


def _reference_level(c, v):
    h, w = c.shape
    hp, wp = h + h % 2, w + w % 2
    cp = np.zeros((hp, wp), np.uint64)
    vp = np.zeros((hp, wp), np.float32)
    cp[:h, :w] = c
    vp[:h, :w] = v
    return (cp.reshape(hp // 2, 2, wp // 2, 2).sum(axis=(1, 3)),
            vp.reshape(hp // 2, 2, wp // 2, 2).max(axis=(1, 3)))


@pytest.mark.parametrize("shape", [(37, 53), (64, 64), (1, 17), (23, 1), (2, 3), (129, 255)])
def test_against_blockwise_reduction(shape):
    rng = np.random.default_rng(sum(shape))
    c = rng.integers(0, 1 << 20, shape).astype(np.uint32)
    v = (rng.random(shape) * (rng.random(shape) < 0.6)).astype(np.float32) * 60
    pyr = oracle.mipmap(c, v)
    assert len(pyr) == oracle.mipmap_levels(*shape) - 1 == math.ceil(math.log2(max(shape)))
    cc, vv = c.astype(np.uint64), v
    for lc, lv in pyr:
        cc, vv = _reference_level(cc, vv)
        assert np.array_equal(lc, cc) and np.array_equal(lv, vv)
        assert int(lc.sum()) == int(c.astype(np.uint64).sum())
        assert lv.max() == v.max()
    assert pyr[-1][0].shape == (1, 1)


def test_single_cell_has_no_coarser_level():
    assert oracle.mipmap_levels(1, 1) == 1
    assert oracle.mipmap(np.ones((1, 1), np.uint32), np.ones((1, 1), np.float32)) == []
