"""Pin of the oracle's Philox4x64-10 against numpy.random.Philox (library
routine implementing the same published generator)."""
import numpy as np
import pytest

from oracle.philox import philox4x64_10, MASK64


def numpy_block(counter, key):
    # numpy advances the counter before producing a block: starting at c-1
    # makes the first four raw words the block of counter c.
    c = [int(v) for v in counter]
    prev = list(c)
    for k in range(4):          # 256-bit decrement with borrow
        if prev[k] > 0:
            prev[k] -= 1
            break
        prev[k] = MASK64
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(prev, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


CASES = [
    ((0, 0, 0, 0), (0, 0)),
    ((0, 0, 0, 0), (5, 0)),
    ((1, 0, 0, 0), (5, 0)),
    ((12345, 0, 0, 0), (2**63 + 17, 1)),
    ((2047, 5, 0, 0), (987654321, 1)),
    ((MASK64, 0, 0, 0), (3, 1)),            # carry into word 1
    ((MASK64, MASK64, 7, 0), (1, 0)),       # carry into word 2
    ((3, 1, 4, 1), (MASK64, MASK64)),
]


@pytest.mark.parametrize("counter,key", CASES)
def test_block_matches_numpy(counter, key):
    assert philox4x64_10(counter, key) == numpy_block(counter, key)


def test_stream_matches_numpy():
    rng = np.random.Generator(np.random.PCG64(99))
    key = (int(rng.integers(0, 2**63)), 1)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.full(4, MASK64, dtype=np.uint64))
    raw = bg.random_raw(4 * 300)
    for c in range(300):
        assert philox4x64_10((c, 0, 0, 0), key) == tuple(int(v) for v in raw[4 * c:4 * c + 4])
