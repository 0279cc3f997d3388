"""Pin of the oracle's Philox4x64-10 against numpy's independent implementation."""
import numpy as np

from oracle.philox import philox4x64, to_unit, uniforms


def test_blocks_match_numpy():
    rng = np.random.default_rng(5)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(0, 2 ** 62, size=4)]
        key = [int(x) for x in rng.integers(0, 2 ** 62, size=2)]
        # numpy's generator increments its 256-bit counter before each block
        raw = np.random.Philox(counter=ctr, key=key).random_raw(4)
        ctr1 = [ctr[0] + 1, *ctr[1:]]
        mine = philox4x64(*[np.uint64(c) for c in ctr1], np.uint64(key[0]), np.uint64(key[1]))
        assert [int(x) for x in mine] == [int(x) for x in raw]


def test_uniform_sequence_layout():
    U = uniforms(7, 0, np.array([3, 4]), 2, 9, np.arange(10))
    assert U.shape == (2, 10)
    assert np.all((U >= 0) & (U < 1))
    for w, walker in enumerate([3, 4]):
        for q in range(10):
            blk = philox4x64(np.uint64(q // 4), np.uint64(walker), np.uint64(2), np.uint64(9),
                             np.uint64(7), np.uint64(0))
            assert U[w, q] == to_unit(blk[q % 4])
