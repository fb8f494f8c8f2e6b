"""Pins of the range-finder initialisation's generator and sketch."""
import numpy as np

from oracle import cp as ocp
from oracle import sketch as sk


def test_philox_matches_numpy_bit_generator():
    """numpy's Philox (4x64, 10 rounds) with counter c emits the block of
    counter c + 1 first: the published algorithm written out here must give
    the same words."""
    for key, ctr in [([3, 7], [10, 0, 0, 0]), ([0, 0], [0, 0, 0, 0]),
                     ([2 ** 64 - 1, 5], [2 ** 63, 1, 2, 3])]:
        g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                             counter=np.array(ctr, dtype=np.uint64))
        raw = g.random_raw(4)
        nxt = list(ctr)
        nxt[0] = (nxt[0] + 1) % 2 ** 64
        got = sk.philox4x64(np.array(nxt, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(x) for x in got] == [int(x) for x in raw]


def test_sketch_entries_are_standard_normal():
    rng = np.random.default_rng(0)
    others = rng.integers(0, 10 ** 6, size=(20000, 2))
    S = sk.sketch_rows(others, 8, seed=11, j=0)
    assert abs(S.mean()) < 0.02 and abs(S.var() - 1.0) < 0.02
    # columns are uncorrelated, and the same fiber always gets the same row
    c = np.corrcoef(S.T)
    assert np.max(np.abs(c - np.eye(8))) < 0.03
    again = sk.sketch_rows(others[:50], 8, seed=11, j=0)
    assert np.array_equal(again, S[:50])
    other_mode = sk.sketch_rows(others[:50], 8, seed=11, j=1)
    assert not np.allclose(other_mode, S[:50])


def test_range_finder_equals_dense_matricisation_times_sketch():
    """On a tiny tensor (with duplicates) mat(T, j) is materialised
    densely and multiplied by the explicitly materialised S."""
    rng = np.random.default_rng(1)
    dims = (5, 4, 3)
    idx = np.stack([rng.integers(0, d, 80) for d in dims], 1)
    val = rng.standard_normal(80)
    T = ocp.SparseTensor(dims, idx, val)
    R = 5
    for j in range(3):
        oth = [k for k in range(3) if k != j]
        grid = np.stack(np.meshgrid(*[np.arange(dims[k]) for k in oth], indexing="ij"), -1)
        allf = grid.reshape(-1, 2)
        S = sk.sketch_rows(allf, R, seed=5, j=j)
        mat = np.zeros((dims[j], len(allf)))
        col = idx[:, oth[0]] * dims[oth[1]] + idx[:, oth[1]]
        np.add.at(mat, (idx[:, j], col), val)
        np.testing.assert_allclose(sk.range_finder(T, j, R, 5), mat @ S, rtol=1e-12, atol=1e-12)
