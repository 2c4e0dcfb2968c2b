"""Alg. 1's grouping as the library computes it on the host (rss_group_k)
against the oracle's, and its k-anonymity: every padded length is shared by
at least k vertices of the type."""
import numpy as np
import pytest

import synth
from oracle import access


@pytest.fixture(scope="module")
def fss():
    from paper_2209_03526_amd import fss as f
    return f


@pytest.mark.parametrize("k", [1, 2, 3, 6, 50])
def test_group_k_equals_oracle(fss, k):
    types, adj, _ = synth.posting_graph(11, 4000, 500, 30, n_types=3)
    lengths = np.array([len(a) for a in adj], np.uint32)
    padded, group = fss.rss_group_k(lengths, types, k)
    want_p, want_g = access.group_k(lengths, types, k)
    np.testing.assert_array_equal(padded, want_p)
    np.testing.assert_array_equal(group, want_g)
    for t in np.unique(types):
        _, counts = np.unique(padded[types == t], return_counts=True)
        assert counts.min() >= k


def test_group_k_small_types_and_errors(fss):
    padded, group = fss.rss_group_k([3, 1, 2], [0, 0, 1], 4)      # fewer than k: one group per type
    assert padded.tolist() == [3, 3, 2] and group[0] == group[1] != group[2]
    assert fss.LIB.rss_group_k(3, None, None, 2, None, None) == fss.EINVAL
    lengths = np.array([1, 2], np.uint32)
    with pytest.raises(fss.FssError):
        fss.rss_group_k(lengths, lengths, 0)


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_group_k_lists_equals_oracle(fss, k):
    """Several posting-list types per vertex: the library's grouping and
    padded lengths equal the oracle's, and every vertex shares its vector of
    padded lengths with at least k - 1 others of its type."""
    rng = np.random.default_rng(k)
    n = 3000
    types = rng.integers(0, 3, n).astype(np.uint32)
    lengths = np.stack([rng.zipf(1.8, n).clip(0, 40), rng.integers(0, 6, n), rng.zipf(2.2, n).clip(0, 9)]).astype(
        np.uint32)
    padded, group = fss.rss_group_k_lists(lengths, types, k)
    want_p, want_g = access.group_k(lengths, types, k)
    np.testing.assert_array_equal(padded, want_p)
    np.testing.assert_array_equal(group, want_g)
    for t in range(3):
        _, counts = np.unique(padded[:, types == t].T, axis=0, return_counts=True)
        assert counts.min() >= k
    # one list type through the general call is rss_group_k
    p1, g1 = fss.rss_group_k_lists(lengths[:1], types, k)
    p0, g0 = fss.rss_group_k(lengths[0], types, k)
    np.testing.assert_array_equal(p1[0], p0)
    np.testing.assert_array_equal(g1, g0)
    assert fss.LIB.rss_group_k_lists(n, 0, lengths.ctypes.data, types.ctypes.data, k, padded.ctypes.data,
                                     None) == fss.EINVAL
