"""Pin of the secAccess oracle (Alg. 6 over the Alg. 1 encoding): for every
matched vertex of a small random graph, the reconstructed neighbour IDs are
exactly its plaintext neighbours (dummy IDs filtered out) and the fetched
attribute records are those neighbours' attributes."""
import numpy as np

from oracle import access


def test_sec_access_recovers_neighbours_and_attributes():
    rng = np.random.default_rng(1)
    c_count, x_count = 9, 40
    adj = [sorted(rng.choice(x_count, rng.integers(0, 6), replace=False).tolist()) for _ in range(c_count)]
    attr = rng.integers(0, 2**32, (x_count, 2), dtype=np.uint64).astype(np.uint32)
    post, lmax = access.encode_posting_lists(adj, x_count, 5)
    assert lmax == max(len(a) for a in adj)
    post_sh = access.rss_split(post, 6)
    attr_sh = access.rss_split(attr, 7)
    for m in range(c_count):
        idm = np.zeros(c_count, np.uint8)
        idm[m] = 1
        s1 = rng.integers(0, 2, c_count, dtype=np.uint8)
        s2 = rng.integers(0, 2, c_count, dtype=np.uint8)
        ids, attrs = access.sec_access([s1, s2, idm ^ s1 ^ s2], post_sh, attr_sh, x_count, [3, 4, 5],
                                       (10 + m, 20 + m, 30 + m))
        got_ids = ids[0] ^ ids[1] ^ ids[2]
        got = sorted(int(access.unpack_onehot(r, x_count)[0]) for r in got_ids)
        assert got == adj[m]
        got_attr = attrs[0] ^ attrs[1] ^ attrs[2]
        for r, a in zip(got_ids, got_attr):
            np.testing.assert_array_equal(a, attr[int(access.unpack_onehot(r, x_count)[0])])


def test_posting_list_pads_are_zero_vectors():
    adj = [[1, 3], [], [0, 1, 2]]
    post, lmax = access.encode_posting_lists(adj, 4, 2)
    assert lmax == 3 and post.shape == (3, 3, 1)
    assert (post[1] == 0).all()
    assert sorted(int(v).bit_length() - 1 for v in post[0, :, 0] if v) == [1, 3]
