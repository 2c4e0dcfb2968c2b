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


# --------------------------------------------------------------------------- Alg. 1 with k-groups

import synth  # noqa: E402


def test_group_k_hand_example():
    """Lengths 5 1 3 2 8 7 1 4, one type, k = 3: in (length, ID) order the
    vertices are 1 6 3 | 2 7 0 5 4 (the remainder of two joins the last
    group), so 1, 6, 3 pad to 2 and the rest to 8."""
    padded, group = access.group_k([5, 1, 3, 2, 8, 7, 1, 4], [0] * 8, 3)
    assert padded.tolist() == [8, 2, 8, 2, 8, 8, 2, 8]
    assert len(set(group[[1, 6, 3]])) == 1 and len(set(group[[2, 7, 0, 5, 4]])) == 1
    assert group[1] != group[0]
    # two types are grouped apart
    padded, group = access.group_k([1, 9, 2, 9, 3, 9], [0, 1, 0, 1, 0, 1], 3)
    assert padded.tolist() == [3, 9, 3, 9, 3, 9]
    assert len(set(group[[0, 2, 4]])) == 1 and group[0] != group[1]


def _check_groups(lengths, types, padded, group, k):
    for t in np.unique(types):
        ids = np.flatnonzero(types == t)
        gs = sorted(set(group[ids]))
        for g in gs:
            m = np.flatnonzero(group == g)
            assert (types[m] == t).all()
            assert len(m) >= k or len(ids) < k                       # k-anonymity of the padded length
            assert (padded[m] == lengths[m].max()).all()             # padded to the group's longest list
        # groups are runs of the length order: no group reaches below another's longest
        spans = sorted((lengths[group == g].min(), lengths[group == g].max()) for g in gs)
        for (lo1, hi1), (lo2, hi2) in zip(spans, spans[1:]):
            assert hi1 <= lo2


def test_group_k_properties_on_random_graph():
    types, adj, _ = synth.posting_graph(3, 5000, 700, 40, n_types=3)
    lengths = np.array([len(a) for a in adj])
    for k in (2, 4, 6):
        padded, group = access.group_k(lengths, types, k)
        _check_groups(lengths, types, padded, group, k)
        for t in np.unique(types):              # every padded value is shared by at least k vertices of the type
            vals, counts = np.unique(padded[types == t], return_counts=True)
            assert counts.min() >= k
    # a grouping in ID order instead of length order breaks the runs
    bad = np.zeros(lengths.size, np.int64)
    ids = np.flatnonzero(types == 0)
    for g in range(ids.size // 4):
        bad[ids[4 * g:4 * g + 4]] = g + 1
    spans = sorted((lengths[bad == g].min(), lengths[bad == g].max()) for g in range(1, ids.size // 4 + 1))
    assert any(hi1 > lo2 for (lo1, hi1), (lo2, hi2) in zip(spans, spans[1:]))


def test_group_k_several_list_types_hand_example():
    """Two list types per vertex (e.g. friends and employers), one type of
    vertex, k = 2.  Length vectors (list 0, list 1): v0 (2, 5), v1 (1, 0),
    v2 (2, 1), v3 (1, 7), v4 (3, 3).  In order of the vector: v1 (1, 0),
    v3 (1, 7) | v2 (2, 1), v0 (2, 5), v4 (3, 3); each list type pads to its
    group's longest."""
    lengths = np.array([[2, 1, 2, 1, 3], [5, 0, 1, 7, 3]])
    padded, group = access.group_k(lengths, [0] * 5, 2)
    assert padded[0].tolist() == [3, 1, 3, 1, 3]
    assert padded[1].tolist() == [5, 7, 5, 7, 5]
    assert group[1] == group[3] and group[0] == group[2] == group[4] and group[0] != group[1]
    # one list type in a (1, n) array is the single-list grouping
    p1, g1 = access.group_k(lengths[:1], [0] * 5, 2)
    p0, g0 = access.group_k(lengths[0], [0] * 5, 2)
    assert p1[0].tolist() == p0.tolist() and g1.tolist() == g0.tolist()


def test_group_k_several_list_types_is_k_automorphic():
    """Every vertex shares its whole vector of padded lengths with at least
    k - 1 others of its type (Alg. 1 picks one group per vertex for all its
    list types); grouping each list type on its own does not give that."""
    rng = np.random.default_rng(5)
    n, k = 400, 4
    types = rng.integers(0, 2, n)
    lengths = np.stack([rng.zipf(1.8, n).clip(0, 30), rng.integers(0, 9, n), rng.zipf(2.5, n).clip(0, 12)])
    padded, group = access.group_k(lengths, types, k)
    for t in (0, 1):
        vecs = [tuple(padded[:, v]) for v in np.flatnonzero(types == t)]
        _, counts = np.unique(np.array(vecs), axis=0, return_counts=True)
        assert counts.min() >= k
        for l in range(3):
            m = types == t
            for g in set(group[m]):
                sel = group == g
                assert (padded[l, sel] == lengths[l, sel].max()).all()
    # separately per list type: some vertex's vector of padded lengths is unique
    sep = np.stack([access.group_k(lengths[l], types, k)[0] for l in range(3)])
    vecs = [tuple(sep[:, v]) for v in np.flatnonzero(types == 0)]
    _, counts = np.unique(np.array(vecs), axis=0, return_counts=True)
    assert counts.min() < k


def test_encoding_places_true_ids_among_zero_dummies():
    types, adj, _ = synth.posting_graph(4, 300, 90, 12)
    lengths = np.array([len(a) for a in adj])
    padded, _ = access.group_k(lengths, types, 3)
    slots = synth.posting_slots(9, lengths, padded)
    rec, off = access.encode_posting_lists_k(adj, 90, padded, slots)
    assert rec.shape == (int(padded.sum()), 3) and off[-1] == rec.shape[0]
    at = 0
    for v, nbrs in enumerate(adj):
        block = rec[off[v]:off[v + 1]]
        assert block.shape[0] == padded[v]
        pops = [sum(bin(int(w)).count("1") for w in r) for r in block]
        assert sum(pops) == len(nbrs) and max(pops + [0]) <= 1          # one-hot or all-zero
        for i, x in enumerate(nbrs):
            assert access.unpack_onehot(block[int(slots[at + i])], 90).tolist() == [x]
        at += len(nbrs)
    sh = access.rss_split_prf(rec, 71, 72, 3)
    np.testing.assert_array_equal(sh[0] ^ sh[1] ^ sh[2], rec)
    np.testing.assert_array_equal(sh[0].reshape(-1), access.rss.prf_words(71, 3, rec.size))


def test_sec_access_csr_recovers_neighbours_and_attributes():
    """Alg. 6 over the k-grouped CSR encoding: every matched vertex's kept IDs
    are exactly its true neighbours, their attribute records exactly theirs."""
    types, adj, attr = synth.posting_graph(5, 60, 50, 9)
    lengths = np.array([len(a) for a in adj])
    padded, _ = access.group_k(lengths, types, 4)
    rec, off = access.encode_posting_lists_k(adj, 50, padded, synth.posting_slots(6, lengths, padded))
    post = access.rss_split_prf(rec, 11, 12, 0)
    attr_sh = access.rss_split(attr, 13)
    rng = np.random.default_rng(2)
    for m in range(0, 60, 7):
        idm = np.zeros(60, np.uint8)
        idm[m] = 1
        s1 = rng.integers(0, 2, 60, dtype=np.uint8)
        s2 = rng.integers(0, 2, 60, dtype=np.uint8)
        ids, attrs = access.sec_access_csr([s1, s2, idm ^ s1 ^ s2], post, off, attr_sh, 50, [3, 4, 5], (7, 8, 9 + m))
        got_ids = ids[0] ^ ids[1] ^ ids[2]
        got = sorted(int(access.unpack_onehot(r, 50)[0]) for r in got_ids)
        assert got == adj[m].tolist()
        got_attr = attrs[0] ^ attrs[1] ^ attrs[2]
        for r, a in zip(got_ids, got_attr):
            np.testing.assert_array_equal(a, attr[int(access.unpack_onehot(r, 50)[0])])
