"""Pins of the oracle's two-party AND (Beaver triples) and bit packing.

Truth table: for every combination of the four share bits x0, x1, y0, y1 and
random triples, the reconstructed output is (x0 ^ x1) & (y0 ^ y1) -- the AND of
shared bits of Sec. III-B / Sec. V-D computed in its two-party form.  The
mutation checks plant mistakes in a copy of the oracle's close step and show
the truth table catches each."""
import numpy as np

from oracle import fss


def _full(bit):
    return np.uint32(0xFFFFFFFF if bit else 0)


def test_truth_table_with_random_triples():
    for trial in range(8):
        t = fss.triples(1000 + trial, 5, trial, 16)
        (a0, a1), (b0, b1), (c0, c1) = t["a"], t["b"], t["c"]
        np.testing.assert_array_equal((a0 ^ a1) & (b0 ^ b1), c0 ^ c1)
        for v in range(16):
            x0, x1, y0, y1 = [(v >> k) & 1 for k in range(4)]
            x = (np.full(16, _full(x0)), np.full(16, _full(x1)))
            y = (np.full(16, _full(y0)), np.full(16, _full(y1)))
            z0, z1 = fss.beaver_and(x, y, t, 16 * 32)
            expect = _full((x0 ^ x1) & (y0 ^ y1))
            assert ((z0 ^ z1) == expect).all()


def test_random_words_and_pad_bits():
    rng = np.random.default_rng(2)
    nrows = 1000
    nw = (nrows + 31) // 32
    vm = fss.valid_mask(nrows)
    x = (rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm,
         rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm)
    y = (rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm,
         rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm)
    z0, z1 = fss.beaver_and(x, y, fss.triples(3, 4, 5, nw), nrows)
    np.testing.assert_array_equal(z0 ^ z1, (x[0] ^ x[1]) & (y[0] ^ y[1]))
    assert (z0[-1] >> (nrows % 32)) == 0 and (z1[-1] >> (nrows % 32)) == 0


def test_triple_words_by_index():
    full = fss.triples(9, 1, 2, 40)
    idx = np.array([0, 7, 39, 13], np.uint32)
    part = fss.triples(9, 1, 2, 0, words=idx)
    for k in ("a", "b", "c"):
        for b in range(2):
            np.testing.assert_array_equal(part[k][b], full[k][b][idx])


def test_mutations_are_caught(monkeypatch):
    t = fss.triples(1, 1, 1, 4)
    good_close = fss.and_close

    def dropped_de(party, d, e, a_b, b_b, c_b):
        return c_b ^ (d & b_b) ^ (e & a_b)

    def swapped(party, d, e, a_b, b_b, c_b):
        z = c_b ^ (d & a_b) ^ (e & b_b)
        return z ^ (d & e) if party == 0 else z

    for bad in (dropped_de, swapped):
        monkeypatch.setattr(fss, "and_close", bad)
        caught = False
        for v in range(16):
            x0, x1, y0, y1 = [(v >> k) & 1 for k in range(4)]
            x = (np.full(4, _full(x0)), np.full(4, _full(x1)))
            y = (np.full(4, _full(y0)), np.full(4, _full(y1)))
            z0, z1 = fss.beaver_and(x, y, t, 128)
            caught |= bool(((z0 ^ z1) != _full((x0 ^ x1) & (y0 ^ y1))).any())
        assert caught
    monkeypatch.setattr(fss, "and_close", good_close)


def test_pack_bits_layout():
    bits = np.zeros(70, np.uint8)
    bits[[0, 31, 32, 69]] = 1
    w = fss.pack_bits(bits)
    assert w.tolist() == [0x80000001, 0x00000001, 0x20]
    np.testing.assert_array_equal(fss.unpack_bits(w, 70), bits)
