"""Pins of the oracle's DPF / DCF and masked-input predicates against what the
paper and the mathematics fix:

* FSS correctness (Def. 3): Eval(k0, x) xor Eval(k1, x) = f(x) for the point
  function [x == alpha] (DPF) and the comparison [x < alpha] (DCF), with
  beta = 1 in Z_2 (Sec. V-C), checked over whole 8- and 12-bit domains.
* Special cases with closed forms: DCF at alpha = 0 is identically 0; at
  alpha = 2^n - 1 it is 1 everywhere but the top value.
* Masked-input predicates (Sec. V-C): with xhat = x + r, the keys reconstruct
  [x == a] and [lo <= x < hi], for every row mask r; r = 0 reduces to the
  unmasked functions.
* Each party's output alone is not the function (a share, not the value).
* The half-tree structure (a published construction, restated in the
  oracle): on the special path the parties' seeds differ by one offset, off
  it they are equal.
* Planted mistakes: copies of the oracle built with one deliberate error
  each (a dropped offset term, a right child that forgets its parent, the
  value bit from the wrong position, an off-by-one leaf mask, no orthomorphism
  in the hash, a dropped running value, t from the wrong bit, a lost wrap
  bit) fail at least one of these pins.
"""
import shutil
import subprocess
import numpy as np
import pytest

from oracle import fss


def _dpf_recon(n, alpha, seed, xs):
    k0, k1 = fss.dpf_gen(n, alpha, seed, alpha)
    return fss.dpf_eval_points(0, k0, n, xs) ^ fss.dpf_eval_points(1, k1, n, xs), (k0, k1)


def _dcf_recon(n, alpha, seed, xs):
    k0, k1 = fss.dcf_gen(n, alpha, seed, alpha)
    return fss.dcf_eval_points(0, k0, n, xs) ^ fss.dcf_eval_points(1, k1, n, xs), (k0, k1)


def test_dpf_exhaustive_8bit():
    xs = np.arange(256, dtype=np.uint32)
    for alpha in range(256):
        y, _ = _dpf_recon(8, alpha, 11, xs)
        np.testing.assert_array_equal(y, (xs == alpha).astype(np.uint8))


def test_dcf_exhaustive_8bit():
    xs = np.arange(256, dtype=np.uint32)
    for alpha in range(256):
        y, _ = _dcf_recon(8, alpha, 12, xs)
        np.testing.assert_array_equal(y, (xs < alpha).astype(np.uint8))


def test_dpf_dcf_12bit_domain():
    xs = np.arange(4096, dtype=np.uint32)
    rng = np.random.default_rng(3)
    alphas = list(rng.integers(0, 4096, 24)) + [0, 1, 127, 128, 4095, 4094, 2048]
    for alpha in alphas:
        y, _ = _dpf_recon(12, int(alpha), 13, xs)
        np.testing.assert_array_equal(y, (xs == alpha).astype(np.uint8))
        y, _ = _dcf_recon(12, int(alpha), 14, xs)
        np.testing.assert_array_equal(y, (xs < alpha).astype(np.uint8))


def test_dcf_closed_forms():
    for n in (8, 12):
        xs = np.arange(1 << n, dtype=np.uint32)
        y, _ = _dcf_recon(n, 0, 21, xs)
        assert not y.any()
        top = (1 << n) - 1
        y, _ = _dcf_recon(n, top, 22, xs)
        expect = np.ones(1 << n, np.uint8)
        expect[top] = 0
        np.testing.assert_array_equal(y, expect)


def test_32bit_points_near_alpha():
    rng = np.random.default_rng(4)
    for alpha in [0, 1, 2**31, 2**32 - 1] + [int(a) for a in rng.integers(0, 2**32, 12, dtype=np.uint64)]:
        pts = {0, 2**32 - 1, alpha, (alpha - 1) % 2**32, (alpha + 1) % 2**32,
               alpha ^ 1, alpha ^ 0x80, alpha ^ (1 << 31)}
        pts |= {int(v) for v in rng.integers(0, 2**32, 40, dtype=np.uint64)}
        xs = np.array(sorted(pts), dtype=np.uint32)
        y, _ = _dpf_recon(32, alpha, 31, xs)
        np.testing.assert_array_equal(y, (xs.astype(np.uint64) == alpha).astype(np.uint8))
        y, _ = _dcf_recon(32, alpha, 32, xs)
        np.testing.assert_array_equal(y, (xs.astype(np.uint64) < alpha).astype(np.uint8))


def test_single_share_is_not_the_function():
    xs = np.arange(4096, dtype=np.uint32)
    _, (k0, k1) = _dcf_recon(12, 1000, 41, xs)
    s0 = fss.dcf_eval_points(0, k0, 12, xs)
    assert 0.3 < s0.mean() < 0.7
    _, (k0, k1) = _dpf_recon(12, 1000, 42, xs)
    s1 = fss.dpf_eval_points(1, k1, 12, xs)
    assert 0.3 < s1.mean() < 0.7


def test_correction_words_common_roots_distinct():
    _, (k0, k1) = _dcf_recon(12, 777, 51, np.arange(4, dtype=np.uint32))
    for f in ("cw", "vcw", "cwleaf"):
        np.testing.assert_array_equal(k0[f], k1[f])
    delta = k0["root"] ^ k1["root"]
    # the roots differ by the offset Delta: t bits (bit 0) differ, bit 1 is clear
    # in both seeds, in Delta and in every correction word
    assert delta[0, 0] & 3 == 1
    assert (k0["root"][:, 0] & 2).max() == 0 and (k0["cw"][:, :5, 0] & 2).max() == 0


def test_half_tree_invariant_along_the_special_path():
    """On alpha's path the two parties' seeds differ by the roots' offset at
    every level; a walk that leaves the path has equal seeds from the first
    level where it leaves (so everything after cancels)."""
    n = 12
    for alpha, x in [(777, 777), (777, 776), (0, 4095), (4095, 2048), (1234, 1234 ^ 0x200)]:
        k0, k1 = fss.dcf_gen(n, alpha, 52, alpha)
        delta = k0["root"][0] ^ k1["root"][0]
        p0, p1 = fss.dcf_path(k0, n, x), fss.dcf_path(k1, n, x)
        hi = [(x >> (n - i)) == (alpha >> (n - i)) for i in range(n - 6)]   # still on the path after i levels
        for i in range(n - 6):
            if hi[i]:
                np.testing.assert_array_equal(p0[i] ^ p1[i], delta)
            else:
                np.testing.assert_array_equal(p0[i], p1[i])
        k0, k1 = fss.dpf_gen(n, alpha, 53, alpha)
        assert not np.array_equal(k0["cw"][0, 0], k0["cw"][0, 1])


def test_correction_bits_do_not_reveal_alpha():
    """For a fixed alpha and fresh seeds, every value-correction bit, every
    t bit of a correction word and their XOR take both values: the key's bits
    hide alpha (a value bit taken from the same position as the t bit would
    make their XOR a function of alpha's bits)."""
    n, alpha = 12, 0b101101110010
    keys = [fss.dcf_gen(n, alpha, 900 + i, 5)[0] for i in range(48)]
    vcw = np.array([[(int(k["vcw"][0]) >> i) & 1 for i in range(n - 7)] for k in keys])
    t_cw = np.array([[int(k["cw"][0, i, 0]) & 1 for i in range(n - 7)] for k in keys])
    for bits in (vcw, t_cw, vcw ^ t_cw):
        assert ((bits.min(axis=0) == 0) & (bits.max(axis=0) == 1)).all()


# --------------------------------------------------------------------------- masked input

def _masked_eq(n, a, xs, r, seed=5, query=1, pred=0):
    k0, k1 = fss.keygen_eq(n, seed, query, pred, a, r)
    xhat = (xs.astype(np.uint64) + r).astype(np.uint32)
    return fss.eval_eq(n, 0, k0, xhat) ^ fss.eval_eq(n, 1, k1, xhat)


def _masked_range(n, lo, hi, xs, r, seed=6, query=1, pred=1):
    k0, k1 = fss.keygen_range(n, seed, query, pred, lo, hi, r)
    xhat = (xs.astype(np.uint64) + r).astype(np.uint32)
    return fss.eval_range(n, 0, k0, xhat) ^ fss.eval_range(n, 1, k1, xhat)


def test_masked_eq_exhaustive_8bit():
    xs = np.arange(256, dtype=np.uint32)
    rng = np.random.default_rng(9)
    for a in range(256):
        r = rng.integers(0, 2**32, 256, dtype=np.uint64).astype(np.uint32)
        np.testing.assert_array_equal(_masked_eq(8, a, xs, r, pred=a), (xs == a).astype(np.uint8))


def test_masked_range_8bit():
    xs = np.arange(256, dtype=np.uint32)
    rng = np.random.default_rng(10)
    pairs = [(0, 0), (5, 5), (255, 255), (0, 255), (0, 1), (254, 255), (0, 128), (128, 255), (17, 18)]
    while len(pairs) < 240:
        lo, hi = sorted(int(v) for v in rng.integers(0, 256, 2))
        pairs.append((lo, hi))
    for i, (lo, hi) in enumerate(pairs):
        r = rng.integers(0, 2**32, 256, dtype=np.uint64).astype(np.uint32)
        y = _masked_range(8, lo, hi, xs, r, pred=i)
        np.testing.assert_array_equal(y, ((xs >= lo) & (xs < hi)).astype(np.uint8))


def test_masked_range_wraps_both_ways():
    """Masks chosen so that L = lo + r wraps past 2^n while U does not, and
    neither or both wrap."""
    n, lo, hi = 8, 40, 90
    xs = np.arange(256, dtype=np.uint32)
    for r0 in (0, 100, 180, 200, 230, 255):
        r = np.full(256, r0, np.uint32)
        y = _masked_range(n, lo, hi, xs, r, pred=r0)
        np.testing.assert_array_equal(y, ((xs >= lo) & (xs < hi)).astype(np.uint8))


def test_zero_mask_reduces_to_unmasked():
    xs = np.arange(4096, dtype=np.uint32)
    r = np.zeros(4096, np.uint32)
    np.testing.assert_array_equal(_masked_eq(12, 1234, xs, r), (xs == 1234).astype(np.uint8))
    np.testing.assert_array_equal(_masked_range(12, 100, 3000, xs, r),
                                  ((xs >= 100) & (xs < 3000)).astype(np.uint8))


def test_masked_32bit_boundaries():
    rng = np.random.default_rng(12)
    for lo, hi in [(0, 2**32 - 1), (2**31, 2**31 + 1), (3, 3), (1000, 2**30),
                   (int(rng.integers(0, 2**31)), int(rng.integers(2**31, 2**32 - 1)))]:
        xs = np.array(sorted({0, 2**32 - 1, lo, hi, (lo - 1) % 2**32, (hi - 1) % 2**32,
                              (hi + 1) % 2**32, lo + 1} |
                             {int(v) for v in rng.integers(0, 2**32, 64, dtype=np.uint64)}),
                      dtype=np.uint32)
        r = rng.integers(0, 2**32, xs.size, dtype=np.uint64).astype(np.uint32)
        y = _masked_range(32, lo, hi, xs, r)
        x64 = xs.astype(np.uint64)
        np.testing.assert_array_equal(y, ((x64 >= lo) & (x64 < hi)).astype(np.uint8))
        a = int(xs[3])
        np.testing.assert_array_equal(_masked_eq(32, a, xs, r), (xs == a).astype(np.uint8))


def test_range_rejects_bad_bounds():
    with pytest.raises(ValueError):
        fss.keygen_range(8, 1, 1, 1, 9, 3, np.zeros(1, np.uint32))
    with pytest.raises(ValueError):
        fss.keygen_range(8, 1, 1, 1, 0, 256, np.zeros(1, np.uint32))


def test_keys_depend_on_row_not_position():
    """A sample of rows gets exactly the keys the full table would give."""
    r = np.random.default_rng(13).integers(0, 2**32, 100, dtype=np.uint64).astype(np.uint32)
    full0, full1 = fss.keygen_range(32, 77, 3, 2, 10, 5000, r)
    rows = np.array([0, 17, 99, 50], np.uint32)
    s0, s1 = fss.keygen_range(32, 77, 3, 2, 10, 5000, r[rows], rows=rows)
    assert s0.tobytes() == full0[rows].tobytes() and s1.tobytes() == full1[rows].tobytes()
    e0, _ = fss.keygen_eq(32, 77, 3, 2, 10, r)
    t0, _ = fss.keygen_eq(32, 77, 3, 2, 10, r[rows], rows=rows)
    assert t0.tobytes() == e0[rows].tobytes()


def test_mask_open_identity():
    rng = np.random.default_rng(14)
    x = rng.integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    x0 = rng.integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    x1 = (x.astype(np.uint64) - x0).astype(np.uint32)
    r = rng.integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    xhat = fss.mask_open(x0, x1, r)
    assert ((xhat.astype(np.int64) - r.astype(np.int64)) % 2**32 == x).all()


@pytest.mark.parametrize("n", [9, 13, 17, 21, 25, 29, 31])
def test_all_domain_widths(n):
    """Every width nu = n - 7 of the early-terminated trees: points at, around
    and far from alpha, and the domain ends."""
    rng = np.random.default_rng(n)
    top = (1 << n) - 1
    for alpha in [0, 1, top, 1 << (n - 1), int(rng.integers(0, top))]:
        pts = {0, top, alpha, (alpha - 1) % (1 << n), (alpha + 1) % (1 << n), alpha ^ 127, alpha ^ 128,
               (alpha & ~127) % (1 << n), (alpha | 127) % (1 << n)}
        pts |= {int(v) for v in rng.integers(0, top + 1, 40, dtype=np.uint64)}
        xs = np.array(sorted(pts), dtype=np.uint32)
        y, _ = _dpf_recon(n, alpha, 7 * n, xs)
        np.testing.assert_array_equal(y, (xs == alpha).astype(np.uint8))
        y, _ = _dcf_recon(n, alpha, 7 * n + 1, xs)
        np.testing.assert_array_equal(y, (xs < alpha).astype(np.uint8))


# --------------------------------------------------------------------------- tree hash and planted mistakes

def _openssl_ecb(key: bytes, data: bytes) -> bytes:
    return subprocess.run(["openssl", "enc", "-aes-128-ecb", "-nopad", "-K", key.hex()],
                          input=data, stdout=subprocess.PIPE, check=True).stdout


def _hash_pin():
    """H(x) = AES_K(sigma(x)) xor sigma(x), K = 00..0f, sigma(a || b) = (a xor b) || a
    on the 8-byte halves, against openssl's AES."""
    rng = np.random.default_rng(61)
    xs = [rng.bytes(16) for _ in range(16)]
    sig = [bytes(a ^ b for a, b in zip(x[:8], x[8:])) + x[:8] for x in xs]
    enc = _openssl_ecb(bytes(range(16)), b"".join(sig))
    for i, x in enumerate(xs):
        want = bytes(a ^ b for a, b in zip(enc[16 * i:16 * i + 16], sig[i]))
        assert fss.tree_hash(x) == want


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not present")
def test_tree_hash_is_fixed_key_aes_with_orthomorphism():
    _hash_pin()


def _fast_pins():
    xs = np.arange(256, dtype=np.uint32)
    for alpha in (0, 1, 77, 127, 128, 200, 255):
        y, _ = _dpf_recon(8, alpha, 11, xs)
        np.testing.assert_array_equal(y, (xs == alpha).astype(np.uint8))
        y, _ = _dcf_recon(8, alpha, 12, xs)
        np.testing.assert_array_equal(y, (xs < alpha).astype(np.uint8))
    for alpha in (300, 3000):
        xs12 = np.arange(4096, dtype=np.uint32)
        y, _ = _dcf_recon(12, alpha, 14, xs12)
        np.testing.assert_array_equal(y, (xs12 < alpha).astype(np.uint8))
    test_masked_range_wraps_both_ways()
    test_half_tree_invariant_along_the_special_path()
    test_correction_bits_do_not_reveal_alpha()
    if shutil.which("openssl"):
        _hash_pin()


@pytest.mark.parametrize("plant", range(1, 9))
def test_planted_mistakes_are_caught(plant, tmp_path, monkeypatch):
    _fast_pins()            # the real oracle passes
    path = fss.build(path=str(tmp_path / f"liboracle_plant{plant}.so"), plant=plant)
    monkeypatch.setattr(fss, "_lib", fss.load(path))
    if plant == 5 and not shutil.which("openssl"):
        pytest.skip("the hash pin needs openssl")
    with pytest.raises(AssertionError):
        _fast_pins()
