"""Python face of the CPU oracle (ctypes over ``liboracle.so`` plus numpy).

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use this module.  The product library never
imports it, and it never imports the product.

The compiled part (``fss_oracle.c``) holds AES-128, the tree hash, the DPF/DCF
Gen/Eval pairs, masked-input key generation and the dealer's counter-mode
randomness.  This file adds the pieces that are plain bitwise algebra:
opening masked values, Beaver AND on packed share words, and bit packing.

Passages followed (paper: OblivGM, arXiv 2209.03526):
  * 2-of-2 additive sharing over Z_{2^k}: Sec. V-B.
  * FSS Gen/Eval: Def. 3 (Sec. III-C); DPF/DCF/IC for =, <, ranges: Sec. V-C.
  * Opening an additively masked value x + r: Sec. V-C (masked-input approach).
  * Bit strings packed into 32-bit words: Sec. VII-A (protocol instantiation).
  * AND of shared bits and aggregation of several predicates by AND:
    Sec. III-B and Sec. V-D (multi-predicate aggregation).  The two-party AND
    here is Beaver's triple method (the paper's three-party replicated AND is
    replaced because the shares are two-party); parity of this step is pinned
    by its truth table.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DPF_KEY = np.dtype([("root", "u1", 16), ("cw", "u1", (32, 16)), ("cwleaf", "u1", 16)])
DCF_KEY = np.dtype([("root", "u1", 16), ("cw", "u1", (32, 16)), ("vcw", "<u4"), ("cwleaf", "u1", 16)])
RANGE_KEY = np.dtype([("upper", DCF_KEY), ("lower", DCF_KEY)])


def build(force: bool = False, path: str = _LIB_PATH, plant: int = 0) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over rows only).  ``plant``
    > 0 builds a copy with one deliberate mistake (for the tests that show the
    pins catch it) at ``path``."""
    if force or plant or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", f"-DORACLE_PLANT={int(plant)}", "-o", tmp, _SRC])
        os.replace(tmp, path)
    return path


_lib = None


def load(path: str):
    """A ctypes handle on a built oracle library with every signature set."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    u32, u64, i32, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
    sig = {
        "oracle_sbox": ([ctypes.c_uint8], ctypes.c_uint8),
        "oracle_aes128_expand": ([P, P], None),
        "oracle_aes128_encrypt": ([P, P, P], None),
        "oracle_hash": ([P, P], None),
        "oracle_dcf_path": ([P, u32, u32, P], None),
        "oracle_rng_block": ([u64, u32, u32, u32, u32, u32, P], None),
        "oracle_rng_blocks": ([u64, u32, u32, u32, u32, u32, sz, P], None),
        "oracle_dpf_gen_seeded": ([u32, u32, u64, u32, P, P], None),
        "oracle_dcf_gen_seeded": ([u32, u32, u64, u32, P, P], None),
        "oracle_dpf_eval_points": ([i32, P, u32, P, sz, P], None),
        "oracle_dcf_eval_points": ([i32, P, u32, P, sz, P], None),
        "oracle_keygen_eq": ([u32, u64, u32, u32, u32, P, P, sz, P, P], None),
        "oracle_keygen_range": ([u32, u64, u32, u32, u32, u32, P, P, sz, P, P], None),
        "oracle_eval_eq": ([u32, i32, P, P, sz, P], None),
        "oracle_eval_range": ([u32, i32, P, P, sz, P], None),
        "oracle_triples": ([u64, u32, u32, P, sz, P, P, P, P, P, P], None),
        "oracle_masks": ([u64, u32, u32, u32, sz, P], None),
        "oracle_sizeof_dpf_key": ([], sz),
        "oracle_sizeof_dcf_key": ([], sz),
        "oracle_sizeof_range_key": ([], sz),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    assert L.oracle_sizeof_dpf_key() == DPF_KEY.itemsize
    assert L.oracle_sizeof_dcf_key() == DCF_KEY.itemsize
    assert L.oracle_sizeof_range_key() == RANGE_KEY.itemsize
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _buf(b: bytes) -> np.ndarray:
    return np.frombuffer(bytes(b), dtype=np.uint8).copy()


# --------------------------------------------------------------------------- AES / tree hash / RNG

def sbox(x: int) -> int:
    return int(lib().oracle_sbox(x))


def aes128_round_keys(key: bytes) -> bytes:
    k = _buf(key)
    rk = np.zeros(176, np.uint8)
    lib().oracle_aes128_expand(_p(k), _p(rk))
    return rk.tobytes()


def aes128_encrypt(key: bytes, block: bytes) -> bytes:
    rk = _buf(aes128_round_keys(key))
    inp = _buf(block)
    out = np.zeros(16, np.uint8)
    lib().oracle_aes128_encrypt(_p(rk), _p(inp), _p(out))
    return out.tobytes()


def tree_hash(x: bytes) -> bytes:
    """H(x) = AES_K(sigma(x)) xor sigma(x), the hash of the half-tree nodes."""
    s = _buf(x)
    out = np.zeros(16, np.uint8)
    lib().oracle_hash(_p(s), _p(out))
    return out.tobytes()


def rng_block(seed: int, domain: int, j: int, query: int, pred: int, elem: int) -> bytes:
    out = np.zeros(16, np.uint8)
    lib().oracle_rng_block(seed, domain, j, query, pred, elem, _p(out))
    return out.tobytes()


def rng_blocks(seed: int, domain: int, j: int, query: int, pred: int, elem0: int, count: int) -> np.ndarray:
    """Blocks (domain, j, query, pred, elem0 + i) for i < count, as a (count, 16)
    uint8 array: rng_block for consecutive counters."""
    out = np.zeros((count, 16), np.uint8)
    if count:
        lib().oracle_rng_blocks(seed, domain, j, query, pred, elem0, count, _p(out))
    return out


# --------------------------------------------------------------------------- DPF / DCF

def dpf_gen(n: int, alpha: int, seed: int, elem: int = 0):
    k0 = np.zeros(1, DPF_KEY)
    k1 = np.zeros(1, DPF_KEY)
    lib().oracle_dpf_gen_seeded(n, alpha, seed, elem, _p(k0), _p(k1))
    return k0, k1


def dcf_gen(n: int, alpha: int, seed: int, elem: int = 0):
    k0 = np.zeros(1, DCF_KEY)
    k1 = np.zeros(1, DCF_KEY)
    lib().oracle_dcf_gen_seeded(n, alpha, seed, elem, _p(k0), _p(k1))
    return k0, k1


def dcf_path(key: np.ndarray, n: int, x: int) -> np.ndarray:
    """Seeds of the nodes the walk of x passes (root first), (n - 6, 16) uint8."""
    out = np.zeros((n - 6, 16), np.uint8)
    lib().oracle_dcf_path(_p(key), n, x, _p(out))
    return out


def dpf_eval_points(party: int, key: np.ndarray, n: int, xs) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.uint32)
    out = np.zeros(xs.size, np.uint8)
    lib().oracle_dpf_eval_points(party, _p(key), n, _p(xs), xs.size, _p(out))
    return out


def dcf_eval_points(party: int, key: np.ndarray, n: int, xs) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.uint32)
    out = np.zeros(xs.size, np.uint8)
    lib().oracle_dcf_eval_points(party, _p(key), n, _p(xs), xs.size, _p(out))
    return out


# --------------------------------------------------------------------------- masked-input predicates

def _rows_arg(rows, count):
    if rows is None:
        return None, None
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    assert rows.size == count
    return rows, _p(rows)


def keygen_eq(n: int, seed: int, query: int, pred: int, a: int, r: np.ndarray, rows=None):
    """Dealer keys for [x == a] on masked input xhat = x + r (one key pair per row).

    ``rows`` (optional) names the table row of each entry; the dealer's random
    seeds depend on the row index, so a sample of rows gets the same keys as
    the full table would."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    if not (0 <= a < (1 << n)):
        raise ValueError("equality predicate needs 0 <= a < 2^n")
    rows, prow = _rows_arg(rows, r.size)
    k0 = np.zeros(r.size, DPF_KEY)
    k1 = np.zeros(r.size, DPF_KEY)
    lib().oracle_keygen_eq(n, seed, query, pred, a, _p(r), prow, r.size, _p(k0), _p(k1))
    return k0, k1


def keygen_range(n: int, seed: int, query: int, pred: int, lo: int, hi: int, r: np.ndarray,
                 rows=None):
    """Dealer keys for [lo <= x < hi] on masked input xhat = x + r."""
    if not (0 <= lo <= hi < (1 << n)):
        raise ValueError("range predicate needs 0 <= lo <= hi < 2^n")
    r = np.ascontiguousarray(r, dtype=np.uint32)
    rows, prow = _rows_arg(rows, r.size)
    k0 = np.zeros(r.size, RANGE_KEY)
    k1 = np.zeros(r.size, RANGE_KEY)
    lib().oracle_keygen_range(n, seed, query, pred, lo, hi, _p(r), prow, r.size, _p(k0), _p(k1))
    return k0, k1


def eval_eq(n: int, party: int, keys: np.ndarray, xhat: np.ndarray) -> np.ndarray:
    xhat = np.ascontiguousarray(xhat, dtype=np.uint32)
    out = np.zeros(xhat.size, np.uint8)
    lib().oracle_eval_eq(n, party, _p(keys), _p(xhat), xhat.size, _p(out))
    return out


def eval_range(n: int, party: int, keys: np.ndarray, xhat: np.ndarray) -> np.ndarray:
    xhat = np.ascontiguousarray(xhat, dtype=np.uint32)
    out = np.zeros(xhat.size, np.uint8)
    lib().oracle_eval_range(n, party, _p(keys), _p(xhat), xhat.size, _p(out))
    return out


def masks(seed: int, query: int, pred: int, count: int, row_offset: int = 0) -> np.ndarray:
    """The dealer's masks drawn from its counter-mode generator (domain 2)."""
    r = np.zeros(count, np.uint32)
    lib().oracle_masks(seed, query, pred, row_offset, count, _p(r))
    return r


def mask_open(x0: np.ndarray, x1: np.ndarray, r: np.ndarray) -> np.ndarray:
    """xhat = x0 + x1 + r (mod 2^32): the value both servers see after opening."""
    return (x0.astype(np.uint64) + x1.astype(np.uint64) + r.astype(np.uint64)).astype(np.uint32)


# --------------------------------------------------------------------------- bits and Beaver AND

def pack_bits(bits: np.ndarray) -> np.ndarray:
    """Row i -> bit (i % 32) of word i // 32; pad bits are zero."""
    bits = np.asarray(bits, dtype=np.uint8)
    nwords = (bits.size + 31) // 32
    padded = np.zeros(nwords * 32, np.uint8)
    padded[:bits.size] = bits & 1
    return np.packbits(padded, bitorder="little").view("<u4").astype(np.uint32)


def unpack_bits(words: np.ndarray, nrows: int) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype="<u4")
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:nrows]


def valid_mask(nrows: int) -> np.ndarray:
    """Packed words with bit 1 for every row < nrows (the public constant 1)."""
    return pack_bits(np.ones(nrows, np.uint8))


def triples(seed: int, query: int, and_id: int, nwords: int, words=None):
    """Both parties' Beaver triples for AND number ``and_id`` of a query, one
    triple word per 32 rows (``words``: optional list of word indices)."""
    if words is not None:
        words = np.ascontiguousarray(words, dtype=np.uint32)
        nwords = words.size
    arrs = [np.zeros(nwords, np.uint32) for _ in range(6)]
    lib().oracle_triples(seed, query, and_id, None if words is None else _p(words), nwords,
                         *[_p(a) for a in arrs])
    a0, a1, b0, b1, c0, c1 = arrs
    return {"a": (a0, a1), "b": (b0, b1), "c": (c0, c1)}


def and_open(x_b, y_b, a_b, b_b):
    """Party b's message: d_b = x_b ^ a_b, e_b = y_b ^ b_b."""
    return x_b ^ a_b, y_b ^ b_b


def and_close(party: int, d, e, a_b, b_b, c_b):
    """z_b = c_b ^ (d & b_b) ^ (e & a_b) ^ [b == 0](d & e), with d, e opened."""
    z = c_b ^ (d & b_b) ^ (e & a_b)
    if party == 0:
        z = z ^ (d & e)
    return z


def beaver_and(x, y, trip, nrows: int):
    """Both parties' AND of shared packed bits x = (x0, x1), y = (y0, y1)."""
    (a0, a1), (b0, b1), (c0, c1) = trip["a"], trip["b"], trip["c"]
    d0, e0 = and_open(x[0], y[0], a0, b0)
    d1, e1 = and_open(x[1], y[1], a1, b1)
    d, e = d0 ^ d1, e0 ^ e1
    vm = valid_mask(nrows)
    z0 = and_close(0, d, e, a0, b0, c0) & vm
    z1 = and_close(1, d, e, a1, b1, c1) & vm
    return z0, z1
