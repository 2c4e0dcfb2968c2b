"""Conversion between the oracle's per-row key records and the library's
structure-of-arrays key batches (layout stated in include/oblivgm_fss.h).
Test helper only: neither side's arithmetic lives here."""
import numpy as np

from oracle import fss as ofss


def pad_rows(n):
    return (n + 63) // 64 * 64


def _planes(np_, nbits, dcf):
    """Byte offset of every plane of one DPF (dcf=False) or DCF sub-key, and
    the sub-key's size: root | cw_0 .. cw_{nu-1} | [vcw] | cwleaf."""
    nu = nbits - 7
    off = {"root": 0}
    for i in range(nu):
        off[("cw", i)] = 16 * np_ * (1 + i)
    base = 16 * np_ * (1 + nu)
    if dcf:
        off["vcw"] = base
        base += 4 * np_
    off["cwleaf"] = base
    return off, base + 16 * np_


def _put(buf, off, n, data, width):
    buf[off:off + n * width] = np.ascontiguousarray(data).view(np.uint8).reshape(-1)


def _get(buf, off, n, width):
    return buf[off:off + n * width]


def _enc(buf, base, np_, nbits, k, dcf):
    off, size = _planes(np_, nbits, dcf)
    n = k.size
    _put(buf, base + off["root"], n, k["root"], 16)
    for i in range(nbits - 7):
        _put(buf, base + off[("cw", i)], n, k["cw"][:, i, :], 16)
    if dcf:
        _put(buf, base + off["vcw"], n, k["vcw"].astype("<u4"), 4)
    _put(buf, base + off["cwleaf"], n, k["cwleaf"], 16)
    return size


def _dec(buf, base, np_, nbits, n, out, dcf):
    off, size = _planes(np_, nbits, dcf)
    out["root"] = _get(buf, base + off["root"], n, 16).reshape(n, 16)
    for i in range(nbits - 7):
        out["cw"][:, i, :] = _get(buf, base + off[("cw", i)], n, 16).reshape(n, 16)
    if dcf:
        out["vcw"] = _get(buf, base + off["vcw"], n, 4).view("<u4")
    out["cwleaf"] = _get(buf, base + off["cwleaf"], n, 16).reshape(n, 16)
    return size


def to_device(kind, nbits, keys):
    """Oracle records (DPF_KEY or RANGE_KEY array) -> device batch bytes."""
    n = keys.size
    np_ = pad_rows(n)
    if kind == 0:
        _, size = _planes(np_, nbits, False)
        buf = np.zeros(size, np.uint8)
        _enc(buf, 0, np_, nbits, keys, False)
        return buf
    _, half = _planes(np_, nbits, True)
    buf = np.zeros(2 * half, np.uint8)
    _enc(buf, 0, np_, nbits, keys["upper"], True)
    _enc(buf, half, np_, nbits, keys["lower"], True)
    return buf


def from_device(kind, nbits, n, buf):
    """Device batch bytes -> oracle records (levels beyond the tree stay zero)."""
    buf = np.asarray(buf, np.uint8)
    np_ = pad_rows(n)
    if kind == 0:
        out = np.zeros(n, ofss.DPF_KEY)
        _dec(buf, 0, np_, nbits, n, out, False)
        return out
    out = np.zeros(n, ofss.RANGE_KEY)
    _, half = _planes(np_, nbits, True)
    up = np.zeros(n, ofss.DCF_KEY)
    lo = np.zeros(n, ofss.DCF_KEY)
    _dec(buf, 0, np_, nbits, n, up, True)
    _dec(buf, half, np_, nbits, n, lo, True)
    out["upper"] = up
    out["lower"] = lo
    return out
