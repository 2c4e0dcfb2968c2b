"""Conversion between the oracle's per-row key records and the library's
structure-of-arrays key batches (layout stated in include/oblivgm_fss.h).
Test helper only: neither side's arithmetic lives here."""
import numpy as np

from oracle import fss as ofss


def pad_rows(n):
    return (n + 63) // 64 * 64


def _dcf_planes(np_, nbits):
    nu = nbits - 7
    off = {"root": 0}
    for i in range(nu):
        off[("scw", i)] = 16 * np_ * (1 + i)
    base = 16 * np_ * (1 + nu)
    off["tl"], off["tr"], off["vcw"], off["cwleaf"] = base, base + 4 * np_, base + 8 * np_, base + 12 * np_
    return off, base + 12 * np_ + 16 * np_


def _dpf_planes(np_, nbits):
    nu = nbits - 7
    off = {"root": 0}
    for i in range(nu):
        off[("scw", i)] = 16 * np_ * (1 + i)
    base = 16 * np_ * (1 + nu)
    off["tl"], off["tr"], off["cwout"] = base, base + 4 * np_, base + 8 * np_
    return off, base + 8 * np_ + 16 * np_


def _put(buf, off, n, data, width):
    buf[off:off + n * width] = np.ascontiguousarray(data).view(np.uint8).reshape(-1)


def _get(buf, off, n, width):
    return buf[off:off + n * width]


def _enc_dcf(buf, base, np_, nbits, k):
    off, size = _dcf_planes(np_, nbits)
    n = k.size
    _put(buf, base + off["root"], n, k["root"], 16)
    for i in range(nbits - 7):
        _put(buf, base + off[("scw", i)], n, k["scw"][:, i, :], 16)
    for f in ("tl", "tr", "vcw"):
        _put(buf, base + off[f], n, k[f].astype("<u4"), 4)
    _put(buf, base + off["cwleaf"], n, k["cwleaf"], 16)
    return size


def _dec_dcf(buf, base, np_, nbits, n, out):
    off, size = _dcf_planes(np_, nbits)
    out["root"] = _get(buf, base + off["root"], n, 16).reshape(n, 16)
    for i in range(nbits - 7):
        out["scw"][:, i, :] = _get(buf, base + off[("scw", i)], n, 16).reshape(n, 16)
    for f in ("tl", "tr", "vcw"):
        out[f] = _get(buf, base + off[f], n, 4).view("<u4")
    out["cwleaf"] = _get(buf, base + off["cwleaf"], n, 16).reshape(n, 16)
    return size


def to_device(kind, nbits, keys):
    """Oracle records (DPF_KEY or RANGE_KEY array) -> device batch bytes."""
    n = keys.size
    np_ = pad_rows(n)
    if kind == 0:
        off, size = _dpf_planes(np_, nbits)
        buf = np.zeros(size, np.uint8)
        _put(buf, off["root"], n, keys["root"], 16)
        for i in range(nbits - 7):
            _put(buf, off[("scw", i)], n, keys["scw"][:, i, :], 16)
        _put(buf, off["tl"], n, keys["tl"].astype("<u4"), 4)
        _put(buf, off["tr"], n, keys["tr"].astype("<u4"), 4)
        _put(buf, off["cwout"], n, keys["cwout"], 16)
        return buf
    _, half = _dcf_planes(np_, nbits)
    buf = np.zeros(2 * half, np.uint8)
    _enc_dcf(buf, 0, np_, nbits, keys["upper"])
    _enc_dcf(buf, half, np_, nbits, keys["lower"])
    return buf


def from_device(kind, nbits, n, buf):
    """Device batch bytes -> oracle records (levels beyond the tree stay zero)."""
    buf = np.asarray(buf, np.uint8)
    np_ = pad_rows(n)
    if kind == 0:
        out = np.zeros(n, ofss.DPF_KEY)
        off, _ = _dpf_planes(np_, nbits)
        out["root"] = _get(buf, off["root"], n, 16).reshape(n, 16)
        for i in range(nbits - 7):
            out["scw"][:, i, :] = _get(buf, off[("scw", i)], n, 16).reshape(n, 16)
        out["tl"] = _get(buf, off["tl"], n, 4).view("<u4")
        out["tr"] = _get(buf, off["tr"], n, 4).view("<u4")
        out["cwout"] = _get(buf, off["cwout"], n, 16).reshape(n, 16)
        return out
    out = np.zeros(n, ofss.RANGE_KEY)
    _, half = _dcf_planes(np_, nbits)
    up = np.zeros(n, ofss.DCF_KEY)
    lo = np.zeros(n, ofss.DCF_KEY)
    _dec_dcf(buf, 0, np_, nbits, n, up)
    _dec_dcf(buf, half, np_, nbits, n, lo)
    out["upper"] = up
    out["lower"] = lo
    return out
