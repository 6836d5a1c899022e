"""ctypes marshalling for the plain-C oracle (test infrastructure only).

Every function here converts numpy arrays and forwards to ``rdhei_oracle.c``;
the arithmetic is in the C file.  The library is built with gcc into
``oracle/_build/`` on first use (or by ``build_oracle()``).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rdhei_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "librdhei_oracle.so")
_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, -O2, no SIMD intrinsics)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build_oracle())
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.or_keystream.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u8p]
    lib.or_chacha20_block.argtypes = [u32p, ctypes.c_uint32, u32p, u8p]
    lib.or_set_keystream.argtypes = [ctypes.c_int]
    lib.or_location_map.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, u8p]
    lib.or_location_map.restype = ctypes.c_int64
    lib.or_redundancy_counts.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_int, i64p]
    lib.or_select_b.argtypes = [i64p, ctypes.c_int, ctypes.c_int]
    lib.or_select_b.restype = ctypes.c_int
    lib.or_max_level.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.or_max_level.restype = ctypes.c_int
    lib.or_rotate.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, u8p, ctypes.c_int, ctypes.c_int]
    lib.or_emr_encrypt.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, u8p,
                                   ctypes.c_void_p]
    lib.or_emr_embed.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, u8p, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_uint64]
    lib.or_emr_embed.restype = ctypes.c_int64
    lib.or_emr_extract.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, u8p, ctypes.c_int64,
                                   ctypes.c_uint64, ctypes.c_uint64]
    lib.or_emr_extract.restype = ctypes.c_int64
    lib.or_emr_recover.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u8p]
    lib.or_lmr_rotated_maps.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.c_uint64, u8p, u8p]
    lib.or_lmr_encrypt.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.c_uint64, u8p, ctypes.c_int64, u8p]
    lib.or_lmr_embed.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, u8p, u8p,
                                 ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
    lib.or_lmr_embed.restype = ctypes.c_int64
    lib.or_lmr_extract.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, u8p, u8p,
                                   ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
    lib.or_lmr_extract.restype = ctypes.c_int64
    lib.or_lmr_recover.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_uint64, ctypes.c_uint64, u8p, u8p, u8p]
    lib.or_plane_encode.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, u8p, ctypes.c_int64]
    lib.or_plane_encode.restype = ctypes.c_int64
    lib.or_plane_decode.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, u8p]
    lib.or_lmr_compress.argtypes = [u8p, u8p, ctypes.c_int32, ctypes.c_int32, u8p, ctypes.c_int64]
    lib.or_lmr_compress.restype = ctypes.c_int64
    lib.or_lmr_decompress.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, u8p, u8p]
    lib.or_lmr_encode.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, u8p,
                                  ctypes.c_void_p, u8p, ctypes.POINTER(ctypes.c_int64)]
    lib.or_demr_tile_b.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, u8p, i64p]
    lib.or_demr_encrypt.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, u8p, u8p,
                                    ctypes.c_void_p]
    lib.or_demr_encrypt.restype = ctypes.c_int
    lib.or_demr_embed.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, u8p, u8p, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_uint64]
    lib.or_demr_embed.restype = ctypes.c_int64
    lib.or_demr_extract.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, u8p, u8p, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_uint64]
    lib.or_demr_extract.restype = ctypes.c_int64
    lib.or_demr_recover.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, u8p, ctypes.c_uint64, ctypes.c_uint64, u8p]
    _lib = lib
    return lib


class _OrMeta(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("min_level", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("redundant", ctypes.c_int64), ("capacity_bits", ctypes.c_int64)]


@dataclass
class OracleMeta:
    b: int
    min_level: int
    max_level: int
    redundant: int
    capacity_bits: int


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _img(I) -> np.ndarray:
    I = np.ascontiguousarray(np.asarray(I), dtype=np.uint8)
    assert I.ndim == 2
    return I


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    P = ctypes.POINTER(ctypes.c_uint32)
    lib.or_philox4x32_10(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def chacha20_block(key_words, counter: int, nonce_words) -> np.ndarray:
    """The 64 output bytes of the ChaCha20 block function."""
    lib = _load()
    k = np.ascontiguousarray(key_words, dtype=np.uint32)
    n = np.ascontiguousarray(nonce_words, dtype=np.uint32)
    assert k.size == 8 and n.size == 3
    out = np.zeros(64, dtype=np.uint8)
    P = ctypes.POINTER(ctypes.c_uint32)
    lib.or_chacha20_block(k.ctypes.data_as(P), counter, n.ctypes.data_as(P), _u8(out))
    return out


KEYSTREAM_PHILOX = 0
KEYSTREAM_CHACHA20 = 1


@contextlib.contextmanager
def keystream_family(family: int):
    """Every oracle call inside the block draws its keystreams from `family`
    (KEYSTREAM_PHILOX or KEYSTREAM_CHACHA20); Philox again afterwards."""
    assert family in (KEYSTREAM_PHILOX, KEYSTREAM_CHACHA20)
    lib = _load()
    lib.or_set_keystream(family)
    try:
        yield
    finally:
        lib.or_set_keystream(KEYSTREAM_PHILOX)


def keystream(key: int, domain: int, first: int, count: int, nonce: int = 0) -> np.ndarray:
    """Bytes [first, first + count) of the stream (key, nonce, domain)."""
    out = np.zeros(max(count, 1), dtype=np.uint8)
    _load().or_keystream(key, nonce, domain, first, count, _u8(out))
    return out[:count]


def location_map(I, b: int):
    I = _img(I)
    L = np.zeros(I.shape, dtype=np.uint8)
    z = _load().or_location_map(_u8(I), I.shape[0], I.shape[1], b, _u8(L))
    return L, int(z)


def redundancy_counts(I, bmin: int, bmax: int) -> np.ndarray:
    I = _img(I)
    Z = np.zeros(bmax - bmin + 1, dtype=np.int64)
    _load().or_redundancy_counts(_u8(I), I.shape[0], I.shape[1], bmin, bmax,
                                 Z.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return Z


def select_b(Z, bmin: int) -> int:
    Z = np.ascontiguousarray(Z, dtype=np.int64)
    return int(_load().or_select_b(Z.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), bmin, bmin + len(Z) - 1))


def max_level(M: int, N: int) -> int:
    return int(_load().or_max_level(M, N))


def rotate(X, s, min_level: int = 1, inverse: bool = False) -> np.ndarray:
    X = _img(X).copy()
    s = _img(s)
    assert s.shape == X.shape
    _load().or_rotate(_u8(X), X.shape[0], X.shape[1], _u8(s), min_level, 1 if inverse else 0)
    return X


def image_keystream(k1: int, M: int, N: int, nonce: int = 0) -> np.ndarray:
    return keystream(k1, 1, 0, M * N, nonce).reshape(M, N)


def emr_encrypt(I, k1: int, nonce: int = 0):
    I = _img(I)
    Ie = np.zeros_like(I)
    m = _OrMeta()
    _load().or_emr_encrypt(_u8(I), I.shape[0], I.shape[1], k1, nonce, _u8(Ie), ctypes.byref(m))
    return Ie, OracleMeta(m.b, m.min_level, m.max_level, m.redundant, m.capacity_bits)


def _msg_buf(nbits: int) -> np.ndarray:
    return np.zeros(max((nbits + 7) // 8, 1), dtype=np.uint8)


def emr_embed(Ie, b: int, msg: np.ndarray, nbits: int, k2: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie).copy()
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    if msg.size == 0:
        msg = _msg_buf(0)
    r = _load().or_emr_embed(_u8(X), X.shape[0], X.shape[1], b, _u8(msg), nbits, k2, nonce)
    if r < 0:
        raise ValueError("message longer than capacity")
    return X


def emr_extract(Ie, b: int, nbits: int, k2: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie)
    out = _msg_buf(nbits)
    _load().or_emr_extract(_u8(X), X.shape[0], X.shape[1], b, _u8(out), nbits, k2, nonce)
    return out[:(nbits + 7) // 8]


def emr_recover(Ie, b: int, k1: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie)
    out = np.zeros_like(X)
    _load().or_emr_recover(_u8(X), X.shape[0], X.shape[1], b, k1, nonce, _u8(out))
    return out


def lmr_rotated_maps(I, b: int, min_level: int, k1: int, nonce: int = 0):
    I = _img(I)
    l_rot = np.zeros_like(I)
    eta_rot = np.zeros_like(I)
    _load().or_lmr_rotated_maps(_u8(I), I.shape[0], I.shape[1], b, min_level, k1, nonce, _u8(l_rot),
                                _u8(eta_rot))
    return l_rot, eta_rot


def lmr_encrypt(I, min_level: int, k1: int, stream: np.ndarray, stream_bits: int, nonce: int = 0) -> np.ndarray:
    I = _img(I)
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    if stream.size == 0:
        stream = _msg_buf(0)
    Ie = np.zeros_like(I)
    _load().or_lmr_encrypt(_u8(I), I.shape[0], I.shape[1], min_level, k1, nonce, _u8(stream), stream_bits,
                           _u8(Ie))
    return Ie


def lmr_embed(Ie, b: int, l_rot, msg, nbits: int, k2: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie).copy()
    l_rot = _img(l_rot)
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    if msg.size == 0:
        msg = _msg_buf(0)
    r = _load().or_lmr_embed(_u8(X), X.shape[0], X.shape[1], b, _u8(l_rot), _u8(msg), nbits, k2, nonce)
    if r < 0:
        raise ValueError("message longer than capacity")
    return X


def lmr_extract(Ie, b: int, l_rot, nbits: int, k2: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie)
    l_rot = _img(l_rot)
    out = _msg_buf(nbits)
    _load().or_lmr_extract(_u8(X), X.shape[0], X.shape[1], b, _u8(l_rot), _u8(out), nbits, k2, nonce)
    return out[:(nbits + 7) // 8]


def lmr_recover(Ie, b: int, min_level: int, k1: int, l_rot, eta_rot, nonce: int = 0) -> np.ndarray:
    X = _img(Ie)
    out = np.zeros_like(X)
    _load().or_lmr_recover(_u8(X), X.shape[0], X.shape[1], b, min_level, k1, nonce,
                           _u8(_img(l_rot)), _u8(_img(eta_rot)), _u8(out))
    return out


def plane_encode(P, cap: int = -1) -> np.ndarray:
    """Bi-level coder: one byte (0/1) per pixel in, bytes out (None if > cap)."""
    P = _img(P)
    cap = cap if cap >= 0 else 16 + 2 * P.size
    out = np.zeros(cap + 1, dtype=np.uint8)
    n = _load().or_plane_encode(_u8(P), P.shape[0], P.shape[1], _u8(out), cap)
    return None if n < 0 else out[:n].copy()


def plane_decode(stream, M: int, N: int) -> np.ndarray:
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    out = np.zeros((M, N), dtype=np.uint8)
    _load().or_plane_decode(_u8(s), int(np.asarray(stream).size), M, N, _u8(out))
    return out


def lmr_compress(eta_rot, l_rot, cap: int):
    """Container of both maps (bytes) or None when longer than cap bytes."""
    eta_rot, l_rot = _img(eta_rot), _img(l_rot)
    out = np.zeros(max(cap, 8) + 1, dtype=np.uint8)
    n = _load().or_lmr_compress(_u8(eta_rot), _u8(l_rot), eta_rot.shape[0], eta_rot.shape[1], _u8(out), cap)
    return None if n < 0 else out[:n].copy()


def lmr_decompress(stream, M: int, N: int):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    eta = np.zeros((M, N), dtype=np.uint8)
    l = np.zeros((M, N), dtype=np.uint8)
    rc = _load().or_lmr_decompress(_u8(s), s.size, M, N, _u8(eta), _u8(l))
    if rc != 0:
        raise ValueError("malformed LMR stream")
    return eta, l


def lmr_encode(I, k1: int, min_level: int = 4, nonce: int = 0):
    """Full LMR encoding with rotation blocks 2^min_level..2^n: (I_e, meta,
    stream bytes) or (None, meta, None) for a bad case."""
    I = _img(I)
    M, N = I.shape
    Ie = np.zeros_like(I)
    m = _OrMeta()
    stream = np.zeros(M * N // 8 + 16, dtype=np.uint8)
    bits = ctypes.c_int64()
    rc = _load().or_lmr_encode(_u8(I), M, N, k1, nonce, min_level, _u8(Ie), ctypes.byref(m), _u8(stream),
                               ctypes.byref(bits))
    meta = OracleMeta(m.b, m.min_level, m.max_level, m.redundant, m.capacity_bits)
    if rc != 0:
        return None, meta, None
    return Ie, meta, stream[: bits.value // 8].copy()


# ---- dynamic b: one b per 64x64 tile (the conclusion's future work; reading in rdhei_oracle.c)
DEMR_TILE = 64


def demr_tile_b(I):
    """(b_t as a (M/64, N/64) uint8 array, Z_b(t) as (M/64, N/64, 6) for b = 2..7)."""
    I = _img(I)
    M, N = I.shape
    assert M % DEMR_TILE == 0 and N % DEMR_TILE == 0
    tb = np.zeros((M // DEMR_TILE, N // DEMR_TILE), dtype=np.uint8)
    Z = np.zeros((M // DEMR_TILE, N // DEMR_TILE, 6), dtype=np.int64)
    _load().or_demr_tile_b(_u8(I), M, N, _u8(tb), Z.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return tb, Z


def demr_encrypt(I, k1: int, nonce: int = 0):
    """(I_e, meta with b = 0, b table in encrypted-tile order)."""
    I = _img(I)
    M, N = I.shape
    assert M % DEMR_TILE == 0 and N % DEMR_TILE == 0
    Ie = np.zeros_like(I)
    bt = np.zeros((M // DEMR_TILE, N // DEMR_TILE), dtype=np.uint8)
    m = _OrMeta()
    rc = _load().or_demr_encrypt(_u8(I), M, N, k1, nonce, _u8(Ie), _u8(bt), ctypes.byref(m))
    assert rc == 0, "rotated b map not constant on an encrypted tile"
    return Ie, OracleMeta(m.b, m.min_level, m.max_level, m.redundant, m.capacity_bits), bt


def demr_embed(Ie, btab, msg, nbits: int, k2: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie).copy()
    bt = np.ascontiguousarray(btab, dtype=np.uint8)
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    if msg.size == 0:
        msg = _msg_buf(0)
    r = _load().or_demr_embed(_u8(X), X.shape[0], X.shape[1], _u8(bt), _u8(msg), nbits, k2, nonce)
    if r < 0:
        raise ValueError("message longer than capacity")
    return X


def demr_extract(Ie, btab, nbits: int, k2: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie)
    bt = np.ascontiguousarray(btab, dtype=np.uint8)
    out = _msg_buf(nbits)
    _load().or_demr_extract(_u8(X), X.shape[0], X.shape[1], _u8(bt), _u8(out), nbits, k2, nonce)
    return out[:(nbits + 7) // 8]


def demr_recover(Ie, btab, k1: int, nonce: int = 0) -> np.ndarray:
    X = _img(Ie)
    bt = np.ascontiguousarray(btab, dtype=np.uint8)
    out = np.zeros_like(X)
    _load().or_demr_recover(_u8(X), X.shape[0], X.shape[1], _u8(bt), k1, nonce, _u8(out))
    return out


def psnr(a, b) -> float:
    """PSNR in dB for 8-bit images (infinite when identical)."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    mse = float(np.mean(d * d))
    if mse == 0.0:
        return float("inf")
    return 10.0 * np.log10(255.0 ** 2 / mse)


__all__ = [n for n in dir() if not n.startswith("_")]
