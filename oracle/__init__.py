"""CPU oracle for Streamlined NTRU Prime key generation -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it; the two share no code.  See ``ntrup_oracle.c`` for what is computed
(OpenSSLNTRU paper, Section 3.1 KeyGen, on the rings of Section 2.1), the
sampling/encoding conventions and the encapsulation / decapsulation core.

Every function here is pinned by ``tests/test_oracle_*.py`` against things the
paper and mathematics fix (brute force on toy rings, library routines, closed
forms), not against itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntrup_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# Parameter sets (p, q, w): Section 2.1 for 653/761/857; sntrup1277 uses the
# round-3 values q=7879, w=492 (the paper names p=1277 without q and w).
PARAMS = {
    653: (653, 4621, 288),
    761: (761, 4591, 286),
    857: (857, 5167, 322),
    1277: (1277, 7879, 492),
}
MAX_ATTEMPTS = 64


def build(force: bool = False) -> str:
    """Compile the oracle with plain gcc -O2 (no intrinsics)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i8p = ctypes.POINTER(ctypes.c_int8)
        i16p = ctypes.POINTER(ctypes.c_int16)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_chacha20_block.argtypes = [u8p, ctypes.c_uint32, u8p, u8p]
        L.oracle_chacha20_block.restype = None
        L.oracle_stream_words.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_int, u32p, ctypes.c_int]
        L.oracle_stream_words.restype = None
        L.oracle_sample_small.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_int, i8p]
        L.oracle_sample_short.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_int, i8p]
        L.oracle_mul_mod.argtypes = [i64p, i64p, ctypes.c_int, ctypes.c_int64, i64p]
        L.oracle_mul_mod.restype = None
        L.oracle_inv_mod.argtypes = [i64p, ctypes.c_int, ctypes.c_int64, i64p]
        L.oracle_keygen.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_uint64, i8p, i8p, i8p, i16p,
                                    ctypes.POINTER(ctypes.c_int)]
        L.oracle_encode_pk.argtypes = [i16p, ctypes.c_int, ctypes.c_int, u8p]
        L.oracle_encode_pk.restype = None
        L.oracle_encode_sk.argtypes = [i8p, i8p, ctypes.c_int, u8p]
        L.oracle_encode_sk.restype = None
        L.oracle_keygen_range.argtypes = [u8p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_uint64,
                                          ctypes.c_long,
                                          ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_keygen_range.restype = ctypes.c_long
        L.oracle_sample_short_stream.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int, i8p]
        L.oracle_encrypt.argtypes = [i16p, i8p, ctypes.c_int, ctypes.c_int, i16p]
        L.oracle_decrypt.argtypes = [i16p, i8p, i8p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, i8p]
        L.oracle_encap.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_uint64, i16p, i16p, i8p]
        L.oracle_decap.argtypes = [i16p, i8p, i8p, i16p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, i8p]
        _lib = L
    return _lib


def _ptr(arr: np.ndarray, ctype):
    assert arr.flags["C_CONTIGUOUS"]
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def _seed(seed) -> np.ndarray:
    s = np.frombuffer(bytes(seed), dtype=np.uint8).copy()
    if s.size != 32:
        raise ValueError("seed must be 32 bytes")
    return s


def chacha20_block(key: bytes, counter: int, nonce: bytes) -> bytes:
    k = _seed(key)
    n = np.frombuffer(bytes(nonce), dtype=np.uint8).copy()
    assert n.size == 12
    out = np.zeros(64, dtype=np.uint8)
    lib().oracle_chacha20_block(_ptr(k, ctypes.c_uint8), counter & 0xFFFFFFFF,
                                _ptr(n, ctypes.c_uint8), _ptr(out, ctypes.c_uint8))
    return out.tobytes()


def stream_words(seed, index: int, p: int, stream: int, nwords: int) -> np.ndarray:
    out = np.zeros(nwords, dtype=np.uint32)
    lib().oracle_stream_words(_ptr(_seed(seed), ctypes.c_uint8), index, p, stream,
                              _ptr(out, ctypes.c_uint32), nwords)
    return out


def sample_small(seed, index: int, p: int, attempt: int) -> np.ndarray:
    g = np.zeros(p, dtype=np.int8)
    rc = lib().oracle_sample_small(_ptr(_seed(seed), ctypes.c_uint8), index, p,
                                   attempt, _ptr(g, ctypes.c_int8))
    assert rc == 0
    return g


def sample_short(seed, index: int, p: int, w: int, stream: int = 0) -> np.ndarray:
    f = np.zeros(p, dtype=np.int8)
    rc = lib().oracle_sample_short_stream(_ptr(_seed(seed), ctypes.c_uint8), index, p, w,
                                          stream, _ptr(f, ctypes.c_int8))
    assert rc == 0
    return f


def mul_mod(a, b, p: int, m: int) -> np.ndarray:
    """a*b in F_m[x]/(x^p - x - 1), result in [0, m)."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    assert a.size == p and b.size == p
    out = np.zeros(p, dtype=np.int64)
    lib().oracle_mul_mod(_ptr(a, ctypes.c_int64), _ptr(b, ctypes.c_int64), p, m,
                         _ptr(out, ctypes.c_int64))
    return out


def inv_mod(a, p: int, m: int):
    """1/a in F_m[x]/(x^p - x - 1) as values in [0, m), or None if a is not a unit."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    assert a.size == p
    out = np.zeros(p, dtype=np.int64)
    rc = lib().oracle_inv_mod(_ptr(a, ctypes.c_int64), p, m, _ptr(out, ctypes.c_int64))
    if rc < 0:
        raise RuntimeError("oracle_inv_mod failed: %d" % rc)
    return out if rc == 1 else None


def keygen(seed, p: int, index: int, q: int | None = None, w: int | None = None):
    """One key pair.  Returns dict with f, g, ginv (int8), h (int16), attempts."""
    if q is None or w is None:
        _, q, w = PARAMS[p]
    f = np.zeros(p, dtype=np.int8)
    g = np.zeros(p, dtype=np.int8)
    ginv = np.zeros(p, dtype=np.int8)
    h = np.zeros(p, dtype=np.int16)
    att = ctypes.c_int(0)
    rc = lib().oracle_keygen(_ptr(_seed(seed), ctypes.c_uint8), p, q, w, index,
                             _ptr(f, ctypes.c_int8), _ptr(g, ctypes.c_int8),
                             _ptr(ginv, ctypes.c_int8), _ptr(h, ctypes.c_int16),
                             ctypes.byref(att))
    if rc != 0:
        raise RuntimeError("oracle_keygen failed: %d" % rc)
    return {"f": f, "g": g, "ginv": ginv, "h": h, "attempts": att.value}


def pk_bytes(p: int) -> int:
    return (13 * p + 7) // 8


def sk_bytes(p: int) -> int:
    return 2 * ((p + 3) // 4)


def encode_pk(h, p: int, q: int) -> bytes:
    h = np.ascontiguousarray(h, dtype=np.int16)
    out = np.zeros(pk_bytes(p), dtype=np.uint8)
    lib().oracle_encode_pk(_ptr(h, ctypes.c_int16), p, q, _ptr(out, ctypes.c_uint8))
    return out.tobytes()


def encode_sk(f, ginv, p: int) -> bytes:
    f = np.ascontiguousarray(f, dtype=np.int8)
    gi = np.ascontiguousarray(ginv, dtype=np.int8)
    out = np.zeros(sk_bytes(p), dtype=np.uint8)
    lib().oracle_encode_sk(_ptr(f, ctypes.c_int8), _ptr(gi, ctypes.c_int8), p,
                           _ptr(out, ctypes.c_uint8))
    return out.tobytes()


def keygen_range(seed, p: int, index0: int, n: int) -> int:
    """Generate keys index0..index0+n-1 (CPU-baseline timing); returns a checksum."""
    _, q, w = PARAMS[p]
    cs = ctypes.c_uint64(0)
    done = lib().oracle_keygen_range(_ptr(_seed(seed), ctypes.c_uint8), p, q, w,
                                     index0, n, ctypes.byref(cs))
    if done != n:
        raise RuntimeError("oracle_keygen_range failed: %d" % done)
    return cs.value


# Encapsulation / decapsulation core (see ntrup_oracle.c: Streamlined NTRU
# Prime's published encryption, restated; the session-key hashes are not
# computed).  r of key `index` comes from this stream of the Short sampler.
ENCAP_STREAM = 0x8000


def encrypt(h, r, p: int) -> np.ndarray:
    """c = Round(h r) in R/q, centered (every c_i a multiple of 3)."""
    _, q, _ = PARAMS[p]
    h = np.ascontiguousarray(h, dtype=np.int16)
    r = np.ascontiguousarray(r, dtype=np.int8)
    c = np.zeros(p, dtype=np.int16)
    rc = lib().oracle_encrypt(_ptr(h, ctypes.c_int16), _ptr(r, ctypes.c_int8), p, q,
                              _ptr(c, ctypes.c_int16))
    assert rc == 0
    return c


def decrypt(c, f, ginv, p: int):
    """(r', weight_ok): r' = (3 f c mod q, mod 3) (1/g) in R/3, replaced by
    (1,..,1,0,..,0) when its weight is not w."""
    _, q, w = PARAMS[p]
    c = np.ascontiguousarray(c, dtype=np.int16)
    f = np.ascontiguousarray(f, dtype=np.int8)
    gi = np.ascontiguousarray(ginv, dtype=np.int8)
    r = np.zeros(p, dtype=np.int8)
    rc = lib().oracle_decrypt(_ptr(c, ctypes.c_int16), _ptr(f, ctypes.c_int8),
                              _ptr(gi, ctypes.c_int8), p, q, w, _ptr(r, ctypes.c_int8))
    assert rc in (0, 1)
    return r, bool(rc)


def encap(seed, p: int, index: int, h):
    """(c, r) of the encapsulation core for key `index` and public key h."""
    _, q, w = PARAMS[p]
    h = np.ascontiguousarray(h, dtype=np.int16)
    c = np.zeros(p, dtype=np.int16)
    r = np.zeros(p, dtype=np.int8)
    rc = lib().oracle_encap(_ptr(_seed(seed), ctypes.c_uint8), p, q, w, index,
                            _ptr(h, ctypes.c_int16), _ptr(c, ctypes.c_int16),
                            _ptr(r, ctypes.c_int8))
    assert rc == 0
    return c, r


def decap(c, f, ginv, p: int, h=None):
    """(r', ok) of the decapsulation core; with h, ok means encrypt(r', h) = c,
    without, that r' had weight w."""
    _, q, w = PARAMS[p]
    c = np.ascontiguousarray(c, dtype=np.int16)
    f = np.ascontiguousarray(f, dtype=np.int8)
    gi = np.ascontiguousarray(ginv, dtype=np.int8)
    r = np.zeros(p, dtype=np.int8)
    hp = None
    if h is not None:
        h = np.ascontiguousarray(h, dtype=np.int16)
        hp = _ptr(h, ctypes.c_int16)
    rc = lib().oracle_decap(_ptr(c, ctypes.c_int16), _ptr(f, ctypes.c_int8),
                            _ptr(gi, ctypes.c_int8), hp, p, q, w, _ptr(r, ctypes.c_int8))
    assert rc in (0, 1)
    return r, bool(rc)
