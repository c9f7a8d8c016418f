"""Batched Streamlined NTRU Prime key generation on AMD MI355X (gfx950).

Thin ctypes binding over ``libntrupkg.so`` (C ABI in ``include/ntrupkg.h``).
Only argument marshalling lives here: every step of key generation runs in
the library's HIP kernels.  torch provides device memory and streams.  The
library is required: importing works without it, but every call raises if
``libntrupkg.so`` is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libntrupkg.so")

PARAM_SETS = (653, 761, 857, 1277)

NTRUP_OK = 0
NTRUP_EIO = -5
NTRUP_EAGAIN = -11
NTRUP_ENOMEM = -12
NTRUP_EINVAL = -22
NTRUP_EFAULT = -14
NTRUP_ETIME = -62
NTRUP_ERANGE = -34
NOALLOC_SCRATCH_BYTES = 32 << 20   # the static scratch of ntrup_batch_keygen_noalloc


class NtrupError(RuntimeError):
    def __init__(self, code: int, what: str, hip_error: int = 0):
        self.code = code
        self.hip_error = hip_error
        msg = "%s failed: %s (%d)" % (what, strerror(code), code)
        if hip_error:
            msg += ", hipError %d" % hip_error
        super().__init__(msg)


class _Job(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("first_index", ctypes.c_uint64), ("n", ctypes.c_size_t),
                ("pk", ctypes.c_void_p), ("sk", ctypes.c_void_p),
                ("h", ctypes.c_void_p), ("f", ctypes.c_void_p), ("ginv", ctypes.c_void_p)]


class _Config(ctypes.Structure):
    _fields_ = [("group_size", ctypes.c_int), ("lanes_per_key", ctypes.c_int),
                ("retry_lanes_per_key", ctypes.c_int), ("retry_parallel_attempts", ctypes.c_int),
                ("retry_passes", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("product_engine", ctypes.c_int), ("inverse_share", ctypes.c_int),
                ("persistent", ctypes.c_int), ("r3_batch", ctypes.c_int), ("recip_jump", ctypes.c_int),
                ("group_form", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libntrupkg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libntrupkg.so not built (run __graft_entry__.build() or "
                          "python paper_2106_08759_amd/build.py); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint64
    sig = {
        "ntrup_params": (i32, [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(sz),
                               ctypes.POINTER(sz)]),
        "ntrup_ctx_create": (i32, [ctypes.POINTER(vp), i32, sz]),
        "ntrup_ctx_destroy": (i32, [vp]),
        "ntrup_ctx_reserve": (i32, [vp, i32, sz]),
        "ntrup_ctx_workspace_bytes": (sz, [vp]),
        "ntrup_workspace_bytes": (sz, [i32, sz]),
        "ntrup_last_hip_error": (i32, [vp]),
        "ntrup_strerror": (ctypes.c_char_p, [i32]),
        "ntrup_get_config": (i32, [vp, i32, ctypes.POINTER(_Config)]),
        "ntrup_set_config": (i32, [vp, i32, ctypes.POINTER(_Config)]),
        "ntrup_batch_keygen": (i32, [vp, i32, ctypes.c_char_p, u64, sz, vp, vp, vp, vp, vp, vp]),
        "ntrup_keygen_plain": (i32, [vp, i32, ctypes.c_char_p, u64, sz, vp, vp, vp]),
        "ntrup_batch_keygen_noalloc": (i32, [vp, i32, ctypes.c_char_p, u64, sz, vp, vp, vp, vp, vp, vp]),
        "ntrup_batch_keygen_mixed": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(_Job), sz, vp]),
        "ntrup_ctx_status": (i32, [vp, vp]),
        "ntrup_ctx_timing_begin": (i32, [vp, i32]),
        "ntrup_ctx_timing_end": (i32, [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]),
        "ntrup_op_mul_rq": (i32, [vp, i32, vp, vp, vp, sz, i32, vp]),
        "ntrup_op_mul_r3": (i32, [vp, i32, vp, vp, vp, sz, vp]),
        "ntrup_op_recip_rq": (i32, [vp, i32, vp, vp, vp, sz, vp]),
        "ntrup_op_recip_r3": (i32, [vp, i32, vp, vp, vp, sz, vp]),
        "ntrup_op_batch_inv_rq": (i32, [vp, i32, vp, vp, sz, sz, vp]),
        "ntrup_op_sample": (i32, [vp, i32, ctypes.c_char_p, u64, sz, i32, vp, vp, vp]),
        "ntrup_batch_encap": (i32, [vp, i32, ctypes.c_char_p, u64, sz, vp, vp, vp, vp]),
        "ntrup_batch_decap": (i32, [vp, i32, sz, vp, vp, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().ntrup_strerror(code).decode()
    except ImportError:
        return "error %d" % code


@dataclass(frozen=True)
class Params:
    p: int
    q: int
    w: int
    pk_bytes: int
    sk_bytes: int


def params(p: int) -> Params:
    q, w = ctypes.c_int(), ctypes.c_int()
    pkb, skb = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib().ntrup_params(p, ctypes.byref(q), ctypes.byref(w), ctypes.byref(pkb), ctypes.byref(skb))
    if rc:
        raise NtrupError(rc, "ntrup_params(%d)" % p)
    return Params(p, q.value, w.value, pkb.value, skb.value)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _seed_bytes(seed) -> bytes:
    b = bytes(seed)
    if len(b) != 32:
        raise ValueError("seed must be 32 bytes")
    return b


def workspace_bytes(p: int, n: int) -> int:
    """Device workspace a call of n keys of parameter set p needs."""
    return lib().ntrup_workspace_bytes(p, n)


def noalloc_max_keys(p: int) -> int:
    """Largest n that ntrup_batch_keygen_noalloc takes for parameter set p."""
    lo, hi = 0, 1 << 24
    while lo < hi:
        m = (lo + hi + 1) // 2
        if workspace_bytes(p, m) <= NOALLOC_SCRATCH_BYTES:
            lo = m
        else:
            hi = m - 1
    return lo


class Context:
    """A device context: workspace (at most workspace_budget bytes; 0 = no
    limit), tuned configuration, captured graphs."""

    def __init__(self, device: int = 0, workspace_budget: int = 0):
        import torch
        self.device = device
        self._torch = torch
        h = ctypes.c_void_p()
        rc = lib().ntrup_ctx_create(ctypes.byref(h), device, workspace_budget)
        if rc:
            raise NtrupError(rc, "ntrup_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ntrup_ctx_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc:
            raise NtrupError(rc, what, lib().ntrup_last_hip_error(self._h))

    def _empty(self, shape, dtype):
        return self._torch.empty(shape, dtype=dtype, device="cuda:%d" % self.device)

    # ---- configuration -----------------------------------------------------
    def get_config(self, p: int) -> dict:
        c = _Config()
        self._check(lib().ntrup_get_config(self._h, p, ctypes.byref(c)), "ntrup_get_config")
        return {"group_size": c.group_size, "lanes_per_key": c.lanes_per_key,
                "retry_lanes_per_key": c.retry_lanes_per_key,
                "retry_parallel_attempts": c.retry_parallel_attempts, "retry_passes": c.retry_passes,
                "use_graph": c.use_graph, "product_engine": c.product_engine,
                "inverse_share": c.inverse_share, "persistent": c.persistent, "r3_batch": c.r3_batch,
                "recip_jump": c.recip_jump, "group_form": c.group_form}

    def set_config(self, p: int, **kw):
        cur = self.get_config(p)
        cur.update(kw)
        c = _Config(cur["group_size"], cur["lanes_per_key"], cur["retry_lanes_per_key"],
                    cur["retry_parallel_attempts"], cur["retry_passes"], cur["use_graph"],
                    cur["product_engine"], cur["inverse_share"], cur["persistent"], cur["r3_batch"],
                    cur["recip_jump"], cur["group_form"])
        self._check(lib().ntrup_set_config(self._h, p, ctypes.byref(c)), "ntrup_set_config")

    def reserve(self, p: int, n: int):
        self._check(lib().ntrup_ctx_reserve(self._h, p, n), "ntrup_ctx_reserve")

    def workspace_bytes(self) -> int:
        return lib().ntrup_ctx_workspace_bytes(self._h)

    STAGES = ("sample_short", "r3_main", "r3_retry", "group_prefix", "group_back", "fused")

    def timing_begin(self, max_pipelines: int):
        self._check(lib().ntrup_ctx_timing_begin(self._h, max_pipelines), "timing_begin")

    def timing_end(self):
        """-> (dict stage -> summed ms, number of pipelines timed)"""
        ms = (ctypes.c_double * len(self.STAGES))()
        cnt = ctypes.c_int()
        self._check(lib().ntrup_ctx_timing_end(self._h, ms, len(self.STAGES), ctypes.byref(cnt)), "timing_end")
        return dict(zip(self.STAGES, list(ms))), cnt.value

    def status(self, stream=None) -> int:
        return lib().ntrup_ctx_status(self._h, _stream(stream))

    # ---- key generation ----------------------------------------------------
    def _raw(self, p: int, n: int):
        t = self._torch
        return (self._empty((n, p), t.int16), self._empty((n, p), t.int8), self._empty((n, p), t.int8))

    def batch_keygen(self, p: int, seed, first_index: int, n: int, pk=None, sk=None,
                     stream=None, check: bool = True, plain: bool = False, raw: bool = False):
        """Keys first_index..first_index+n-1: returns (pk, sk) uint8 device tensors
        of shape [n, pk_bytes] and [n, sk_bytes]; with raw=True also the raw
        centered arrays h (int16), f and 1/g (int8), each [n, p] (raw may also be
        a tuple of three such tensors to write into)."""
        prm = params(p)
        if pk is None:
            pk = self._empty((n, prm.pk_bytes), self._torch.uint8)
        if sk is None:
            sk = self._empty((n, prm.sk_bytes), self._torch.uint8)
        assert pk.is_contiguous() and sk.is_contiguous()
        assert pk.numel() >= n * prm.pk_bytes and sk.numel() >= n * prm.sk_bytes
        if plain:
            assert not raw, "the plain form has no raw outputs"
            rc = lib().ntrup_keygen_plain(self._h, p, _seed_bytes(seed), first_index, n, _ptr(pk), _ptr(sk),
                                          _stream(stream))
            arrays = ()
        else:
            arrays = tuple(raw) if isinstance(raw, (tuple, list)) else self._raw(p, n) if raw else ()
            for a_, dt in zip(arrays, (self._torch.int16, self._torch.int8, self._torch.int8)):
                assert a_.is_contiguous() and a_.dtype == dt and a_.numel() >= n * p
            rp = [_ptr(a) for a in arrays] if raw else [None, None, None]
            rc = lib().ntrup_batch_keygen(self._h, p, _seed_bytes(seed), first_index, n, _ptr(pk), _ptr(sk),
                                          rp[0], rp[1], rp[2], _stream(stream))
        self._check(rc, "keygen")
        if check:
            self._check(self.status(stream), "keygen status")
        return (pk, sk) + tuple(arrays)

    def batch_keygen_noalloc(self, p: int, seed, first_index: int, n: int, pk, sk, raw=None, stream=None,
                             check: bool = True):
        """ntrup_batch_keygen_noalloc: the keys of batch_keygen with the
        library's static scratch as workspace (nothing allocated by the call).
        pk, sk (and raw = (h, f, ginv), optional) are caller-allocated device
        tensors."""
        prm = params(p)
        assert pk.is_contiguous() and sk.is_contiguous()
        assert pk.numel() >= n * prm.pk_bytes and sk.numel() >= n * prm.sk_bytes
        rp = [_ptr(a) for a in raw] if raw is not None else [None, None, None]
        self._check(lib().ntrup_batch_keygen_noalloc(self._h, p, _seed_bytes(seed), first_index, n, _ptr(pk),
                                                     _ptr(sk), rp[0], rp[1], rp[2], _stream(stream)),
                    "keygen_noalloc")
        if check:
            self._check(self.status(stream), "keygen status")
        return pk, sk

    def keygen_plain(self, p: int, seed, first_index: int, n: int, **kw):
        return self.batch_keygen(p, seed, first_index, n, plain=True, **kw)

    def batch_keygen_mixed(self, seed, jobs, stream=None, check: bool = True, raw: bool = False):
        """jobs: list of (p, first_index, n).  Returns a list of (pk, sk), or of
        (pk, sk, h, f, ginv) with raw=True."""
        outs, arr = [], (_Job * len(jobs))()
        for i, (p, first, n) in enumerate(jobs):
            prm = params(p)
            pk = self._empty((n, prm.pk_bytes), self._torch.uint8)
            sk = self._empty((n, prm.sk_bytes), self._torch.uint8)
            arrays = self._raw(p, n) if raw else ()
            outs.append((pk, sk) + tuple(arrays))
            rp = [_ptr(a) for a in arrays] if raw else [None, None, None]
            arr[i] = _Job(p, first, n, _ptr(pk), _ptr(sk), rp[0], rp[1], rp[2])
        self._check(lib().ntrup_batch_keygen_mixed(self._h, _seed_bytes(seed), arr, len(jobs),
                                                   _stream(stream)), "keygen_mixed")
        if check:
            self._check(self.status(stream), "keygen status")
        return outs

    # ---- encapsulation / decapsulation core ------------------------------------
    def _rows(self, t, n: int, p: int, dtype, what: str):
        if t is None:
            return None
        if tuple(t.shape) != (n, p) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous device tensor [%d, %d] of %s" % (what, n, p, dtype))
        return t

    def batch_encap(self, p: int, seed, first_index: int, h, c=None, r=None, stream=None):
        """(c, r): r_i in Short from the encapsulation stream of key
        first_index + i, c_i = Round(h_i r_i) in R/q (h: int16 [n, p])."""
        T = self._torch
        n = h.shape[0]
        self._rows(h, n, p, T.int16, "h")
        c = self._rows(c, n, p, T.int16, "c") if c is not None else self._empty((n, p), T.int16)
        r = self._rows(r, n, p, T.int8, "r") if r is not None else self._empty((n, p), T.int8)
        self._check(lib().ntrup_batch_encap(self._h, p, _seed_bytes(seed), first_index, n, _ptr(h), _ptr(c),
                                            _ptr(r), _stream(stream)), "batch_encap")
        return c, r

    def batch_decap(self, p: int, c, f, ginv, h=None, r=None, ok=None, stream=None):
        """(r', ok): r' = decrypt(c) with the weight check; ok = 1 iff
        Round(h r') = c (with h) or r' had weight w (without)."""
        T = self._torch
        n = c.shape[0]
        self._rows(c, n, p, T.int16, "c")
        self._rows(f, n, p, T.int8, "f")
        self._rows(ginv, n, p, T.int8, "ginv")
        self._rows(h, n, p, T.int16, "h")
        r = self._rows(r, n, p, T.int8, "r") if r is not None else self._empty((n, p), T.int8)
        if ok is None:
            ok = self._empty((n,), T.uint8)
        elif tuple(ok.shape) != (n,) or ok.dtype != T.uint8 or not ok.is_cuda:
            raise ValueError("ok must be a device tensor [%d] of uint8" % n)
        self._check(lib().ntrup_batch_decap(self._h, p, n, _ptr(c), _ptr(f), _ptr(ginv), _ptr(h), _ptr(r),
                                            _ptr(ok), _stream(stream)), "batch_decap")
        return r, ok

    # ---- single operations ---------------------------------------------------
    def mul_rq(self, p: int, a, b, small_a: bool = False, stream=None):
        n = a.shape[0]
        c = self._empty((n, p), self._torch.int16)
        self._check(lib().ntrup_op_mul_rq(self._h, p, _ptr(a), _ptr(b), _ptr(c), n, int(small_a),
                                          _stream(stream)), "op_mul_rq")
        return c

    def mul_r3(self, p: int, a, b, stream=None):
        """c = a * b in R/3 for int8 rows with coefficients in {-1, 0, 1}."""
        n = a.shape[0]
        c = self._empty((n, p), self._torch.int8)
        self._check(lib().ntrup_op_mul_r3(self._h, p, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "op_mul_r3")
        return c

    def recip_rq(self, p: int, a, stream=None):
        n = a.shape[0]
        out = self._empty((n, p), self._torch.int16)
        ok = self._empty((n,), self._torch.int32)
        self._check(lib().ntrup_op_recip_rq(self._h, p, _ptr(a), _ptr(out), _ptr(ok), n,
                                            _stream(stream)), "op_recip_rq")
        return out, ok

    def recip_r3(self, p: int, a, stream=None):
        n = a.shape[0]
        out = self._empty((n, p), self._torch.int8)
        ok = self._empty((n,), self._torch.int32)
        self._check(lib().ntrup_op_recip_r3(self._h, p, _ptr(a), _ptr(out), _ptr(ok), n,
                                            _stream(stream)), "op_recip_r3")
        return out, ok

    def batch_inv_rq(self, p: int, a, group_size: int, stream=None):
        n = a.shape[0]
        out = self._empty((n, p), self._torch.int16)
        self._check(lib().ntrup_op_batch_inv_rq(self._h, p, _ptr(a), _ptr(out), n, group_size,
                                                _stream(stream)), "op_batch_inv_rq")
        return out

    def sample(self, p: int, seed, first_index: int, n: int, attempt: int = 0, stream=None):
        f = self._empty((n, p), self._torch.int8)
        g = self._empty((n, p), self._torch.int8)
        self._check(lib().ntrup_op_sample(self._h, p, _seed_bytes(seed), first_index, n, attempt,
                                          _ptr(f), _ptr(g), _stream(stream)), "op_sample")
        return f, g


# ---- host-side decoding of the library's key encodings (format helpers) ----

def decode_pk(pk, p: int):
    """pk bytes [n, pk_bytes] (numpy or torch) -> h int16 [n, p] centered."""
    import numpy as np
    prm = params(p)
    a = np.asarray(pk.cpu() if hasattr(pk, "cpu") else pk, dtype=np.uint8).reshape(-1, prm.pk_bytes)
    bits = np.unpackbits(a, axis=1, bitorder="little")[:, : 13 * p].reshape(-1, p, 13)
    vals = (bits.astype(np.int32) << np.arange(13, dtype=np.int32)).sum(axis=2)
    return (vals - (prm.q - 1) // 2).astype(np.int16)


def decode_sk(sk, p: int):
    """sk bytes [n, sk_bytes] -> (f, ginv) int8 [n, p] each."""
    import numpy as np
    prm = params(p)
    a = np.asarray(sk.cpu() if hasattr(sk, "cpu") else sk, dtype=np.uint8).reshape(-1, prm.sk_bytes)
    half = prm.sk_bytes // 2

    def trits(b):
        bits = np.unpackbits(b, axis=1, bitorder="little")[:, : 2 * p].reshape(-1, p, 2)
        return (bits[:, :, 0].astype(np.int8) + 2 * bits[:, :, 1].astype(np.int8) - 1)

    return trits(a[:, :half]), trits(a[:, half:])
