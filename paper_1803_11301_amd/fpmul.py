"""Thin Python binding of libfpmul.so (C ABI in include/fpmul.h).

Argument marshalling only: every step of a product runs in the HIP kernels
of the library.  Word arrays live on the GPU as torch ``int64`` tensors (bit
patterns of the uint64 words); torch is used for device memory and streams.
If the library is missing, every call raises: there is no other code path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpmul.so")

EIO, ENOMEM, EINVAL = -5, -12, -22
M64_MAX_PRODUCT_BITS = 1 << 37
NOALLOC_MAX_PRODUCT_BITS = 1 << 25
MAX_PRODUCT_BITS = 1 << 62
SERVER_MAX_PRODUCT_BITS = M64_MAX_PRODUCT_BITS
BATCH_MAX_PRODUCT_BITS = 1 << 22

# (name, restype, argtypes) of every symbol include/fpmul.h declares
_V, _U64, _I, _SZ, _P = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p
SIGNATURES = {
    "polymul": (_I, [_P, _U64, _P, _U64, _P]),
    "polymul_ctx_create": (_I, [ctypes.POINTER(_V), _I, _SZ]),
    "polymul_ctx_destroy": (_I, [_V]),
    "polymul_ex": (_I, [_V, _P, _U64, _P, _U64, _P, _V]),
    "polymul_ex_noalloc": (_I, [_V, _P, _U64, _P, _U64, _P, _V]),
    "polymul_batch": (_I, [_V, ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P, _P, _U64, _P, _V]),
    "polymul_set_small_field": (_I, [_V, _I]),
    "polymul_set_large_field": (_I, [_V, _I]),
    "polymul_tune": (_I, [_V, _I, _I, ctypes.c_char_p, ctypes.c_char_p, _SZ]),
    "polymul_tune_load": (_I, [_V, ctypes.c_char_p, ctypes.POINTER(_I)]),
    "polymul_tune_get": (_I, [_V, _I, ctypes.c_char_p, _SZ]),
    "polymul_graph_create": (_I, [_V, _P, _U64, _P, _U64, _P, ctypes.POINTER(_V)]),
    "polymul_batch_graph_create": (_I, [_V, ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P, _P, _U64, _P,
                                        ctypes.POINTER(_V)]),
    "polymul_graph_launch": (_I, [_V, _V]),
    "polymul_graph_destroy": (_I, [_V]),
    "polymul_server_create": (_I, [ctypes.POINTER(_V), _V, _SZ, ctypes.c_uint32]),
    "polymul_server_destroy": (_I, [_V]),
    "polymul_server_set_policy": (_I, [_V, _U64, ctypes.c_uint32]),
    "polymul_submit": (_I, [_V, _P, _U64, _P, _U64, _P, ctypes.POINTER(_U64)]),
    "polymul_submit_resident": (_I, [_V, _V, _P, _U64, _P, ctypes.POINTER(_U64)]),
    "polymul_resident_create": (_I, [_V, _P, _U64, _U64, ctypes.POINTER(_V)]),
    "polymul_resident_destroy": (_I, [_V]),
    "polymul_resident_mul": (_I, [_V, _V, _P, _U64, _P, _V]),
    "polymul_poll": (_I, [_V, _U64, ctypes.POINTER(_I)]),
    "polymul_wait": (_I, [_V, _U64]),
    "polymul_wait_times": (_I, [_V, _U64, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "polymul_ticket_times": (_I, [_V, _U64, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "polymul_server_tickets": (_I, [_V, ctypes.POINTER(_U64)]),
    "polymul_addfft": (_I, [_V, _P, _U64, _I, _P, _V]),
    "polymul_iaddfft": (_I, [_V, _P, _I, _P, _U64, _V]),
    "polymul_pointwise": (_I, [_V, _P, _P, _I, _P, _V]),
    "polymul_basiscvt": (_I, [_V, _P, _U64, _I, _I, _P, _V]),
    "polymul_profile_enable": (_I, [_V, _I]),
    "polymul_profile_report": (_I, [_V, ctypes.c_char_p, _SZ]),
    "polymul_last_error": (ctypes.c_char_p, []),
    "polymul_version": (ctypes.c_char_p, []),
}


class FpmulError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """Load libfpmul.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: the library and torch share one HIP runtime, and the
        # first libamdhip64 loaded into the process is the one both use; torch
        # initialises only with the runtime it ships with
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with paper_1803_11301_amd/build.py "
                "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise FpmulError(rc, lib().polymul_last_error().decode())


def _dptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("expected a CUDA tensor")
    if not t.is_contiguous() or t.dtype != torch.int64:
        raise ValueError("expected a contiguous int64 tensor of 64-bit words")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def nwords(bits: int) -> int:
    return (bits + 63) // 64


class Context:
    """A library context (constant tables and workspace) for one GPU."""

    def __init__(self, device: int = 0, workspace_cap: int = 0):
        h = ctypes.c_void_p()
        _check(lib().polymul_ctx_create(ctypes.byref(h), device, workspace_cap))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().polymul_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool = True):
        _check(lib().polymul_profile_enable(self.handle, 1 if on else 0))

    def profile_report(self) -> dict:
        """{kernel name: (launches, total ms)} since profiling was enabled."""
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().polymul_profile_report(self.handle, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms = line.split()
            out[name] = (int(cnt), float(ms))
        return out

    def polymul(self, a, len_a: int, b, len_b: int, out=None, stream=None):
        """C = A * B, stream-ordered.  Returns the output tensor."""
        import torch
        lc = len_a + len_b - 1 if (len_a and len_b) else 0
        if out is None:
            out = torch.empty(max(1, nwords(lc)), dtype=torch.int64, device=a.device)
        _check(lib().polymul_ex(self.handle, _dptr(a), len_a, _dptr(b), len_b, _dptr(out), _stream(stream)))
        return out

    def polymul_noalloc(self, a, len_a: int, b, len_b: int, out, stream=None):
        """polymul_ex_noalloc: the same product with the library's device
        scratch as workspace (products up to 2^25 bits; out is required)."""
        _check(lib().polymul_ex_noalloc(self.handle, _dptr(a), len_a, _dptr(b), len_b, _dptr(out),
                                        _stream(stream)))
        return out

    def polymul_batch(self, a_pool, a_off, len_a, b_pool, b_off, len_b, out_pool, out_off,
                      max_product_bits: int, status=None, stream=None):
        """count = len(len_a) products in one launch; every argument is a CUDA
        int64 tensor (status: int32 or None), see polymul_batch in fpmul.h."""
        import torch
        count = int(len_a.numel())
        if status is not None and (status.dtype != torch.int32 or not status.is_contiguous()):
            raise ValueError("status must be a contiguous int32 tensor")
        for t in (a_off, b_off, len_b, out_off):
            if int(t.numel()) != count:
                raise ValueError("descriptor arrays must have one entry per product")
        _check(lib().polymul_batch(self.handle, count, _dptr(a_pool), _dptr(a_off), _dptr(len_a),
                                   _dptr(b_pool), _dptr(b_off), _dptr(len_b), _dptr(out_pool), _dptr(out_off),
                                   max_product_bits, status.data_ptr() if status is not None else None,
                                   _stream(stream)))
        return out_pool

    def set_small_field(self, max_log2n: int):
        """Batch items (and polymul_ex products up to 2^16 bits) with transforms of
        at most 2^max_log2n bits run over GF(2^32); 0 keeps GF(2^64)."""
        _check(lib().polymul_set_small_field(self.handle, max_log2n))

    def set_large_field(self, min_log2n: int):
        """Products (polymul_ex) with transforms of at least 2^min_log2n bits run
        over GF(2^128); transforms above 2^37 bits always do."""
        _check(lib().polymul_set_large_field(self.handle, min_log2n))

    def tune(self, log2n: int, reps: int = 3, cache_path=None) -> str:
        """polymul_tune: time the fused path's schedules for 2^log2n-bit
        transforms, keep the fastest; returns the one-line report."""
        buf = ctypes.create_string_buffer(512)
        _check(lib().polymul_tune(self.handle, log2n, reps,
                                  None if cache_path is None else os.fsencode(cache_path), buf, len(buf)))
        return buf.value.decode()

    def tune_load(self, cache_path) -> int:
        """polymul_tune_load: apply the cache lines for this device; returns their number."""
        n = ctypes.c_int()
        _check(lib().polymul_tune_load(self.handle, os.fsencode(cache_path), ctypes.byref(n)))
        return n.value

    def schedule(self, log2n: int) -> str:
        """polymul_tune_get: the schedule used for 2^log2n-bit transforms."""
        buf = ctypes.create_string_buffer(256)
        _check(lib().polymul_tune_get(self.handle, log2n, buf, len(buf)))
        return buf.value.decode()

    def addfft(self, a, len_a: int, log2n: int, values=None, stream=None):
        import torch
        if values is None:
            values = torch.empty(1 << (log2n - 6), dtype=torch.int64, device=a.device)
        _check(lib().polymul_addfft(self.handle, _dptr(a), len_a, log2n, _dptr(values), _stream(stream)))
        return values

    def iaddfft(self, values, log2n: int, out_bits: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(max(1, nwords(out_bits)), dtype=torch.int64, device=values.device)
        _check(lib().polymul_iaddfft(self.handle, _dptr(values), log2n, _dptr(out), out_bits, _stream(stream)))
        return out

    def pointwise(self, fa, fb, log2n: int, fc=None, stream=None):
        """fc[j] = fa[j] * fb[j] on two transforms of the same log2n; fc may be fa or fb."""
        import torch
        if fc is None:   # the library checks log2n; size the output only when it is valid
            fc = torch.empty(1 << max(0, log2n - 6), dtype=torch.int64, device=fa.device)
        _check(lib().polymul_pointwise(self.handle, _dptr(fa), _dptr(fb), log2n, _dptr(fc), _stream(stream)))
        return fc

    def basiscvt(self, x, length: int, log2n: int, inverse: bool = False, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(max(1, nwords(1 << log2n)), dtype=torch.int64, device=x.device)
        _check(lib().polymul_basiscvt(self.handle, _dptr(x), length, log2n, 1 if inverse else 0,
                                      _dptr(out), _stream(stream)))
        return out


def polymul(a, len_a: int, b, len_b: int, out=None):
    """Synchronous product on the current device (library-owned context)."""
    import torch
    lc = len_a + len_b - 1 if (len_a and len_b) else 0
    if out is None:
        out = torch.empty(max(1, nwords(lc)), dtype=torch.int64, device=a.device)
    _check(lib().polymul(_dptr(a), len_a, _dptr(b), len_b, _dptr(out)))
    return out


class Graph:
    """A captured launch chain (polymul_graph_create or
    polymul_batch_graph_create), replayed with launch()."""

    def __init__(self, handle):
        self.handle = handle

    @classmethod
    def product(cls, ctx: "Context", a, len_a: int, b, len_b: int, out) -> "Graph":
        h = ctypes.c_void_p()
        _check(lib().polymul_graph_create(ctx.handle, _dptr(a), len_a, _dptr(b), len_b, _dptr(out),
                                          ctypes.byref(h)))
        return cls(h)

    @classmethod
    def batch(cls, ctx: "Context", a_pool, a_off, len_a, b_pool, b_off, len_b, out_pool, out_off,
              max_product_bits: int, status=None) -> "Graph":
        h = ctypes.c_void_p()
        _check(lib().polymul_batch_graph_create(ctx.handle, int(len_a.numel()), _dptr(a_pool), _dptr(a_off),
                                                _dptr(len_a), _dptr(b_pool), _dptr(b_off), _dptr(len_b),
                                                _dptr(out_pool), _dptr(out_off), max_product_bits,
                                                status.data_ptr() if status is not None else None,
                                                ctypes.byref(h)))
        return cls(h)

    def launch(self, stream=None):
        _check(lib().polymul_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            lib().polymul_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Resident:
    """An operand kept on the device as its forward transform
    (polymul_resident_create), for products with many B."""

    def __init__(self, ctx: "Context", a, len_a: int, max_product_bits: int):
        h = ctypes.c_void_p()
        _check(lib().polymul_resident_create(ctx.handle, _dptr(a), len_a, max_product_bits, ctypes.byref(h)))
        self.handle = h
        self.len_a = len_a

    def mul(self, ctx: "Context", b, len_b: int, out=None, stream=None):
        """C = A * B reusing A's transform, stream-ordered; returns out."""
        import torch
        lc = self.len_a + len_b - 1 if len_b else 0
        if out is None:
            out = torch.empty(max(1, nwords(lc)), dtype=torch.int64, device=b.device)
        _check(lib().polymul_resident_mul(ctx.handle, self.handle, _dptr(b), len_b, _dptr(out), _stream(stream)))
        return out

    def close(self):
        if self.handle:
            lib().polymul_resident_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching product server on a Context (polymul_server_* in fpmul.h).

    Operands and outputs are CUDA int64 tensors (or raw device addresses) the
    caller keeps alive until the ticket is done."""

    def __init__(self, ctx: Context, hbm_budget: int = 4 << 30, slots: int = 8, batch_limit_bits: int = 1 << 20,
                 max_batch: int = 512):
        h = ctypes.c_void_p()
        _check(lib().polymul_server_create(ctypes.byref(h), ctx.handle, hbm_budget, slots))
        self.handle = h
        self.ctx = ctx
        try:
            _check(lib().polymul_server_set_policy(self.handle, batch_limit_bits, max_batch))
        except FpmulError:
            self.close()
            raise

    def close(self):
        if self.handle:
            lib().polymul_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _addr(x):
        return x if isinstance(x, int) else _dptr(x)

    def submit(self, a, len_a: int, b, len_b: int, out) -> int:
        t = ctypes.c_uint64()
        _check(lib().polymul_submit(self.handle, self._addr(a), len_a, self._addr(b), len_b, self._addr(out),
                                    ctypes.byref(t)))
        return t.value

    def submit_resident(self, res: "Resident", b, len_b: int, out) -> int:
        t = ctypes.c_uint64()
        _check(lib().polymul_submit_resident(self.handle, res.handle, self._addr(b), len_b, self._addr(out),
                                             ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(lib().polymul_poll(self.handle, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        """Block until the ticket is done and release it; returns its
        (submit, launch, done) times in ns since the server was created."""
        s, st, d = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().polymul_wait_times(self.handle, ticket, ctypes.byref(s), ctypes.byref(st), ctypes.byref(d)))
        return s.value, st.value, d.value

    def outstanding(self) -> int:
        """Tickets submitted and not yet released by wait."""
        n = ctypes.c_uint64()
        _check(lib().polymul_server_tickets(self.handle, ctypes.byref(n)))
        return n.value

    def times(self, ticket: int):
        """(submit, launch, done) in ns since the server was created, for a
        ticket not yet released by wait."""
        s, st, d = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().polymul_ticket_times(self.handle, ticket, ctypes.byref(s), ctypes.byref(st), ctypes.byref(d)))
        return s.value, st.value, d.value


def pack_words(arrays):
    """Concatenate word arrays (numpy uint64) into one pool: returns
    (pool, word offsets), each array starting at its offset."""
    import numpy as np
    offs = np.zeros(len(arrays), dtype=np.int64)
    total = 0
    for k, a in enumerate(arrays):
        offs[k] = total
        total += max(1, int(a.size))
    pool = np.zeros(max(1, total), dtype=np.uint64)
    for k, a in enumerate(arrays):
        pool[offs[k]: offs[k] + a.size] = a
    return pool, offs


def out_layout(len_a, len_b):
    """Word offsets and pool size for the products of a batch."""
    import numpy as np
    la = np.asarray(len_a, dtype=np.int64)
    lb = np.asarray(len_b, dtype=np.int64)
    words = np.where((la > 0) & (lb > 0), (la + lb - 1 + 63) // 64, 0)
    words = np.maximum(words, 1)
    offs = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.int64)
    return offs, int(words.sum())


def version() -> str:
    return lib().polymul_version().decode()
