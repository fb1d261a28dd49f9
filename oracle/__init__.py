"""CPU oracle for the product in GF(2)[x] (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library.

The oracle is the plain definition of the product (Sec. 2.1; Alg. 5 output):
``c_k = XOR_{i+j=k} a_i b_j``.  The heavy lifting is plain C (``oracle.c``,
schoolbook and Karatsuba word products); this module loads it with ctypes
and adds tiny pure-Python references for brute-force pins.

Arrays are numpy ``uint64`` word arrays, bit ``k`` at bit ``k % 64`` of word
``k // 64``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11",
               "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_polymul.argtypes = [_u64p, ctypes.c_uint64, _u64p, ctypes.c_uint64,
                                     _u64p, ctypes.c_int, ctypes.c_int]
        L.oracle_polymul.restype = ctypes.c_int
        L.oracle_product_words.argtypes = [_u64p, ctypes.c_uint64, _u64p, ctypes.c_uint64,
                                           _u64p, ctypes.c_uint64, _u64p]
        L.oracle_product_words.restype = None
        L.oracle_gf64_mul.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_gf64_mul.restype = ctypes.c_uint64
        L.oracle_eval.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_eval.restype = ctypes.c_uint64
        L.oracle_clmul64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _u64p]
        L.oracle_clmul64.restype = None
        L.oracle_set_impl.argtypes = [ctypes.c_int]
        L.oracle_set_impl.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def nwords(bits: int) -> int:
    return (bits + 63) // 64


def polymul(a: np.ndarray, len_a: int, b: np.ndarray, len_b: int,
            method: str = "karatsuba", threads: int = 1) -> np.ndarray:
    """Product of two bit polynomials; returns ceil((la+lb-1)/64) words."""
    lc = len_a + len_b - 1 if (len_a and len_b) else 0
    out = np.zeros(max(1, nwords(lc)), dtype=np.uint64)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    if a.size == 0:
        a = np.zeros(1, np.uint64)
    if b.size == 0:
        b = np.zeros(1, np.uint64)
    m = {"schoolbook": 0, "karatsuba": 1}[method]
    lib().oracle_polymul(_ptr(a), len_a, _ptr(b), len_b, _ptr(out), m, threads)
    return out[: nwords(lc)]


def product_words(a, len_a, b, len_b, idx) -> np.ndarray:
    """Selected output words of the product, each from the definition."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.zeros(idx.size, dtype=np.uint64)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    lib().oracle_product_words(_ptr(a), len_a, _ptr(b), len_b, _ptr(idx), idx.size, _ptr(out))
    return out


def gf64_mul(x: int, y: int) -> int:
    """Product in GF(2)[x]/(x^64+x^4+x^3+x+1) (Sec. 4.3 modulus)."""
    return int(lib().oracle_gf64_mul(x, y))


def eval_at(a: np.ndarray, length: int, z: int) -> int:
    """A(z) for a bit polynomial A of ``length`` bits and z in GF(2^64)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if a.size == 0:
        return 0
    return int(lib().oracle_eval(_ptr(a), length, z))


def clmul64(a: int, b: int, hw: bool) -> int:
    out = np.zeros(2, np.uint64)
    lib().oracle_clmul64(a, b, 1 if hw else 0, _ptr(out))
    return int(out[0]) | (int(out[1]) << 64)


def set_impl(hw: int) -> int:
    """-1 queries; 0 forces the software word product; 1 forces PCLMULQDQ."""
    return int(lib().oracle_set_impl(hw))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ---------------------------------------------------------------------------
# tiny pure-Python references (Python ints as bit vectors)
# ---------------------------------------------------------------------------

def py_clmul(a: int, b: int) -> int:
    """Carry-less product of two Python ints, one bit of b at a time."""
    r = 0
    i = 0
    while b >> i:
        if (b >> i) & 1:
            r ^= a << i
        i += 1
    return r


def words_to_int(w: np.ndarray, length: int) -> int:
    """Little-endian words -> Python int (the first ``length`` bits)."""
    v = int.from_bytes(np.ascontiguousarray(w, dtype="<u8").tobytes(), "little")
    return v & ((1 << length) - 1) if length >= 0 else v


def int_to_words(v: int, length: int) -> np.ndarray:
    """Python int -> ceil(length / 64) little-endian words (bits at or above length dropped)."""
    n = nwords(length)
    if n <= 0:
        return np.zeros(0, dtype=np.uint64)
    v &= (1 << (64 * n)) - 1
    return np.frombuffer(v.to_bytes(8 * n, "little"), dtype="<u8").astype(np.uint64)
