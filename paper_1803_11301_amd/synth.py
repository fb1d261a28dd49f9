"""Seeded synthetic inputs (no arithmetic of the multiplication method).

The one module shared by the HIP path's tests, the oracle's tests and
``bench.py``.  It only draws bits and lengths; it multiplies nothing.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", 2014): the state advances by 0x9E3779B97F4A7C15 and each
output is the state passed through the variant-13 finaliser
``z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
z ^= z >> 31``.  Output ``i`` (0-based) of the stream with seed ``s`` is the
finaliser applied to ``s + (i + 1) * 0x9E3779B97F4A7C15`` mod 2^64, which lets
numpy produce a whole stream at once.

Workloads (the paper benchmarks products of uniformly random bit polynomials,
Sec. 5.1):
  * single products: operand A from seed s, operand B from seed s + 1, words
    in stream order, bits at or above the length masked to zero;
  * a batch of products with log-uniform lengths, 10% sparse at density 0.01;
  * a serving stream: Poisson arrivals with log-uniform lengths.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1

SEED_SMALL = 0x5EED0016     # 2^16 x 2^16 bits
SEED_MID = 0x5EED0024       # 2^24 x 2^24 bits, top bit forced
SEED_LARGE = 0x5EED0030     # 2^30 x 2^30 bits
SEED_BATCH = 0x5EED4096     # 4096 products, log-uniform 2^10 .. 2^20 bits
SEED_SERVE = 0x5EED05E5     # Poisson stream, log-uniform 2^12 .. 2^24 bits


def _mix(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream for ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + i * GOLDEN
        return _mix(z)


def splitmix64_scalar(state: int) -> tuple[int, int]:
    """One step of the reference recurrence: returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def nwords(bits: int) -> int:
    return (bits + 63) // 64


def mask_tail(words: np.ndarray, length: int) -> np.ndarray:
    n = nwords(length)
    words = words[:n].copy()
    if length % 64 and n:
        words[n - 1] &= np.uint64((1 << (length % 64)) - 1)
    return words


def dense_poly(seed: int, length: int, top_bit: bool = False) -> np.ndarray:
    """Uniform random bit polynomial of ``length`` bits (words of the stream)."""
    w = mask_tail(splitmix64(seed, max(nwords(length), 1)), length)
    if top_bit and length:
        k = length - 1
        w[k // 64] |= np.uint64(1 << (k % 64))
    return w[: nwords(length)]


def _as_i64(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >> 63 else v


def dense_poly_device(seed: int, length: int, device, chunk_words: int = 1 << 26):
    """``dense_poly(seed, length)`` generated on a torch device (int64 words of
    the same bits), for operands too large to draw on the host.  int64
    products wrap modulo 2^64, and a logical shift is an arithmetic shift
    masked to the low 64 - k bits."""
    import torch
    n = max(nwords(length), 1)
    out = torch.empty(n, dtype=torch.int64, device=device)

    def shr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    golden, m1, m2 = _as_i64(int(GOLDEN)), _as_i64(int(_M1)), _as_i64(int(_M2))
    for off in range(0, n, chunk_words):
        cnt = min(chunk_words, n - off)
        z = torch.arange(off + 1, off + cnt + 1, dtype=torch.int64, device=device)
        z.mul_(golden).add_(_as_i64(seed))
        z.bitwise_xor_(shr(z, 30)).mul_(m1)
        z.bitwise_xor_(shr(z, 27)).mul_(m2)
        z.bitwise_xor_(shr(z, 31))
        out[off:off + cnt] = z
        del z
    if length % 64 and length:
        out[n - 1] &= (1 << (length % 64)) - 1
    if length == 0:
        out.zero_()
    return out


def unit_floats(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the 53 high bits of each output."""
    x = splitmix64(seed, count, start) >> np.uint64(11)
    return x.astype(np.float64) * (1.0 / (1 << 53))


def sparse_poly(seed: int, length: int, density: float = 0.01) -> np.ndarray:
    """Each bit set independently with probability ``density``."""
    out = np.zeros(max(nwords(length), 1), dtype=np.uint64)
    chunk = 1 << 22
    for off in range(0, length, chunk):
        n = min(chunk, length - off)
        hit = np.nonzero(unit_floats(seed, n, off) < density)[0] + off
        np.bitwise_or.at(out, hit // 64, np.left_shift(np.uint64(1), (hit % 64).astype(np.uint64)))
    return out[: nwords(length)]


def single_pair(seed: int, length: int, top_bit: bool = False):
    """(A, B) for a single product: A from ``seed``, B from ``seed + 1``."""
    return dense_poly(seed, length, top_bit), dense_poly(seed + 1, length, top_bit)


@dataclass
class BatchItem:
    len_a: int
    len_b: int
    sparse: bool
    seed_a: int
    seed_b: int


def batch_plan(count: int = 4096, seed: int = SEED_BATCH, lo: int = 10, hi: int = 20,
               sparse_frac: float = 0.1) -> list[BatchItem]:
    """Per product five draws from the master stream: u, u', u'', seed_a, seed_b.
    Lengths are floor(2^(lo + (hi - lo) u)); the pair is sparse if u'' < sparse_frac."""
    raw = splitmix64(seed, 5 * count).reshape(count, 5)
    f = (raw[:, :3] >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    items = []
    span = hi - lo
    for p in range(count):
        la = int(math.floor(2.0 ** (lo + span * f[p, 0])))
        lb = int(math.floor(2.0 ** (lo + span * f[p, 1])))
        items.append(BatchItem(la, lb, bool(f[p, 2] < sparse_frac), int(raw[p, 3]), int(raw[p, 4])))
    return items


def batch_operands(item: BatchItem):
    if item.sparse:
        return sparse_poly(item.seed_a, item.len_a), sparse_poly(item.seed_b, item.len_b)
    return dense_poly(item.seed_a, item.len_a), dense_poly(item.seed_b, item.len_b)


def serve_plan(count: int, rate_per_s: float, seed: int = SEED_SERVE, lo: int = 12, hi: int = 24):
    """Arrival times (s) and lengths for a Poisson stream; six draws per request:
    inter-arrival u, length draws u', u'', operand seeds, spare."""
    raw = splitmix64(seed, 6 * count).reshape(count, 6)
    f = (raw[:, :3] >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    gaps = -np.log1p(-f[:, 0]) / rate_per_s
    t = np.cumsum(gaps)
    span = hi - lo
    la = np.floor(2.0 ** (lo + span * f[:, 1])).astype(np.int64)
    lb = np.floor(2.0 ** (lo + span * f[:, 2])).astype(np.int64)
    return t, la, lb, raw[:, 3].copy(), raw[:, 4].copy()
