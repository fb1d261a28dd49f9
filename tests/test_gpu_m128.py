"""GPU parity of the m = 128 variant (GF(2^128), l_m = 7) against the CPU oracle.

Products above 2^37 bits must run over GF(2^128) (the field bound after
Prop. 2); polymul_set_large_field runs the same path on products of any size,
which is how the small and mid-size cases below reach it.  The full-size cases
have one short operand so that every output word can be recomputed from the
definition over a window of the long operand: word w of A B depends on the
words w - nb .. w of A only (nb = words of B).

Every case prints its name, sizes and seed before touching the GPU.
"""
import random
import sys

import numpy as np
import pytest

import oracle as O
from paper_1803_11301_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx128():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_11301_amd import fpmul
    c = fpmul.Context(0)
    c.set_large_field(7)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(words):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    if w.size == 0:
        w = np.zeros(1, np.uint64)
    return torch.from_numpy(w.view(np.int64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def gpu_product(ctx, a, la, b, lb):
    out = ctx.polymul(dev(a), la, dev(b), lb)
    return host(out)[: O.nwords(la + lb - 1)]


def rand_words(rng, length):
    return O.int_to_words(rng.getrandbits(length) if length else 0, length)


@pytest.mark.parametrize("la,lb", [(100, 29), (128, 1), (1, 128), (129, 1), (64, 65), (65, 64), (200, 300),
                                   (255, 2), (1000, 1049), (4096, 4096), (4097, 4095), (8191, 1), (65536, 65536),
                                   (70001, 3), (3, 70001), ((1 << 17) + 9, (1 << 16) - 3)])
def test_m128_products_exact(ctx128, la, lb):
    say("m128", la, lb)
    rng = random.Random(la * 7 + lb)
    a, b = rand_words(rng, la), rand_words(rng, lb)
    assert np.array_equal(gpu_product(ctx128, a, la, b, lb), O.polymul(a, la, b, lb, threads=8))


@pytest.mark.parametrize("la,lb", [((1 << 20) + 3, (1 << 19) - 5), (1 << 21, 1 << 21), ((1 << 22) + 17, (1 << 22) - 100),
                                   (1 << 24, 1 << 24)])
def test_m128_larger_products_exact(ctx128, la, lb):
    say("m128 larger", la, lb)
    seed = 0x5EED0128 + la
    a, b = synth.dense_poly(seed, la), synth.dense_poly(seed + 1, lb)
    assert np.array_equal(gpu_product(ctx128, a, la, b, lb), O.polymul(a, la, b, lb, threads=16))


def test_m128_small_length_sweep(ctx128):
    """Every pair of lengths in a ragged set whose product reaches 2^7 bits."""
    say("m128 sweep")
    rng = random.Random(128)
    lens = [1, 2, 5, 31, 63, 64, 65, 66, 100, 127, 128, 129, 191, 256, 257, 511]
    for la in lens:
        for lb in lens:
            if la + lb - 1 < 128:
                continue
            a, b = rand_words(rng, la), rand_words(rng, lb)
            assert np.array_equal(gpu_product(ctx128, a, la, b, lb), O.polymul(a, la, b, lb)), (la, lb)


def test_m128_closed_forms(ctx128):
    say("m128 closed forms")
    # x^a x^b = x^(a+b)
    for ea, eb in [(0, 127), (127, 0), (100, 200), (4095, 4096), (70000, 1)]:
        a = O.int_to_words(1 << ea, ea + 1)
        b = O.int_to_words(1 << eb, eb + 1)
        got = gpu_product(ctx128, a, ea + 1, b, eb + 1)
        assert O.words_to_int(got, ea + eb + 1) == 1 << (ea + eb)
    # A A = A(x^2): bit i goes to bit 2i
    rng = random.Random(5)
    for L in [64, 65, 1000, 1 << 14]:
        f = rng.getrandbits(L)
        a = O.int_to_words(f, L)
        got = O.words_to_int(gpu_product(ctx128, a, L, a, L), 2 * L - 1)
        spread = 0
        for i in range(L):
            if (f >> i) & 1:
                spread |= 1 << (2 * i)
        assert got == spread


def test_m128_same_as_m64(ctx128):
    """The two fields give the same product (Prop. 2 for each m)."""
    from paper_1803_11301_amd import fpmul
    say("m128 vs m64")
    c64 = fpmul.Context(0)
    try:
        for la, lb in [(3000, 5000), (1 << 18, 1 << 18), ((1 << 23) - 1, 1 << 23)]:
            a, b = synth.dense_poly(la, la), synth.dense_poly(lb + 1, lb)
            da, db = dev(a), dev(b)
            x = host(ctx128.polymul(da, la, db, lb))
            y = host(c64.polymul(da, la, db, lb))
            assert np.array_equal(x, y), (la, lb)
    finally:
        torch.cuda.synchronize()
        c64.close()


def test_m128_sparse_and_tail_bits(ctx128):
    say("m128 sparse / tail bits")
    la, lb = 50001, 40003
    a, b = synth.sparse_poly(21, la), synth.sparse_poly(22, lb)
    assert np.array_equal(gpu_product(ctx128, a, la, b, lb), O.polymul(a, la, b, lb))
    # garbage above the length in the last input word is ignored; the output tail is zeroed
    a2, b2 = a.copy(), b.copy()
    a2[-1] |= ~np.uint64((1 << (la % 64)) - 1)
    b2[-1] |= ~np.uint64((1 << (lb % 64)) - 1)
    got = gpu_product(ctx128, a2, la, b2, lb)
    assert np.array_equal(got, O.polymul(a, la, b, lb))
    lc = la + lb - 1
    assert int(got[-1]) >> (lc % 64) == 0


def test_large_field_threshold_rejected_outside_range(ctx128):
    from paper_1803_11301_amd import fpmul
    say("m128 threshold range")
    for bad in (6, 39, -1):
        with pytest.raises(fpmul.FpmulError):
            ctx128.set_large_field(bad)


# --------------------------------------------------------------------------
# full size: one long operand on the device, windows recomputed on the host
# --------------------------------------------------------------------------

def _check_windows(A, la, b, lb, got, samples):
    nb = O.nwords(lb)
    na = O.nwords(la)
    for w in samples:
        s = max(0, w - nb - 1)
        e = min(w + 1, na)
        win = A[s:e].cpu().numpy().view(np.uint64).copy()
        lw = la - 64 * s if e == na else 64 * (e - s)
        ref = O.product_words(win, lw, b, lb, np.array([w - s], np.uint64))[0]
        assert int(got[w].item()) & ((1 << 64) - 1) == int(ref), ("word", w)


def _full_size_case(la, lb, seed, threshold=None):
    from paper_1803_11301_amd import fpmul
    say("full size", la, "x", lb, "seed", hex(seed), "large-field threshold", threshold)
    A = synth.dense_poly_device(seed, la, "cuda")
    b = synth.dense_poly(seed + 1, lb)
    B = dev(b)
    torch.cuda.empty_cache()
    c = fpmul.Context(0)
    try:
        if threshold is not None:
            c.set_large_field(threshold)
        out = c.polymul(A, la, B, lb)
        torch.cuda.synchronize()
        lc = la + lb - 1
        nc = O.nwords(lc)
        rng = random.Random(seed)
        samples = {0, 1, 2, nc // 2, nc - 2, nc - 1} | {rng.randrange(nc) for _ in range(120)}
        for k in range(6, 64):
            if (1 << k) < nc:
                samples |= {(1 << k) - 1, 1 << k}
        _check_windows(A, la, b, lb, out, sorted(samples))
        assert int(out[nc - 1].item()) >> (lc % 64) == 0 if lc % 64 else True
    finally:
        torch.cuda.synchronize()
        c.close()
        del A, B
        torch.cuda.empty_cache()


def test_m64_per_step_path_above_fused_sizes():
    """A 2^33-bit transform: BasisCvt, Encode and Decode step by step, with the
    resident-table butterfly passes at l = 27."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _full_size_case((1 << 32) + 1, 4096, 0x5EED0033)


def test_m64_at_its_largest_product():
    """A product of exactly 2^37 bits, the largest GF(2^64) takes (a 2^37-bit
    transform, l = 31 in the resident-table butterfly passes)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, total = torch.cuda.mem_get_info()
    if free < (120 << 30):
        pytest.skip("needs 120 GiB of free device memory")
    _full_size_case((1 << 37) - 4095, 4096, 0x5EED0037 + 64)


def test_m128_at_2e33_bits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _full_size_case((1 << 32) + 1, 4096, 0x5EED0033, threshold=33)


def test_m128_beyond_the_m64_bound():
    """A product of 2^37 + 4096 bits: a 2^38-bit transform, past what GF(2^64)
    can hold, so it runs over GF(2^128) without any setting (16 GiB operand,
    16 GiB output, 128 GiB workspace)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, total = torch.cuda.mem_get_info()
    if free < (200 << 30):
        pytest.skip("needs 200 GiB of free device memory")
    _full_size_case((1 << 37) + 1, 4096, 0x5EED0038)


def test_m128_balanced_2e37_words():
    """The bench shape, 2^37 x 2^37 bits over GF(2^128): the 16 lowest and 16
    highest output words (the definition computes them from the lowest or
    highest words of A and B alone) and 8 words from the middle of the
    product, each of which collects about 2^31 word products of the whole of
    A and B (the operands are copied to the host; the oracle computes those
    words on parallel host threads)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, total = torch.cuda.mem_get_info()
    if free < (230 << 30):
        pytest.skip("needs 230 GiB of free device memory")
    from concurrent.futures import ThreadPoolExecutor
    from paper_1803_11301_amd import fpmul
    L, seed = 1 << 37, 0x5EED0037
    say("balanced 2^37 x 2^37 end and middle words, seeds", hex(seed), hex(seed + 1))
    A = synth.dense_poly_device(seed, L, "cuda")
    B = synth.dense_poly_device(seed + 1, L, "cuda")
    torch.cuda.empty_cache()
    c = fpmul.Context(0)
    try:
        out = c.polymul(A, L, B, L)
        torch.cuda.synchronize()
        nc, na = out.numel(), A.numel()
        for w in list(range(16)) + list(range(nc - 16, nc)):
            if w < na:
                a_w = A[: w + 1].cpu().numpy().view(np.uint64)
                b_w = B[: w + 1].cpu().numpy().view(np.uint64)
                ref = O.product_words(a_w, 64 * (w + 1), b_w, 64 * (w + 1), np.array([w], np.uint64))[0]
            else:
                s0 = w - na   # only words s0 .. of A and B reach word w
                a_w = A[s0:].cpu().numpy().view(np.uint64)
                b_w = B[s0:].cpu().numpy().view(np.uint64)
                ref = O.product_words(a_w, L - 64 * s0, b_w, L - 64 * s0, np.array([w - 2 * s0], np.uint64))[0]
            assert int(out[w].item()) & ((1 << 64) - 1) == int(ref), ("word", w)
        rng = random.Random(37)
        mid = sorted({nc // 2 - 2, nc // 2 - 1, nc // 2, nc // 2 + 1, nc // 4, 3 * nc // 4,
                      rng.randrange(nc // 8, 7 * nc // 8), rng.randrange(nc // 8, 7 * nc // 8)})
        got = [int(out[w].item()) & ((1 << 64) - 1) for w in mid]
        del out
        say("middle words", mid, "on the host")
        a_h = A.cpu().numpy().view(np.uint64)
        b_h = B.cpu().numpy().view(np.uint64)
        with ThreadPoolExecutor(max_workers=len(mid)) as ex:
            refs = list(ex.map(lambda w: int(O.product_words(a_h, L, b_h, L, np.array([w], np.uint64))[0]), mid))
        assert got == refs, [w for w, g, r in zip(mid, got, refs) if g != r]
    finally:
        torch.cuda.synchronize()
        c.close()
        del A, B
        torch.cuda.empty_cache()
