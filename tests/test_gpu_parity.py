"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Every case prints its name, sizes and seed before touching the GPU.
"""
import random
import sys

import numpy as np
import pytest

import oracle as O
from oracle import cantor as F
from paper_1803_11301_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_11301_amd import fpmul
    c = fpmul.Context(0)
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


# --------------------------------------------------------------------------
# stages
# --------------------------------------------------------------------------

@pytest.mark.parametrize("log2n", [0, 1, 2, 3, 5, 6, 7, 8, 10, 12])
def test_basiscvt_against_definition(ctx, log2n):
    say("basiscvt", log2n)
    rng = random.Random(log2n)
    n = 1 << log2n
    for length in sorted({1, n // 2 + 1, n}):
        if length > n:
            continue
        f = rng.getrandbits(length)
        got = host(ctx.basiscvt(dev(O.int_to_words(f, length)), length, log2n))
        g = O.words_to_int(got, n)
        assert g == F.to_novelpoly(f, n)
        back = host(ctx.basiscvt(dev(got), n, log2n, inverse=True))
        assert O.words_to_int(back, n) == f


@pytest.mark.parametrize("log2n", [6, 7, 8, 9, 12, 13, 16, 17, 18, 19, 24, 26, 27])
def test_addfft_is_evaluation_at_sigma(ctx, log2n):
    say("addfft", log2n)
    rng = random.Random(100 + log2n)
    n = 1 << log2n
    l = log2n - 6
    la = n // 2
    a = rand_words(rng, la)
    vals = host(ctx.addfft(dev(a), la, log2n))
    js = sorted({0, (1 << l) - 1} | {rng.randrange(1 << l) for _ in range(12)})
    for j in js:
        assert F.tower_to_poly(int(vals[j])) == O.eval_at(a, la, F.point(l, j)), j
    back = host(ctx.iaddfft(dev(vals), log2n, la))
    assert np.array_equal(back[: O.nwords(la)], a)


def test_addfft_full_length_operand_round_trip(ctx):
    say("addfft full length")
    rng = random.Random(7)
    log2n = 14
    n = 1 << log2n
    a = rand_words(rng, n)
    vals = host(ctx.addfft(dev(a), n, log2n))
    for j in (0, 3, 255):
        assert F.tower_to_poly(int(vals[j])) == O.eval_at(a, n, F.point(log2n - 6, j))
    assert np.array_equal(host(ctx.iaddfft(dev(vals), log2n, n)), a)


def test_addfft_round_trip_above_fused_sizes():
    """polymul_addfft / polymul_iaddfft at a 2^33-bit transform (the per-step
    path): the inverse gives a full-length ragged A back, and for a 2^20-bit A
    (the same full-size butterflies, cheap to evaluate on the host) sampled
    values are A at the points of Sigma."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_11301_amd import fpmul
    log2n, la, seed = 33, (1 << 32) + 12345, 0x5EED0A33
    say("addfft round trip", log2n, la, hex(seed))
    A = synth.dense_poly_device(seed, la, "cuda")
    c = fpmul.Context(0)
    try:
        back = c.iaddfft(c.addfft(A, la, log2n), log2n, la)
        torch.cuda.synchronize()
        assert torch.equal(back, A)
        del back
        ls = 1 << 20
        a = synth.dense_poly(seed + 1, ls)
        vals = c.addfft(dev(a), ls, log2n)
        torch.cuda.synchronize()
        for j in (0, 12345, (1 << 27) - 1):
            assert F.tower_to_poly(int(vals[j].item()) & ((1 << 64) - 1)) == \
                O.eval_at(a, ls, F.point(log2n - 6, j))
    finally:
        torch.cuda.synchronize()
        c.close()
        del A
        torch.cuda.empty_cache()


def test_frobenius_identity_on_transform(ctx):
    # the transform of A^2 is the elementwise square of the transform of A (Eq. 1)
    say("frobenius")
    rng = random.Random(3)
    log2n, la = 12, 1500
    a = rand_words(rng, la)
    a2 = O.polymul(a, la, a, la)
    va = host(ctx.addfft(dev(a), la, log2n))
    va2 = host(ctx.addfft(dev(a2), 2 * la - 1, log2n))
    for j in range(0, va.size, 7):
        assert F.tower_to_poly(int(va2[j])) == F.sqr(F.tower_to_poly(int(va[j])))


# --------------------------------------------------------------------------
# products
# --------------------------------------------------------------------------

def test_small_config_exact(ctx):
    L = 1 << 16
    say("2^16 x 2^16", hex(synth.SEED_SMALL))
    a, b = synth.single_pair(synth.SEED_SMALL, L)
    assert np.array_equal(gpu_product(ctx, a, L, b, L), O.polymul(a, L, b, L, threads=8))


@pytest.mark.parametrize("la,lb", [(1, 1), (1, 2), (2, 1), (3, 5), (31, 34), (32, 33), (33, 32), (63, 1), (64, 1),
                                   (65, 1), (64, 64), (65, 64), (100, 29), (127, 128), (1000, 3), (4096, 4096),
                                   (4097, 4095), (1, 1 << 16), ((1 << 16) + 1, 77), (12345, 6789), (1 << 17, 1),
                                   (70001, 60001)])
def test_length_sweep(ctx, la, lb):
    say("sweep", la, lb)
    rng = random.Random(la * 131 + lb)
    a, b = rand_words(rng, la), rand_words(rng, lb)
    assert np.array_equal(gpu_product(ctx, a, la, b, lb), O.polymul(a, la, b, lb, threads=8))


def test_every_small_length_pair(ctx):
    say("all lengths 1..40")
    rng = random.Random(77)
    for la in range(1, 41):
        for lb in range(1, 41, 3):
            a, b = rand_words(rng, la), rand_words(rng, lb)
            assert np.array_equal(gpu_product(ctx, a, la, b, lb), O.polymul(a, la, b, lb)), (la, lb)


def test_closed_forms(ctx):
    say("closed forms")
    rng = random.Random(5)
    la = 20000
    a = rand_words(rng, la)
    av = O.words_to_int(a, la)
    sq = O.words_to_int(gpu_product(ctx, a, la, a, la), 2 * la - 1)
    spread = 0
    for k in range(la):
        if (av >> k) & 1:
            spread |= 1 << (2 * k)
    assert sq == spread
    for p, q in ((0, 0), (5, 70), (4095, 4097), (40000, 123)):
        x = O.int_to_words(1 << p, p + 1)
        y = O.int_to_words(1 << q, q + 1)
        assert O.words_to_int(gpu_product(ctx, x, p + 1, y, q + 1), p + q + 1) == 1 << (p + q)
    k = 9999
    ones = O.int_to_words((1 << k) - 1, k)
    assert O.words_to_int(gpu_product(ctx, O.int_to_words(3, 2), 2, ones, k), k + 1) == (1 << k) | 1


def test_tail_bits_ignored_and_output_tail_zeroed(ctx):
    say("tails")
    la, lb = 130, 70
    a = np.full(3, np.uint64(0xFFFFFFFFFFFFFFFF))
    b = np.full(2, np.uint64(0xFFFFFFFFFFFFFFFF))
    out = torch.full((5,), -1, dtype=torch.int64, device="cuda")
    ctx.polymul(dev(a), la, dev(b), lb, out=out)
    got = host(out)
    ref = O.polymul(a, la, b, lb)
    assert ref.size == 4
    assert np.array_equal(got[: ref.size], ref)
    assert int(got[ref.size - 1]) >> ((la + lb - 1) % 64) == 0
    assert int(got[4]) == 0xFFFFFFFFFFFFFFFF   # beyond the product: untouched


def test_empty_operand_writes_nothing(ctx):
    say("empty")
    out = torch.full((2,), 7, dtype=torch.int64, device="cuda")
    ctx.polymul(dev(np.ones(1, np.uint64)), 0, dev(np.ones(1, np.uint64)), 5, out=out)
    assert host(out).tolist() == [7, 7]


def test_sparse_operands(ctx):
    say("sparse")
    la, lb = 300000, 200000
    a = synth.sparse_poly(11, la)
    b = synth.sparse_poly(12, lb)
    assert np.array_equal(gpu_product(ctx, a, la, b, lb), O.polymul(a, la, b, lb, threads=8))


def test_mid_config_exact(ctx):
    L = 1 << 24
    say("2^24 x 2^24 top bit", hex(synth.SEED_MID))
    a, b = synth.single_pair(synth.SEED_MID, L, top_bit=True)
    got = gpu_product(ctx, a, L, b, L)
    assert np.array_equal(got, O.polymul(a, L, b, L, threads=16))
    assert int(got[-1]) >> 62 == 1   # degree 2^25 - 2 is present


@pytest.mark.parametrize("L", [1 << 25, (1 << 26) - 5])
def test_large_products_exact(ctx, L):
    say(L, "x", L, "whole output against the oracle", hex(synth.SEED_LARGE))
    a, b = synth.single_pair(synth.SEED_LARGE, L)
    got = gpu_product(ctx, a, L, b, L)
    assert np.array_equal(got, O.polymul(a, L, b, L, threads=16))


@pytest.mark.parametrize("la,lb", [(1 << 28, 1 << 28), ((1 << 27) + 9, (1 << 27) - 9), ((1 << 29) - 7, 5)])
def test_sampled_words_with_twelve_and_thirteen_row_bits(ctx, la, lb):
    """Operands and products of 2^12 and 2^13 rows of 2^16 bits, whose
    superset sums run as two register-tile passes (6 + 6 and 7 + 6 row bits):
    sampled output words from the definition and the evaluation identity at
    a random point."""
    say("sampled", la, "x", lb)
    rng = random.Random(la ^ lb)
    a = synth.dense_poly(0x5EED2800 + la % 977, la)
    b = synth.dense_poly(0x5EED2900 + lb % 977, lb)
    got = gpu_product(ctx, a, la, b, lb)
    n = O.nwords(la + lb - 1)
    idx = np.array(sorted({0, 1, n // 3, n // 2, n - 2, n - 1} | {rng.randrange(n) for _ in range(8)}),
                   dtype=np.uint64)
    assert np.array_equal(got[idx.astype(np.int64)], O.product_words(a, la, b, lb, idx))
    z = rng.getrandbits(64) | 1
    assert O.gf64_mul(O.eval_at(a, la, z), O.eval_at(b, lb, z)) == O.eval_at(got, la + lb - 1, z)


def _golden_digest(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")) as f:
        return json.load(f)[name]


@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_single_product_workloads_match_oracle_digest(ctx, name):
    """The whole output of each single-product workload (2^16, 2^24 with the top
    bit forced, and the 2^30 x 2^30-bit headline product) against the SHA-256
    of the oracle's product, stored by tests/golden/make_digests.py.  The
    product is unique (Prop. 2), so equal digests mean equal outputs; a few
    words are also checked one by one from the definition, which names the
    word that differs if the digest does not match."""
    import hashlib
    g = _golden_digest(name)
    L = g["len_a"]
    say(name, L, "x", L, "digest", g["seed_a"])
    a, b = synth.single_pair(int(g["seed_a"], 16), L, top_bit=g["top_bit"])
    got = gpu_product(ctx, a, L, b, L)
    assert got.size == g["words"]
    rng = random.Random(30)
    nw = got.size
    idx = np.array(sorted({0, 1, nw // 2 - 1, nw // 2, nw - 1} | {rng.randrange(nw) for _ in range(11)}), np.uint64)
    assert np.array_equal(got[idx.astype(np.int64)], O.product_words(a, L, b, L, idx))
    assert hashlib.sha256(np.ascontiguousarray(got, dtype="<u8").tobytes()).hexdigest() == g["sha256"]


def test_synchronous_polymul_entry_point(ctx):
    """polymul(): the synchronous product with the library-owned context of the
    current device, on the 2^16 x 2^16 workload, and its argument errors."""
    import ctypes
    from paper_1803_11301_amd import fpmul
    L = 1 << 16
    say("polymul() 2^16 x 2^16", hex(synth.SEED_SMALL))
    a, b = synth.single_pair(synth.SEED_SMALL, L)
    ta, tb = dev(a), dev(b)
    out = torch.full((O.nwords(2 * L - 1),), -1, dtype=torch.int64, device="cuda")
    lib = fpmul.lib()
    assert lib.polymul(ta.data_ptr(), L, tb.data_ptr(), L, out.data_ptr()) == 0
    # synchronous: the result is there without a further synchronisation
    assert np.array_equal(out.cpu().numpy().view(np.uint64), O.polymul(a, L, b, L, threads=8))
    assert lib.polymul(None, L, tb.data_ptr(), L, out.data_ptr()) == fpmul.EINVAL
    assert "null" in lib.polymul_last_error().decode()
    assert lib.polymul(ta.data_ptr(), L, tb.data_ptr(), L, None) == fpmul.EINVAL
    # the output overlapping an input
    assert lib.polymul(ta.data_ptr(), L, tb.data_ptr(), L, ta.data_ptr()) == fpmul.EINVAL
    assert lib.polymul(ta.data_ptr(), L, tb.data_ptr(), L, tb.data_ptr() + 8) == fpmul.EINVAL
    assert "overlap" in lib.polymul_last_error().decode()
    # host memory is refused
    hbuf = np.zeros(O.nwords(2 * L - 1), np.uint64)
    assert lib.polymul(ta.data_ptr(), L, tb.data_ptr(), L, hbuf.ctypes.data_as(ctypes.c_void_p)) == fpmul.EINVAL
    # an empty operand: nothing written, success
    keep = out.clone()
    assert lib.polymul(ta.data_ptr(), 0, tb.data_ptr(), L, out.data_ptr()) == 0
    assert torch.equal(out, keep)


# --------------------------------------------------------------------------
# errors
# --------------------------------------------------------------------------

def test_error_codes(ctx):
    say("errors")
    from paper_1803_11301_amd import fpmul
    L = fpmul.lib()
    a = dev(np.ones(2, np.uint64))
    out = dev(np.zeros(4, np.uint64))
    # output overlapping an input
    assert L.polymul_ex(ctx.handle, a.data_ptr(), 64, a.data_ptr(), 64, a.data_ptr(), None) == fpmul.EINVAL
    # host memory is not accepted
    host_buf = np.zeros(4, np.uint64)
    assert L.polymul_ex(ctx.handle, host_buf.ctypes.data, 64, a.data_ptr(), 64, out.data_ptr(), None) == fpmul.EINVAL
    # beyond the 2^62-bit limit (rejected before any launch)
    assert L.polymul_ex(ctx.handle, a.data_ptr(), 1 << 62, a.data_ptr(), 2, out.data_ptr(), None) == fpmul.EINVAL
    assert "2^62" in L.polymul_last_error().decode()
    assert L.polymul_ex(ctx.handle, a.data_ptr(), (1 << 62) + 1, a.data_ptr(), 1, out.data_ptr(), None) \
        == fpmul.EINVAL
    # workspace above the context cap
    big = dev(np.zeros(2000, np.uint64))
    big_out = dev(np.zeros(4000, np.uint64))
    small = fpmul.Context(0, workspace_cap=1 << 10)
    assert L.polymul_ex(small.handle, big.data_ptr(), 100000, big.data_ptr(), 100000, big_out.data_ptr(), None) \
        == fpmul.ENOMEM
    small.close()


# --------------------------------------------------------------------------
# transform reuse and squaring (pointwise on transforms)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("log2n", [12, 20, 24])
def test_transform_reuse_one_operand_many_products(ctx, log2n):
    rng = random.Random(log2n)
    n = 1 << log2n
    la = n // 2 - 7
    say("transform reuse", log2n)
    a = rand_words(rng, la)
    fa = ctx.addfft(dev(a), la, log2n)
    for k in range(3):
        lb = rng.randint(1, n // 2)
        b = rand_words(rng, lb)
        fb = ctx.addfft(dev(b), lb, log2n)
        fc = ctx.pointwise(fa, fb, log2n)
        got = host(ctx.iaddfft(fc, log2n, la + lb - 1))[: O.nwords(la + lb - 1)]
        if log2n <= 20:
            assert np.array_equal(got, O.polymul(a, la, b, lb)), k
        else:
            nw = O.nwords(la + lb - 1)
            idx = np.array(sorted({0, nw - 1, nw // 2} | {rng.randrange(nw) for _ in range(5)}), dtype=np.uint64)
            assert np.array_equal(got[idx.astype(np.int64)], O.product_words(a, la, b, lb, idx)), k
    # fa is still the transform of A
    assert np.array_equal(host(ctx.iaddfft(fa, log2n, la)), a)


@pytest.mark.parametrize("log2n", [7, 16, 23])
def test_squaring_through_one_transform_is_bit_spread(ctx, log2n):
    # A^2 in GF(2)[x] spreads bit i to bit 2i (Frobenius); computed as
    # addfft(A), pointwise(fa, fa) in place, iaddfft
    rng = random.Random(100 + log2n)
    n = 1 << log2n
    la = n // 2
    say("squaring", log2n)
    a = rand_words(rng, la)
    fa = ctx.addfft(dev(a), la, log2n)
    ctx.pointwise(fa, fa, log2n, fc=fa)
    got = host(ctx.iaddfft(fa, log2n, 2 * la - 1))[: O.nwords(2 * la - 1)]
    bits = np.unpackbits(a.view(np.uint8), bitorder="little")[:la]
    spread = np.zeros(2 * la - 1 + 1, dtype=np.uint8)
    spread[0:2 * la:2] = bits
    want = np.packbits(spread[: 64 * O.nwords(2 * la - 1)], bitorder="little")
    want = np.frombuffer(np.pad(want, (0, 8 * O.nwords(2 * la - 1) - want.size)).tobytes(), dtype=np.uint64)
    assert np.array_equal(got, want)


def bit_spread(words, la):
    """Words of A(x)^2 for A of la bits: bit i of A at bit 2i (Frobenius over
    GF(2)), trimmed to the 2 la - 1 bits of the square."""
    w = np.asarray(words, dtype=np.uint64)[: O.nwords(la)]

    def spread32(x):
        x = x & np.uint64(0xFFFFFFFF)
        for sh, m in ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF), (4, 0x0F0F0F0F0F0F0F0F),
                      (2, 0x3333333333333333), (1, 0x5555555555555555)):
            x = (x | (x << np.uint64(sh))) & np.uint64(m)
        return x

    out = np.empty(2 * w.size, dtype=np.uint64)
    out[0::2] = spread32(w)
    out[1::2] = spread32(w >> np.uint64(32))
    return out[: O.nwords(2 * la - 1)]


@pytest.mark.parametrize("la", [70001, (1 << 20) + 7, (1 << 24) - 3, (1 << 25) + 1, (1 << 29) + 3, (1 << 31) - 5])
def test_square_through_one_forward_transform(ctx, la):
    """polymul_ex with the same operand twice takes one forward transform and
    squares it pointwise: every route (fused with a 2^22-bit transform, the
    short-transform bottom pass, the resident-table passes, the per-step
    path above 2^31 bits) against the bit spread of A, and the smallest
    against the oracle as well."""
    say("square", la)
    a = synth.dense_poly(0x5EED5000 + la % 1000, la)
    ta = dev(a)
    got = host(ctx.polymul(ta, la, ta, la))[: O.nwords(2 * la - 1)]
    assert np.array_equal(got, bit_spread(a, la))
    if la < 1 << 17:
        assert np.array_equal(got, O.polymul(a, la, a, la, threads=8))
    del ta
    torch.cuda.empty_cache()


@pytest.mark.parametrize("la,lb", [(1000, 700), ((1 << 20) + 3, 1 << 20)])
def test_one_buffer_two_lengths_is_not_a_square(ctx, la, lb):
    # the same pointer with two lengths multiplies A by its own low lb bits
    say("one buffer", la, lb)
    a = rand_words(random.Random(la + lb), la)
    ta = dev(a)
    got = host(ctx.polymul(ta, la, ta, lb))[: O.nwords(la + lb - 1)]
    assert np.array_equal(got, O.polymul(a, la, O.int_to_words(O.words_to_int(a, la) & ((1 << lb) - 1), lb), lb,
                                         threads=8))


def test_pointwise_rejects_bad_arguments(ctx):
    from paper_1803_11301_amd import fpmul
    t = torch.zeros(64, dtype=torch.int64, device="cuda")
    with pytest.raises(fpmul.FpmulError):
        ctx.pointwise(t, t, 5)
    with pytest.raises(fpmul.FpmulError):
        ctx.pointwise(t[:32], t[16:48], 11, fc=t[8:40])   # overlapping output that is neither input


@pytest.mark.parametrize("la,lb", [(1 << 16, 1 << 16), ((1 << 16) + 5, (1 << 16) - 9), (1 << 15, (1 << 16) + 1),
                                   (1 << 17, 1 << 17), ((1 << 18) + 3, (1 << 18) - 7), (1 << 19, 1 << 19),
                                   ((1 << 20) - 10, 5), ((1 << 19) - 1, (1 << 19) + 5), (1 << 20, 1 << 20),
                                   (1000, (1 << 20) - 1), ((1 << 20) + 1, 1 << 10)])
def test_mid_size_products_exact(ctx, la, lb):
    """Products of more than 2^16 and at most 2^21 bits, computed with 2^22-bit
    transforms on the fused path (short operands: few rows, short columns;
    operands of different row counts one after the other)."""
    say("mid size", la, lb)
    rng = random.Random(la * 3 + lb)
    a, b = rand_words(rng, la), rand_words(rng, lb)
    assert np.array_equal(gpu_product(ctx, a, la, b, lb), O.polymul(a, la, b, lb, threads=8))
