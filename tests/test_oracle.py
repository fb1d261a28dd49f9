"""Pins for the CPU oracle (the plain product in GF(2)[x]).

Each check ties the oracle to something other than its own formula: numpy's
integer convolution taken mod 2 (a library routine that is the GF(2) product
on 0/1 arrays), closed forms of GF(2)[x] (Frobenius squaring, monomials,
geometric sums), ring laws, the exact degree of a product, evaluation at
random field points (Schwartz-Zippel), and schoolbook against Karatsuba.
"""
import random

import numpy as np
import pytest

import oracle as O
from paper_1803_11301_amd import synth


def bits_of(words, length):
    v = O.words_to_int(words, length)
    return np.array([(v >> k) & 1 for k in range(length)], dtype=np.int64)


def conv_mod2(a_words, la, b_words, lb):
    """numpy integer convolution of the 0/1 coefficient arrays, reduced mod 2."""
    c = np.convolve(bits_of(a_words, la), bits_of(b_words, lb)) % 2
    return O.int_to_words(sum(int(x) << k for k, x in enumerate(c.tolist())), la + lb - 1)


def rand_poly(rng, length):
    v = rng.getrandbits(length) if length else 0
    return O.int_to_words(v, length), v


def test_clmul_word_soft_equals_hw():
    rng = random.Random(1)
    if O.set_impl(-1) != 1:
        pytest.skip("host has no PCLMULQDQ")
    for _ in range(2000):
        a, b = rng.getrandbits(64), rng.getrandbits(64)
        assert O.clmul64(a, b, hw=False) == O.clmul64(a, b, hw=True)
    assert O.clmul64(1 << 63, 1 << 63, hw=False) == 1 << 126


@pytest.mark.parametrize("method", ["schoolbook", "karatsuba"])
def test_all_pairs_up_to_8_bits_against_convolution(method):
    # every pair of polynomials with len_a, len_b in {1..8}: checked against
    # numpy's convolution for a sample of lengths and exhaustively at 8x8
    for la in (1, 3, 8):
        for lb in (1, 5, 8):
            for av in range(1 << la):
                for bv in range(0, 1 << lb, 7 if la * lb > 16 else 1):
                    aw = O.int_to_words(av, la)
                    bw = O.int_to_words(bv, lb)
                    got = O.polymul(aw, la, bw, lb, method=method)
                    assert O.words_to_int(got, la + lb - 1) == O.words_to_int(conv_mod2(aw, la, bw, lb), la + lb - 1)


def test_exhaustive_8x8_products_equal_python_ints():
    # all 2^16 pairs of 8-bit polynomials: the carry-less product is also the
    # integer product with carries discarded bit by bit, i.e. XOR of shifts
    table = {}
    for av in range(256):
        for bv in range(256):
            table[(av, bv)] = O.py_clmul(av, bv)
    aw = np.zeros(1, np.uint64)
    bw = np.zeros(1, np.uint64)
    for av in range(256):
        for bv in range(256):
            aw[0] = av
            bw[0] = bv
            got = O.polymul(aw, 8, bw, 8, method="karatsuba")
            assert int(got[0]) == table[(av, bv)]


@pytest.mark.parametrize("seed", range(6))
def test_random_lengths_against_convolution(seed):
    rng = random.Random(100 + seed)
    for _ in range(4):
        la, lb = rng.randint(1, 300), rng.randint(1, 300)
        aw, _ = rand_poly(rng, la)
        bw, _ = rand_poly(rng, lb)
        ref = conv_mod2(aw, la, bw, lb)
        for method in ("schoolbook", "karatsuba"):
            assert np.array_equal(O.polymul(aw, la, bw, lb, method=method), ref)


@pytest.mark.parametrize("la,lb", [(64 * 33, 64 * 33), (64 * 100 + 5, 64 * 37 + 63), (2 ** 16, 2 ** 16),
                                   (2 ** 16 - 1, 3), (64 * 65, 64 * 64 + 1), (1 << 15, (1 << 15) + 77)])
def test_karatsuba_equals_schoolbook(la, lb):
    rng = random.Random(la * 7 + lb)
    aw, _ = rand_poly(rng, la)
    bw, _ = rand_poly(rng, lb)
    s = O.polymul(aw, la, bw, lb, method="schoolbook")
    k1 = O.polymul(aw, la, bw, lb, method="karatsuba", threads=1)
    k8 = O.polymul(aw, la, bw, lb, method="karatsuba", threads=8)
    assert np.array_equal(s, k1)
    assert np.array_equal(s, k8)


def test_square_is_bit_spread():
    # Frobenius in GF(2)[x]: A(x)^2 = A(x^2), bit i of A goes to bit 2i
    rng = random.Random(5)
    for la in (1, 63, 64, 65, 1000, 4096 + 17):
        aw, av = rand_poly(rng, la)
        got = O.words_to_int(O.polymul(aw, la, aw, la), 2 * la - 1)
        spread = 0
        for k in range(la):
            if (av >> k) & 1:
                spread |= 1 << (2 * k)
        assert got == spread


def test_monomials_and_geometric_sums():
    for a in (0, 1, 63, 64, 100, 1000):
        for b in (0, 5, 64, 777):
            aw = O.int_to_words(1 << a, a + 1)
            bw = O.int_to_words(1 << b, b + 1)
            assert O.words_to_int(O.polymul(aw, a + 1, bw, b + 1), a + b + 1) == 1 << (a + b)
    for a in (1, 3, 64, 129):
        p = (1 << a) | 1
        w = O.int_to_words(p, a + 1)
        assert O.words_to_int(O.polymul(w, a + 1, w, a + 1), 2 * a + 1) == (1 << (2 * a)) | 1
    for k in (1, 2, 63, 64, 65, 500, 4100):
        ones = O.int_to_words((1 << k) - 1, k)
        xp1 = O.int_to_words(0b11, 2)
        assert O.words_to_int(O.polymul(xp1, 2, ones, k), k + 1) == (1 << k) | 1


def test_ring_laws_and_degree():
    rng = random.Random(9)
    for _ in range(5):
        la, lb, lc = rng.randint(100, 3000), rng.randint(100, 3000), rng.randint(100, 3000)
        aw, av = rand_poly(rng, la)
        bw, bv = rand_poly(rng, lb)
        cw, cv = rand_poly(rng, lc)
        ab = O.polymul(aw, la, bw, lb)
        ba = O.polymul(bw, lb, aw, la)
        assert np.array_equal(ab, ba)
        # distributivity A (B + C) = A B + A C
        L = max(lb, lc)
        bc = O.int_to_words(bv ^ cv, L)
        left = O.words_to_int(O.polymul(aw, la, bc, L), la + L - 1)
        right = O.words_to_int(ab, la + lb - 1) ^ O.words_to_int(O.polymul(aw, la, cw, lc), la + lc - 1)
        assert left == right
        # associativity (A B) C = A (B C)
        abc1 = O.words_to_int(O.polymul(ab, la + lb - 1, cw, lc), la + lb + lc - 2)
        bcw = O.polymul(bw, lb, cw, lc)
        abc2 = O.words_to_int(O.polymul(aw, la, bcw, lb + lc - 1), la + lb + lc - 2)
        assert abc1 == abc2
        # exact degree: deg(AB) = deg A + deg B (GF(2)[x] has no zero divisors)
        da, db = av.bit_length() - 1, bv.bit_length() - 1
        assert O.words_to_int(ab, la + lb - 1).bit_length() - 1 == da + db
    one = O.int_to_words(1, 1)
    aw, av = rand_poly(rng, 777)
    assert O.words_to_int(O.polymul(aw, 777, one, 1), 777) == av
    zero = O.int_to_words(0, 10)
    assert O.words_to_int(O.polymul(aw, 777, zero, 10), 786) == 0


def test_tail_bits_ignored_and_output_tail_zero():
    la, lb = 70, 65
    aw = np.array([~np.uint64(0), ~np.uint64(0)], np.uint64)
    bw = np.array([~np.uint64(0), ~np.uint64(0)], np.uint64)
    got = O.polymul(aw, la, bw, lb)
    ref = conv_mod2(O.int_to_words((1 << la) - 1, la), la, O.int_to_words((1 << lb) - 1, lb), lb)
    assert np.array_equal(got, ref)
    assert int(got[-1]) >> ((la + lb - 1) % 64) == 0


def test_empty_operands():
    assert O.polymul(np.zeros(0, np.uint64), 0, np.ones(1, np.uint64), 1).size == 0


def test_field_modulus_is_irreducible():
    from oracle import cantor
    assert cantor.is_irreducible_modulus()


def test_field_mul_c_and_python_agree():
    from oracle import cantor
    rng = random.Random(3)
    for _ in range(500):
        x, y = rng.getrandbits(64), rng.getrandbits(64)
        assert O.gf64_mul(x, y) == cantor.mul(x, y)
    # x * x^63 = x^64 = x^4 + x^3 + x + 1
    assert O.gf64_mul(2, 1 << 63) == 0x1B


def test_eval_matches_bitwise_horner():
    from oracle import cantor
    rng = random.Random(4)
    for la in (1, 64, 65, 300):
        aw, av = rand_poly(rng, la)
        z = rng.getrandbits(64)
        assert O.eval_at(aw, la, z) == cantor.eval_gf2poly(av, z)


@pytest.mark.parametrize("la,lb", [(2 ** 16, 2 ** 16), (12345, 54321), (64, 1)])
def test_product_at_random_points(la, lb):
    # Schwartz-Zippel: C(z) = A(z) B(z) at random z in GF(2^64)
    rng = random.Random(la ^ lb)
    aw, _ = rand_poly(rng, la)
    bw, _ = rand_poly(rng, lb)
    cw = O.polymul(aw, la, bw, lb)
    for _ in range(8):
        z = rng.getrandbits(64)
        assert O.eval_at(cw, la + lb - 1, z) == O.gf64_mul(O.eval_at(aw, la, z), O.eval_at(bw, lb, z))


def test_sampled_words_equal_full_product():
    a, b = synth.single_pair(synth.SEED_SMALL, 1 << 12)
    full = O.polymul(a, 1 << 12, b, 1 << 12)
    idx = np.array([0, 1, 17, 63, 64, 100, full.size - 1, full.size + 3], np.uint64)
    got = O.product_words(a, 1 << 12, b, 1 << 12, idx)
    for q, w in enumerate(idx.tolist()):
        assert int(got[q]) == (int(full[w]) if w < full.size else 0)


def test_planted_mistake_is_caught():
    # a product with one flipped coefficient must fail the point check
    rng = random.Random(11)
    aw, _ = rand_poly(rng, 500)
    bw, _ = rand_poly(rng, 400)
    cw = O.polymul(aw, 500, bw, 400).copy()
    cw[3] ^= np.uint64(1 << 7)
    z = rng.getrandbits(64)
    assert O.eval_at(cw, 899, z) != O.gf64_mul(O.eval_at(aw, 500, z), O.eval_at(bw, 400, z))
