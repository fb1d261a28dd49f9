"""Pins for the Cantor-basis field facts and for the step-by-step model of Alg. 5.

The facts checked are the ones the paper states (Sec. 2.2-3): the basis
recursion, nested subfields, the order of squaring on basis elements (Eq. 5),
s_i(v_j) = v_{j-i} (Eq. 4), two-term subspace polynomials for power-of-two i,
Prop. 1 (Sigma is a Frobenius partition, |Omega| = n) and Prop. 2 (E_Sigma is
a bijection).  The model of the method must reproduce the plain product and
its transform must equal evaluation at the points of Sigma.
"""
import random

import numpy as np
import pytest

import oracle as O
from oracle import cantor as F
from oracle import method_model as MM


def cantor_coords(x):
    """Inverse of iota by elimination over the basis (test-side helper)."""
    v = F.cantor_basis()
    rows = [(v[i], 1 << i) for i in range(64)]
    basis = {}
    for val, comb in rows:
        for b in sorted(basis, reverse=True):
            if (val >> b) & 1:
                val ^= basis[b][0]
                comb ^= basis[b][1]
        assert val
        basis[val.bit_length() - 1] = (val, comb)
    c = 0
    for b in sorted(basis, reverse=True):
        if (x >> b) & 1:
            x ^= basis[b][0]
            c ^= basis[b][1]
    assert x == 0
    return c


def test_basis_recursion_and_independence():
    v = F.cantor_basis()
    assert v[0] == 1
    for i in range(1, 64):
        assert F.sqr(v[i]) ^ v[i] == v[i - 1]
        assert v[i] & 1 == 0  # the stated root choice
    cantor_coords(0)  # elimination succeeds only for an independent basis


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_nested_subfields(k):
    # V_{2^k} = span(v_0 .. v_{2^k - 1}) is a subfield (Sec. 2.2.1)
    rng = random.Random(k)
    size = 1 << k
    for _ in range(40):
        x = F.iota(rng.getrandbits(size))
        y = F.iota(rng.getrandbits(size))
        assert cantor_coords(F.mul(x, y)) >> size == 0


def test_order_of_squaring_on_basis():
    # Ord_phi(v_i) = 2 * 2^floor(log2 i) for i > 0 (Eq. 5)
    v = F.cantor_basis()
    for i in list(range(1, 20)) + [31, 32, 33, 47, 63]:
        x, j = v[i], 0
        while True:
            x = F.sqr(x)
            j += 1
            if x == v[i]:
                break
        assert j == 2 * (1 << (i.bit_length() - 1))


def test_squaring_in_cantor_coordinates_is_shift_xor():
    rng = random.Random(2)
    for _ in range(30):
        c = rng.getrandbits(64)
        assert cantor_coords(F.sqr(F.iota(c))) == c ^ (c >> 1)


def test_subspace_polynomial_is_product_over_subspace():
    # s_i(x) = prod_{a in V_i} (x - a), expanded over GF(2^64), for i <= 4
    for i in range(5):
        coeffs = [1]  # field-coefficient polynomial, index = degree
        for a_c in range(1 << i):
            a = F.iota(a_c)
            nxt = [0] * (len(coeffs) + 1)
            for d, c in enumerate(coeffs):
                nxt[d + 1] ^= c
                nxt[d] ^= F.mul(c, a)
            coeffs = nxt
        s = F.subspace_poly(i)
        assert all(c in (0, 1) for c in coeffs)
        assert sum(c << d for d, c in enumerate(coeffs)) == s


def test_two_term_subspace_polynomials():
    for i in range(1, 12):
        two = F.subspace_poly(i) == (1 << (1 << i)) | 2
        assert two == (i & (i - 1) == 0)


def test_subspace_polynomial_values_are_shifts():
    # s_i(v_j) = v_{j-i} for j >= i, so s_i(alpha) = alpha-bar >> i (Eq. 4)
    rng = random.Random(7)
    for i in range(0, 7):
        s = F.subspace_poly(i)
        for _ in range(6):
            c = rng.getrandbits(64)
            assert F.eval_gf2poly(s, F.iota(c)) == F.iota(c >> i)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_frobenius_partition(l):
    # Prop. 1: the m images of Sigma under squaring are disjoint, the m-th is Sigma
    sigma = {F.point(l, j) for j in range(1 << l)}
    seen = set()
    cur = set(sigma)
    for _ in range(64):
        assert not (cur & seen)
        seen |= cur
        cur = {F.sqr(x) for x in cur}
    assert cur == sigma
    assert len(seen) == 64 << l


@pytest.mark.parametrize("l", [0, 1])
def test_evaluation_at_sigma_is_a_bijection(l):
    # Prop. 2: A -> (A(p))_{p in Sigma} on GF(2)[x]_{<n} has full rank n
    n = 64 << l
    pts = [F.point(l, j) for j in range(1 << l)]
    basis = {}
    for k in range(n):
        img = 0
        for j, p in enumerate(pts):
            img |= F.eval_gf2poly(1 << k, p) << (64 * j)
        for b in sorted(basis, reverse=True):
            if (img >> b) & 1:
                img ^= basis[b]
        assert img != 0
        basis[img.bit_length() - 1] = img


def test_novelpoly_conversion():
    for f in range(1 << 8):
        g = F.to_novelpoly(f, 256)
        assert F.from_novelpoly(g) == f
    assert F.to_novelpoly(0b100, 4) == 0b110          # x^2 = X_1 + X_2
    assert F.to_novelpoly(0b1000, 4) == 0b1110        # x^3 = X_1 + X_2 + X_3
    for k in range(40):
        assert F.novelpoly_X(k).bit_length() - 1 == k  # deg X_k = k
    for t in range(5):
        assert F.to_novelpoly(F.subspace_poly(t), 1 << (t + 1)) == 1 << (1 << t)


def test_encode_reading_full_rank_and_literal_index_singular():
    v = F.cantor_basis()
    rows = MM.encode_rows()
    MM.gf2_inverse_rows(rows)   # raises if singular
    literal = []
    for j in range(64):
        r = 1
        for k in range(6):
            if (j >> k) & 1:
                r = F.mul(r, v[32 - 1 - k])
        literal.append(r)
    with pytest.raises(ValueError):
        MM.gf2_inverse_rows(literal)


@pytest.mark.parametrize("l", [0, 1, 2, 4])
def test_transform_is_evaluation_at_sigma(l):
    rng = random.Random(l)
    n = 64 << l
    a = rng.getrandbits(n // 2)
    vals = MM.forward(a, n)
    for j in range(1 << l):
        assert vals[j] == F.eval_gf2poly(a, F.point(l, j))
    assert MM.inverse(vals, n) == a


def test_frobenius_identity_on_transform():
    # transform(A^2) = transform(A)^2 elementwise (Eq. 1)
    rng = random.Random(21)
    n = 256
    a = rng.getrandbits(n // 2)
    a2 = O.py_clmul(a, a)
    assert MM.forward(a2, n) == [F.sqr(x) for x in MM.forward(a, n)]


@pytest.mark.parametrize("la,lb", [(1, 1), (3, 4), (33, 31), (64, 1), (100, 29), (257, 255), (700, 324), (1000, 1049)])
def test_model_product_equals_oracle(la, lb):
    rng = random.Random(la * 1000 + lb)
    a, b = rng.getrandbits(la), rng.getrandbits(lb)
    ref = O.py_clmul(a, b)
    assert MM.fp_polymul(a, la, b, lb) == ref


def test_model_exhaustive_small():
    for a in range(0, 1 << 6):
        for b in range(0, 1 << 6, 3):
            assert MM.fp_polymul(a, 6, b, 6) == O.py_clmul(a, b)


def test_tower_basis_is_a_basis_and_multiplicative():
    # the 64 tower units are independent, and multiplying by an element of V_8
    # acts on each byte alone (V_8 = GF(2^8) is a subfield, Sec. 2.2.1)
    tb = F.tower_basis()
    basis = {}
    for t, x in enumerate(tb):
        for b in sorted(basis, reverse=True):
            if (x >> b) & 1:
                x ^= basis[b]
        assert x
        basis[x.bit_length() - 1] = x
    beta = F.iota(0b10110110)
    for k in range(8):
        for u in range(8):
            prod = F.mul(tb[8 * k + u], beta)
            # the product must lie in the span of the units of byte k
            span = {}
            for w in range(8):
                y = tb[8 * k + w]
                for b in sorted(span, reverse=True):
                    if (y >> b) & 1:
                        y ^= span[b]
                span[y.bit_length() - 1] = y
            for b in sorted(span, reverse=True):
                if (prod >> b) & 1:
                    prod ^= span[b]
            assert prod == 0


# --------------------------------------------------------------------------
# m = 128 (GF(2^128), l_m = 7): the same readings one field up
# --------------------------------------------------------------------------

from oracle import method_model128 as M128   # noqa: E402


def test_m128_modulus_irreducible_and_basis():
    assert M128.is_irreducible_modulus()
    v = M128.cantor_basis()
    assert v[0] == 1
    for i in range(1, 128):
        assert M128.mul(v[i], v[i]) ^ v[i] == v[i - 1]
    assert M128.rank(v) == 128
    # V_64 = span(v_0 .. v_63) is the subfield GF(2^64): closed under products
    rng = random.Random(64)
    for _ in range(20):
        x = M128.iota(rng.getrandbits(64))
        y = M128.iota(rng.getrandbits(64))
        assert M128.rank(list(v[:64]) + [M128.mul(x, y)]) == 64


def test_m128_encode_reading_full_rank_and_literal_index_singular():
    assert M128.rank(M128.encode_rows()) == 128
    M128.inverse_rows(M128.encode_rows())
    literal = M128.encode_rows(index=lambda k: 64 - 1 - k)
    assert M128.rank(literal) < 128
    with pytest.raises(ValueError):
        M128.inverse_rows(literal)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_m128_transform_is_evaluation_at_sigma(l):
    rng = random.Random(128 + l)
    n = 128 << l
    a = rng.getrandbits(n // 2)
    vals = M128.forward(a, n)
    for j in range(1 << l):
        assert vals[j] == M128.eval_gf2poly(a, M128.iota((1 << (l + 64)) ^ j))
    assert M128.inverse(vals, n) == a


@pytest.mark.parametrize("la,lb", [(1, 1), (64, 65), (100, 29), (129, 1), (200, 300), (513, 511)])
def test_m128_model_product_equals_oracle(la, lb):
    rng = random.Random(la * 77 + lb)
    a, b = rng.getrandbits(la), rng.getrandbits(lb)
    assert M128.fp_polymul(a, la, b, lb) == O.py_clmul(a, b)


@pytest.mark.parametrize("i", [0, 1, 2, 3, 4])
def test_butterfly_step_identity(i):
    # One butterfly layer from the definitions alone: on a coset beta + V_{i+1}
    # the values of g = g_lo + X_{2^i} g_hi (X_{k + 2^i} = X_k s_i for k < 2^i)
    # are those of h0 = g_lo + s_i(beta) g_hi on beta + V_i and of
    # h1 = h0 + g_hi on beta + v_i + V_i, because s_i is GF(2)-linear, vanishes
    # on V_i and s_i(v_i) = 1 (Eq. 4).  Checked with the direct evaluation, at
    # the base points the kernels use: alpha + b 2^(i+1), alpha = v_{l+32},
    # whose multiplier is the element with Cantor vector 2^(32+l-i) + 2b.
    rng = random.Random(100 + i)
    l = i + 3
    h = 1 << i
    for b in range(1 << (l - i - 1)):
        beta = (1 << (l + 32)) ^ (b << (i + 1))
        g = [rng.getrandbits(64) for _ in range(2 * h)]
        c = MM.s_eval(i, beta)
        assert c == F.iota((1 << (32 + l - i)) ^ (2 * b))
        h0 = [g[t] ^ F.mul(c, g[h + t]) for t in range(h)]
        h1 = [h0[t] ^ g[h + t] for t in range(h)]
        assert MM.evaluate(g, beta) == MM.evaluate(h0, beta) + MM.evaluate(h1, beta ^ (1 << i))


def test_interpolate_inverts_evaluate():
    rng = random.Random(7)
    for l in range(0, 5):
        g = [rng.getrandbits(64) for _ in range(1 << l)]
        alpha = (1 << (l + 32)) ^ rng.getrandbits(l + 1) << l
        assert MM.interpolate(MM.evaluate(g, alpha), alpha) == g
