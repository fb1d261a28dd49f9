"""Cantor basis and evaluation points of the method (test infrastructure only).

Plain, slow Python on ints.  Used to state what the intermediate transforms
must equal by definition, so that HIP stages can be checked one by one:

* the field: GF(2^64) = GF(2)[x]/(x^64 + x^4 + x^3 + x + 1) (Sec. 4.3);
* the Cantor basis v_0 = 1, v_i^2 + v_i = v_{i-1} (Sec. 2.2, Eq. 2), each v_i
  written in that polynomial representation.  Each equation has two roots,
  v and v + 1; this module takes the root whose bit 0 is clear (a reading: the
  paper does not fix the root, and the product does not depend on it);
* Cantor coordinates: the element whose vector is the integer c is
  sum_{bit i of c} v_i (Sec. 2.2, the "line" notation);
* subspace polynomials s_i via the recursion s_0 = x, s_{i+1} = s_i^2 + s_i
  (Sec. 2.2.2), which are GF(2)[x] polynomials;
* the novelpoly basis X_k = prod_{bit i of k} s_i (Def. novelpoly), and the
  conversion of a bit polynomial to it by repeated division by s_i (the
  Bernstein-Chou form the paper describes in Sec. 2.3.1) -- the plain
  definition of the BasisCvt output;
* the evaluation points of the Frobenius partition Sigma = v_{l+m/2} + V_l
  (Eq. 6): point j is the element with Cantor vector 2^(l+32) XOR j, so that
  the transform output j is A(point j) (Eq. 8 together with Alg. 2's output
  order).
"""
from __future__ import annotations

from functools import lru_cache

M = 64
MOD_LOW = 0x1B  # x^4 + x^3 + x + 1
MASK = (1 << 64) - 1


def clmul(a: int, b: int) -> int:
    r = 0
    while b:
        low = b & -b
        r ^= a << (low.bit_length() - 1)
        b ^= low
    return r


def reduce128(p: int) -> int:
    """p mod (x^64 + x^4 + x^3 + x + 1) by long division from the top bit."""
    while p >> 64:
        k = p.bit_length() - 1
        p ^= (1 << k) ^ (MOD_LOW << (k - 64))
    return p


def mul(a: int, b: int) -> int:
    return reduce128(clmul(a, b))


def sqr(a: int) -> int:
    return mul(a, a)


def power(a: int, e: int) -> int:
    r = 1
    while e:
        if e & 1:
            r = mul(r, a)
        a = sqr(a)
        e >>= 1
    return r


def _solve_artin_schreier(c: int) -> int:
    """The root x of x^2 + x = c with bit 0 clear (Gaussian elimination on the
    GF(2)-linear map x -> x^2 + x, whose kernel is {0, 1})."""
    cols = [sqr(1 << t) ^ (1 << t) for t in range(M)]
    # equations: row r says sum_t x_t * bit_r(cols[t]) = bit_r(c)
    rows = []
    for r in range(M):
        mask = 0
        for t in range(M):
            if (cols[t] >> r) & 1:
                mask |= 1 << t
        rows.append([mask, (c >> r) & 1])
    piv_of_col = {}
    rank = 0
    for t in range(M):
        p = next((r for r in range(rank, M) if (rows[r][0] >> t) & 1), None)
        if p is None:
            continue
        rows[rank], rows[p] = rows[p], rows[rank]
        for r in range(M):
            if r != rank and (rows[r][0] >> t) & 1:
                rows[r][0] ^= rows[rank][0]
                rows[r][1] ^= rows[rank][1]
        piv_of_col[t] = rank
        rank += 1
    for r in range(rank, M):
        if rows[r][1]:
            raise ValueError("no root")
    x = 0
    for t, r in piv_of_col.items():
        if rows[r][1]:
            x |= 1 << t
    if x & 1:
        x ^= 1
    assert sqr(x) ^ x == c
    return x


@lru_cache(maxsize=None)
def cantor_basis() -> tuple:
    v = [1]
    for i in range(1, M):
        v.append(_solve_artin_schreier(v[-1]))
    return tuple(v)


def iota(cvec: int) -> int:
    """Element with Cantor coordinate vector cvec, in the polynomial representation."""
    v = cantor_basis()
    r = 0
    i = 0
    while cvec:
        if cvec & 1:
            r ^= v[i]
        cvec >>= 1
        i += 1
    return r


@lru_cache(maxsize=None)
def tower_basis() -> tuple:
    """Polynomial-representation images of the 64 unit vectors of the tower
    representation the GPU path stores values in: unit 8k+u is v_u * W_k with
    W_k = v_8^(k&1) v_16^((k>>1)&1) v_32^(k>>2).  (A representation choice of
    the implementation, independent of the paper; the product does not depend
    on it.)"""
    v = cantor_basis()
    out = []
    for k in range(8):
        w = 1
        if k & 1:
            w = mul(w, v[8])
        if k & 2:
            w = mul(w, v[16])
        if k & 4:
            w = mul(w, v[32])
        for u in range(8):
            out.append(mul(v[u], w))
    return tuple(out)


def tower_to_poly(x: int) -> int:
    tb = tower_basis()
    r = 0
    t = 0
    while x:
        if x & 1:
            r ^= tb[t]
        x >>= 1
        t += 1
    return r


def point(l: int, j: int) -> int:
    """Point j of Sigma = v_{l+32} + V_l: Cantor vector 2^(l+32) XOR j."""
    return iota((1 << (l + 32)) ^ j)


@lru_cache(maxsize=None)
def subspace_poly(i: int) -> int:
    """s_i as a GF(2)[x] polynomial (int bit k = coefficient of x^k), via
    s_0 = x and s_{i+1} = s_i^2 + s_i."""
    s = 0b10
    for _ in range(i):
        s = clmul(s, s) ^ s
    return s


def novelpoly_X(k: int) -> int:
    """X_k = product of s_i over the set bits i of k (GF(2)[x] polynomial)."""
    r = 1
    i = 0
    while k:
        if k & 1:
            r = clmul(r, subspace_poly(i))
        k >>= 1
        i += 1
    return r


def _polydivmod(a: int, b: int):
    q = 0
    db = b.bit_length() - 1
    while a and a.bit_length() - 1 >= db:
        s = a.bit_length() - 1 - db
        q ^= 1 << s
        a ^= b << s
    return q, a


def to_novelpoly(f: int, n: int) -> int:
    """Coefficients g of f = sum_k g_k X_k (f of degree < n, n a power of 2),
    by dividing by s_t with 2^t = n/2 and recursing on remainder and quotient."""
    if n <= 2:
        return f
    t = (n // 2).bit_length() - 1
    q, r = _polydivmod(f, subspace_poly(t))
    return to_novelpoly(r, n // 2) | (to_novelpoly(q, n // 2) << (n // 2))


def from_novelpoly(g: int) -> int:
    """f = sum_k g_k X_k."""
    f = 0
    k = 0
    while g:
        if g & 1:
            f ^= novelpoly_X(k)
        g >>= 1
        k += 1
    return f


def eval_gf2poly(f: int, z: int) -> int:
    """f(z) for a GF(2)[x] polynomial f and field element z (Horner)."""
    acc = 0
    for k in range(f.bit_length() - 1, -1, -1):
        acc = mul(acc, z) ^ ((f >> k) & 1)
    return acc


def eval_field_poly(coeffs, z: int) -> int:
    """sum_k coeffs[k] z^k with field-element coefficients."""
    acc = 0
    for c in reversed(coeffs):
        acc = mul(acc, z) ^ c
    return acc


def is_irreducible_modulus() -> bool:
    """Rabin's test for x^64 + x^4 + x^3 + x + 1: x^(2^64) = x mod P and
    gcd(x^(2^32) - x, P) = 1 (64 has the single prime divisor 2)."""
    P = (1 << 64) | MOD_LOW

    def polymod(a, b):
        return _polydivmod(a, b)[1]

    def gcd(a, b):
        while b:
            a, b = b, polymod(a, b)
        return a

    x = 0b10
    y = x
    for _ in range(32):
        y = mul(y, y)
    if gcd(P, y ^ x) != 1:
        return False
    for _ in range(32):
        y = mul(y, y)
    return y == x
