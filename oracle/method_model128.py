"""The m = 128 variant of the paper's multiplication in plain Python (test
infrastructure only).

The same steps as ``method_model`` (Alg. 5: BasisCvt, Encode, Butterfly,
pointwise products, and their inverses) over GF(2^128) with l_m = 7, for
small n, so that the reading taken for m = 128 is checked against the plain
product on the CPU:

* the field: GF(2)[x] / (x^128 + x^7 + x^2 + x + 1) (the polynomial the
  paper names for its m = 128 variant, Sec. 4.3), written here with its own
  Cantor basis v_0 = 1, v_i^2 + v_i = v_{i-1}, each root taken with bit 0
  clear (the rule of ``cantor`` for m = 64);
* Encode rows r_j = product of v_{64-k} over the set bits k of j, k < 7
  (Eq. 9 read as for m = 64: layer l + k of the virtual length-n transform
  multiplies by s_{l+k}(v_{l+64}) = v_{64-k});
* Butterfly at alpha = v_{l+64} (Alg. 2), s_i(z) = the Cantor vector of z
  shifted right by i (Eq. 4).

BasisCvt does not depend on the field: ``cantor.to_novelpoly``.
"""
from __future__ import annotations

from functools import lru_cache

from . import cantor

M = 128
LM = 7
MOD_LOW = (1 << 7) | (1 << 2) | (1 << 1) | 1   # x^7 + x^2 + x + 1


def clmul(a: int, b: int) -> int:
    return cantor.clmul(a, b)


def reduce(p: int) -> int:
    """p mod (x^128 + x^7 + x^2 + x + 1) by long division from the top bit."""
    while p >> M:
        k = p.bit_length() - 1
        p ^= (1 << k) ^ (MOD_LOW << (k - M))
    return p


def mul(a: int, b: int) -> int:
    return reduce(clmul(a, b))


def is_irreducible_modulus() -> bool:
    """Rabin's test: x^(2^128) = x mod P and gcd(x^(2^64) - x, P) = 1
    (128 has the single prime divisor 2)."""
    P = (1 << M) | MOD_LOW

    def polymod(a, b):
        return cantor._polydivmod(a, b)[1]

    def gcd(a, b):
        while b:
            a, b = b, polymod(a, b)
        return a

    x = 0b10
    y = x
    for _ in range(64):
        y = mul(y, y)
    if gcd(P, y ^ x) != 1:
        return False
    for _ in range(64):
        y = mul(y, y)
    return y == x


def _solve_artin_schreier(c: int) -> int:
    """The root of x^2 + x = c with bit 0 clear (Gaussian elimination on the
    GF(2)-linear map x -> x^2 + x, whose kernel is {0, 1})."""
    cols = [mul(1 << t, 1 << t) ^ (1 << t) for t in range(M)]
    rows = []
    for r in range(M):
        mask = 0
        for t in range(M):
            if (cols[t] >> r) & 1:
                mask |= 1 << t
        rows.append([mask, (c >> r) & 1])
    piv = {}
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
        piv[t] = rank
        rank += 1
    for r in range(rank, M):
        if rows[r][1]:
            raise ValueError("no root")
    x = 0
    for t, r in piv.items():
        if rows[r][1]:
            x |= 1 << t
    if x & 1:
        x ^= 1
    assert mul(x, x) ^ x == c
    return x


@lru_cache(maxsize=None)
def cantor_basis() -> tuple:
    v = [1]
    for _ in range(1, M):
        v.append(_solve_artin_schreier(v[-1]))
    return tuple(v)


def iota(cvec: int) -> int:
    """Element with Cantor coordinate vector cvec."""
    v = cantor_basis()
    r = 0
    i = 0
    while cvec:
        if cvec & 1:
            r ^= v[i]
        cvec >>= 1
        i += 1
    return r


def s_eval(i: int, cvec: int) -> int:
    """s_i at the element with Cantor vector cvec (Eq. 4)."""
    return iota(cvec >> i)


def encode_rows(index=lambda k: M // 2 - k) -> list:
    """r_j = product of v_{index(k)} over the set bits k < LM of j."""
    v = cantor_basis()
    rows = []
    for j in range(M):
        r = 1
        for k in range(LM):
            if (j >> k) & 1:
                r = mul(r, v[index(k)])
        rows.append(r)
    return rows


def rank(vectors) -> int:
    basis = {}
    for val in vectors:
        for b in sorted(basis, reverse=True):
            if (val >> b) & 1:
                val ^= basis[b]
        if val:
            basis[val.bit_length() - 1] = val
    return len(basis)


def inverse_rows(rows: list) -> list:
    """Q with: if f = XOR_{bit j of a} rows[j] then a = XOR_{bit t of f} Q[t]."""
    n = len(rows)
    basis = {}
    for j, val in enumerate(rows):
        comb = 1 << j
        for b in sorted(basis, reverse=True):
            if (val >> b) & 1:
                val ^= basis[b][0]
                comb ^= basis[b][1]
        if val == 0:
            raise ValueError("singular")
        hb = val.bit_length() - 1
        for b in list(basis):
            if (basis[b][0] >> hb) & 1:
                basis[b] = (basis[b][0] ^ val, basis[b][1] ^ comb)
        basis[hb] = (val, comb)
    return [basis[t][1] for t in range(n)]


def x_basis_at(cvec: int, l: int) -> list:
    """[X_k(x) for k < 2^l] at the point with Cantor vector cvec: X_k is the
    product of s_i over the set bits of k (s_i(v_i) = 1 for this basis)."""
    vals = [1]
    for i in range(l):
        si = s_eval(i, cvec)
        vals = vals + [mul(v, si) for v in vals]
    return vals


def evaluate(g: list, alpha_c: int) -> list:
    """Values of sum_k g_k X_k at alpha + j (alpha as a Cantor vector), from
    the definition of the basis: what Alg. 2 computes."""
    l = len(g).bit_length() - 1
    out = []
    for j in range(len(g)):
        v = 0
        for gk, xk in zip(g, x_basis_at(alpha_c ^ j, l)):
            if gk:
                v ^= mul(gk, xk)
        out.append(v)
    return out


def _inv(a: int) -> int:
    r, e = 1, (1 << M) - 2
    while e:
        if e & 1:
            r = mul(r, a)
        a = mul(a, a)
        e >>= 1
    return r


def interpolate(vals: list, alpha_c: int) -> list:
    """g with evaluate(g, alpha_c) == vals, by Gauss-Jordan elimination on
    [X_k(alpha + j)] over GF(2^128) (distinct points, deg X_k = k)."""
    n = len(vals)
    l = n.bit_length() - 1
    rows = [x_basis_at(alpha_c ^ j, l) + [vals[j]] for j in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if rows[r][col])
        rows[col], rows[piv] = rows[piv], rows[col]
        inv = _inv(rows[col][col])
        rows[col] = [mul(inv, x) for x in rows[col]]
        for r in range(n):
            if r != col and rows[r][col]:
                f = rows[r][col]
                rows[r] = [x ^ mul(f, y) for x, y in zip(rows[r], rows[col])]
    return [rows[k][n] for k in range(n)]


def params(n: int):
    l = n.bit_length() - 1 - LM
    assert n == 1 << (l + LM) and l >= 0
    return l, 1 << l


def encode(abits: int, n: int) -> list:
    l, n_p = params(n)
    r = encode_rows()
    out = []
    for i in range(n_p):
        f = 0
        for j in range(M):
            if (abits >> (j * n_p + i)) & 1:
                f ^= r[j]
        out.append(f)
    return out


def decode(h: list, n: int) -> int:
    l, n_p = params(n)
    q = inverse_rows(encode_rows())
    bits = 0
    for i in range(n_p):
        a = 0
        for t in range(M):
            if (h[i] >> t) & 1:
                a ^= q[t]
        for j in range(M):
            if (a >> j) & 1:
                bits |= 1 << (j * n_p + i)
    return bits


def forward(a: int, n: int) -> list:
    """BasisCvt, Encode, Butterfly at alpha = v_{l+64}."""
    l, _ = params(n)
    return evaluate(encode(cantor.to_novelpoly(a, n), n), 1 << (l + M // 2))


def inverse(vals: list, n: int) -> int:
    l, _ = params(n)
    return cantor.from_novelpoly(decode(interpolate(vals, 1 << (l + M // 2)), n))


def fp_polymul(a: int, len_a: int, b: int, len_b: int) -> int:
    """Alg. 5 over GF(2^128) on Python-int bit polynomials (n >= 128)."""
    if len_a == 0 or len_b == 0:
        return 0
    n = 128
    while n < len_a + len_b - 1:
        n *= 2
    a &= (1 << len_a) - 1
    b &= (1 << len_b) - 1
    ha, hb = forward(a, n), forward(b, n)
    return inverse([mul(x, y) for x, y in zip(ha, hb)], n)


def eval_gf2poly(f: int, z: int) -> int:
    acc = 0
    for k in range(f.bit_length() - 1, -1, -1):
        acc = mul(acc, z) ^ ((f >> k) & 1)
    return acc
