"""The paper's multiplication, step by step in plain Python (test infrastructure only).

Follows Alg. 5 (FP_Polymul) with the steps in the paper's order and notation,
for small n, so that the readings taken where the paper is ambiguous are
checked against the plain product before any kernel relies on them:

* BasisCvt (Alg. 1): the novelpoly coefficients, here by their definition
  (repeated division by s_i, ``cantor.to_novelpoly``);
* Encode (Alg. 4, Eq. 9): f_i = sum_j a_{j n_p + i} r_j.  Reading: r_j is the
  product of v_{m/2-k} over the set bits k of j (k = 0 .. l_m-1).  Bit k of j
  is the offset 2^(l+k) that the butterfly layer i = l+k of the virtual
  length-n transform pairs, and that layer multiplies by s_{l+k}(v_{l+m/2}) =
  v_{m/2-k} by Eq. 4.  The printed index m/2-1-k gives a singular matrix;
* Butterfly (Alg. 2) at alpha = v_{l+m/2}, written recursively as printed:
  h0 = p0 + s_i(alpha) p1, h1 = h0 + p1 (s_i(v_i) = 1), recurse on
  (h0, alpha) and (h1, v_i + alpha);
* pointwise products, iButterfly (the butterfly undone layer by layer),
  Decode (R^{-1} per element, then the bits back to rows), iBasisCvt.
"""
from __future__ import annotations

from . import cantor as F

M = 64
LM = 6


def s_eval(i: int, cvec: int) -> int:
    """s_i at the element with Cantor vector cvec: the vector shifted right by i (Eq. 4)."""
    return F.iota(cvec >> i)


def encode_rows() -> list:
    v = F.cantor_basis()
    rows = []
    for j in range(M):
        r = 1
        for k in range(LM):
            if (j >> k) & 1:
                r = F.mul(r, v[M // 2 - k])
        rows.append(r)
    return rows


def gf2_inverse_rows(rows: list) -> list:
    """Q with: if f = XOR_{bit j of a} rows[j] then a = XOR_{bit t of f} Q[t]."""
    n = len(rows)
    # augment: row t of matrix A (A[j] = rows[j]) ; solve for e_t
    aug = [[rows[j], 1 << j] for j in range(n)]
    # Gaussian elimination on the list of (value, combination) pairs
    basis = {}
    for val, comb in aug:
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
    q = []
    for t in range(n):
        val, comb = basis[t]
        assert val == 1 << t
        q.append(comb)
    return q


def butterfly(g: list, alpha_c: int) -> list:
    """Alg. 2: evaluations of sum_k g_k X_k at alpha + V_{log2 len}, alpha given in
    Cantor coordinates; output j is the value at alpha XOR j."""
    n = len(g)
    if n == 1:
        return [g[0]]
    i = n.bit_length() - 2
    h = n // 2
    p0, p1 = g[:h], g[h:]
    c = s_eval(i, alpha_c)
    h0 = [p0[t] ^ F.mul(c, p1[t]) for t in range(h)]
    h1 = [h0[t] ^ p1[t] for t in range(h)]
    return butterfly(h0, alpha_c) + butterfly(h1, alpha_c ^ (1 << i))


def ibutterfly(vals: list, alpha_c: int) -> list:
    """Inverse of Alg. 2: undo the recursion from the bottom."""
    n = len(vals)
    if n == 1:
        return [vals[0]]
    i = n.bit_length() - 2
    h = n // 2
    h0 = ibutterfly(vals[:h], alpha_c)
    h1 = ibutterfly(vals[h:], alpha_c ^ (1 << i))
    c = s_eval(i, alpha_c)
    p1 = [h0[t] ^ h1[t] for t in range(h)]
    p0 = [h0[t] ^ F.mul(c, p1[t]) for t in range(h)]
    return p0 + p1


def params(n: int):
    l = n.bit_length() - 1 - LM
    assert n == 1 << (l + LM) and 0 <= l < M // 2
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
    q = gf2_inverse_rows(encode_rows())
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
    """BasisCvt, Encode, Butterfly at alpha = v_{l+m/2} (Alg. 5, the forward steps)."""
    l, n_p = params(n)
    g = F.to_novelpoly(a, n)
    f = encode(g, n)
    return butterfly(f, 1 << (l + M // 2))


def inverse(vals: list, n: int) -> int:
    """iButterfly, Decode, iBasisCvt (Alg. 5, the inverse steps)."""
    l, n_p = params(n)
    h = ibutterfly(vals, 1 << (l + M // 2))
    return F.from_novelpoly(decode(h, n))


def transform_size(len_a: int, len_b: int) -> int:
    lc = len_a + len_b - 1
    n = 64
    while n < lc:
        n *= 2
    return n


def fp_polymul(a: int, len_a: int, b: int, len_b: int) -> int:
    """Alg. 5 on Python-int bit polynomials."""
    if len_a == 0 or len_b == 0:
        return 0
    n = transform_size(len_a, len_b)
    a &= (1 << len_a) - 1
    b &= (1 << len_b) - 1
    ha = forward(a, n)
    hb = forward(b, n)
    hc = [F.mul(x, y) for x, y in zip(ha, hb)]
    return inverse(hc, n)
