"""The paper's multiplication, step by step in plain Python (test infrastructure only).

Computes the transform of Alg. 5 (FP_Polymul) from the definitions of its
steps, for small n, so that the readings taken where the paper is ambiguous
are checked against the plain product before any kernel relies on them:

* BasisCvt (Alg. 1): the novelpoly coefficients, here by their definition
  (repeated division by s_i, ``cantor.to_novelpoly``);
* Encode (Alg. 4, Eq. 9): f_i = sum_j a_{j n_p + i} r_j.  Reading: r_j is the
  product of v_{m/2-k} over the set bits k of j (k = 0 .. l_m-1).  Bit k of j
  is the offset 2^(l+k) that the butterfly layer i = l+k of the virtual
  length-n transform pairs, and that layer multiplies by s_{l+k}(v_{l+m/2}) =
  v_{m/2-k} by Eq. 4.  The printed index m/2-1-k gives a singular matrix;
* Butterfly (Alg. 2) at alpha = v_{l+m/2}: what it computes, the values of
  sum_k f_k X_k at the points alpha + j, here evaluated directly from the
  product form of the novel polynomial basis (``evaluate``);
* pointwise products, then the inverse steps: the interpolation that undoes
  that evaluation (Gauss-Jordan on its matrix, ``interpolate``), Decode
  (R^{-1} per element, then the bits back to rows), iBasisCvt.
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


def x_basis_at(cvec: int, l: int) -> list:
    """[X_k(x) for k < 2^l] at the point x with Cantor vector cvec.  The novel
    polynomial basis is the product of the subspace polynomials over the set
    bits of k (Sec. 2.3), each normalised by s_i(v_i), which is 1 for the
    Cantor basis; so X_{k + 2^i} = X_k s_i for k < 2^i."""
    vals = [1]
    for i in range(l):
        si = s_eval(i, cvec)
        vals = vals + [F.mul(v, si) for v in vals]
    return vals


def evaluate(g: list, alpha_c: int) -> list:
    """The values of sum_k g_k X_k at the points alpha + j, j < len(g) (alpha
    given by its Cantor vector), each computed from the definition: what the
    butterfly network of Alg. 2 produces, without its recursion."""
    l = len(g).bit_length() - 1
    out = []
    for j in range(len(g)):
        xs = x_basis_at(alpha_c ^ j, l)
        v = 0
        for gk, xk in zip(g, xs):
            if gk:
                v ^= F.mul(gk, xk)
        out.append(v)
    return out


def _inv(a: int) -> int:
    return F.power(a, (1 << M) - 2)


def interpolate(vals: list, alpha_c: int) -> list:
    """The coefficients g with evaluate(g, alpha_c) == vals: Gauss-Jordan
    elimination on the matrix [X_k(alpha + j)] over GF(2^64), which is
    invertible because the points are distinct and deg X_k = k."""
    n = len(vals)
    l = n.bit_length() - 1
    rows = [x_basis_at(alpha_c ^ j, l) + [vals[j]] for j in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if rows[r][col])
        rows[col], rows[piv] = rows[piv], rows[col]
        inv = _inv(rows[col][col])
        rows[col] = [F.mul(inv, x) for x in rows[col]]
        for r in range(n):
            if r != col and rows[r][col]:
                f = rows[r][col]
                rows[r] = [x ^ F.mul(f, y) for x, y in zip(rows[r], rows[col])]
    return [rows[k][n] for k in range(n)]


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
    return evaluate(f, 1 << (l + M // 2))


def inverse(vals: list, n: int) -> int:
    """iButterfly, Decode, iBasisCvt (Alg. 5, the inverse steps)."""
    l, n_p = params(n)
    h = interpolate(vals, 1 << (l + M // 2))
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
