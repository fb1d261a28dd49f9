// consts_host.h -- host-side construction of the constant tables the kernels use.
//
// Reference field: GF(2^64) = GF(2)[x] / (x^64 + x^4 + x^3 + x + 1), the
// polynomial representation of Sec. 4.3 ("poly" below).  It is used here only
// to derive constants.
//
// Cantor basis (Sec. 2.2, Eq. 2): v_0 = 1 and v_i^2 + v_i = v_{i-1}.  Each
// equation has the two roots v and v + 1; we take the root whose bit 0 is clear
// in the poly representation (the paper leaves the choice open; the product
// does not depend on it).
//
// Device representation ("tower").  V_8, V_16, V_32 are the subfields GF(2^8),
// GF(2^16), GF(2^32) (Sec. 2.2.1), and v_8, v_16, v_32 generate each one over
// the previous: v_{2^k}^2 + v_{2^k} = v_{2^k - 1}.  An element is stored as
// 8 bytes B_0..B_7, x = sum_k B_k W_k with W_k = v_8^{k&1} v_16^{(k>>1)&1}
// v_32^{k>>2}, and each byte B_k is an element of GF(2^8) = V_8 in Cantor
// coordinates (bit u <-> v_u).  So
//   x = x1 v_32 + x0          (x0 = low 32 bits, x1 = high 32 bits, in GF(2^32))
//   a = a1 v_16 + a0          (GF(2^32) element, 16-bit halves in GF(2^16))
//   e = e1 v_8 + e0           (GF(2^16) element, bytes in GF(2^8))
// with the reductions v_8^2 = v_8 + v_7, v_16^2 = v_16 + v_15,
// v_32^2 = v_32 + v_31.  Multiplying by an element of V_8 acts on each byte
// alone, which is what the butterflies exploit; the paper multiplies in the
// poly representation instead because of PCLMULQDQ (Sec. 4.3), which this
// hardware does not have.
//
// Tables built here (all in the tower representation):
//   iota[8][256]  element with Cantor vector c = XOR_k iota[k][(c >> 8k) & 255]
//   enc[64]       Encode rows r_j = prod over set bits k of j (k < 6) of v_{32-k}
//                 (Eq. 9 with the layer index read as in the note below)
//   dec[64]       inverse of the Encode matrix: for f = XOR_{j in a} enc[j],
//                 a = XOR_{t in f} dec[t]  (the bits back, for Decode)
//   mul8[256][256] products in GF(2^8) = V_8, Cantor coordinates
//   v15, v31      v_15 in GF(2^16) and v_31 in GF(2^32), tower coordinates
//   gamma tables  for each d, the 8-bit window tables of multiplication by
//                 v_{32+d}: T[k][e] = v_{32+d} * (e at byte k)
//
// Note on Eq. 9: the first l_m = 6 butterfly layers of the virtual length-n
// transform pair the offsets 2^(l+k), k = 0..5, and layer l+k multiplies by
// s_{l+k}(v_{l+32}) = v_{32-k} (Eq. 4).  The printed index 32-1-k would put
// every r_j in the subfield V_32 and make the 64 x 64 matrix singular.
#pragma once

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <utility>
#include <vector>

namespace fpmul_host {

// ------------------------------------------------------------- poly field --

static inline void clmul64(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi)
{
    lo = 0;
    hi = 0;
    for (int i = 0; i < 64; ++i)
        if ((b >> i) & 1u) {
            lo ^= a << i;
            if (i) hi ^= a >> (64 - i);
        }
}

// x^64 = x^4 + x^3 + x + 1: fold the high word twice
static inline uint64_t reduce(uint64_t lo, uint64_t hi)
{
    uint64_t t = hi ^ (hi << 1) ^ (hi << 3) ^ (hi << 4);
    uint64_t o = (hi >> 63) ^ (hi >> 61) ^ (hi >> 60);
    return lo ^ t ^ o ^ (o << 1) ^ (o << 3) ^ (o << 4);
}

static inline uint64_t pmul(uint64_t a, uint64_t b)
{
    uint64_t lo, hi;
    clmul64(a, b, lo, hi);
    return reduce(lo, hi);
}

// Solve x^2 + x = c in the poly field (a GF(2)-linear system); root with bit 0 clear.
static inline uint64_t solve_x2_plus_x(uint64_t c)
{
    uint64_t col[64];
    for (int t = 0; t < 64; ++t) {
        uint64_t e = 1ull << t;
        col[t] = pmul(e, e) ^ e;
    }
    uint64_t rowm[64];
    int rhs[64];
    for (int r = 0; r < 64; ++r) {
        uint64_t m = 0;
        for (int t = 0; t < 64; ++t)
            if ((col[t] >> r) & 1u) m |= 1ull << t;
        rowm[r] = m;
        rhs[r] = (int)((c >> r) & 1u);
    }
    int pivrow[64];
    for (int t = 0; t < 64; ++t) pivrow[t] = -1;
    int rank = 0;
    for (int t = 0; t < 64 && rank < 64; ++t) {
        int p = -1;
        for (int r = rank; r < 64; ++r)
            if ((rowm[r] >> t) & 1u) { p = r; break; }
        if (p < 0) continue;
        std::swap(rowm[p], rowm[rank]);
        std::swap(rhs[p], rhs[rank]);
        for (int r = 0; r < 64; ++r)
            if (r != rank && ((rowm[r] >> t) & 1u)) {
                rowm[r] ^= rowm[rank];
                rhs[r] ^= rhs[rank];
            }
        pivrow[t] = rank++;
    }
    for (int r = rank; r < 64; ++r)
        if (rhs[r]) throw std::runtime_error("x^2 + x = c has no root");
    uint64_t x = 0;
    for (int t = 0; t < 64; ++t)
        if (pivrow[t] >= 0 && rhs[pivrow[t]]) x |= 1ull << t;
    if (x & 1u) x ^= 1u;
    if ((pmul(x, x) ^ x) != c) throw std::runtime_error("root check failed");
    return x;
}

// Invert a GF(2) 64x64 map given by the images of the unit vectors:
// img[j] = M e_j.  Returns inv with inv[t] = M^{-1} e_t.
static inline void invert64(const uint64_t img[64], uint64_t inv[64])
{
    uint64_t val[64], comb[64];
    for (int j = 0; j < 64; ++j) { val[j] = img[j]; comb[j] = 1ull << j; }
    for (int t = 0; t < 64; ++t) {
        int p = -1;
        for (int r = t; r < 64; ++r)
            if ((val[r] >> t) & 1u) { p = r; break; }
        if (p < 0) throw std::runtime_error("singular 64x64 matrix");
        std::swap(val[p], val[t]);
        std::swap(comb[p], comb[t]);
        for (int r = 0; r < 64; ++r)
            if (r != t && ((val[r] >> t) & 1u)) { val[r] ^= val[t]; comb[r] ^= comb[t]; }
    }
    for (int t = 0; t < 64; ++t) {
        if (val[t] != (1ull << t)) throw std::runtime_error("inversion failed");
        inv[t] = comb[t];
    }
}

static inline uint64_t apply64(const uint64_t cols[64], uint64_t x)
{
    uint64_t r = 0;
    for (int t = 0; t < 64; ++t)
        if ((x >> t) & 1u) r ^= cols[t];
    return r;
}

// ------------------------------------------------------------ tower field --

struct Tower {
    uint8_t mul8[256][256];
    uint16_t v15;      // v_15 in GF(2^16), tower coordinates
    uint32_t v31;      // v_31 in GF(2^32), tower coordinates

    uint8_t m8(uint8_t a, uint8_t b) const { return mul8[a][b]; }

    uint16_t m16(uint16_t a, uint16_t b) const
    {
        uint8_t a0 = a & 255, a1 = a >> 8, b0 = b & 255, b1 = b >> 8;
        uint8_t p0 = m8(a0, b0), p2 = m8(a1, b1), p1 = m8(a0 ^ a1, b0 ^ b1);
        uint8_t hi = p1 ^ p0, lo = p0 ^ m8(p2, 0x80);   // v_7 = Cantor byte 0x80
        return (uint16_t)(lo | (hi << 8));
    }

    uint32_t m32(uint32_t a, uint32_t b) const
    {
        uint16_t a0 = a & 0xFFFF, a1 = a >> 16, b0 = b & 0xFFFF, b1 = b >> 16;
        uint16_t p0 = m16(a0, b0), p2 = m16(a1, b1), p1 = m16(a0 ^ a1, b0 ^ b1);
        uint16_t hi = p1 ^ p0, lo = p0 ^ m16(p2, v15);
        return (uint32_t)lo | ((uint32_t)hi << 16);
    }

    uint64_t m64(uint64_t a, uint64_t b) const
    {
        uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
        uint32_t p0 = m32(a0, b0), p2 = m32(a1, b1), p1 = m32(a0 ^ a1, b0 ^ b1);
        uint32_t hi = p1 ^ p0, lo = p0 ^ m32(p2, v31);
        return (uint64_t)lo | ((uint64_t)hi << 32);
    }
};

struct Tables {
    uint64_t cantor_poly[64];   // v_i in the poly representation
    uint64_t tower_to_poly[64]; // image of tower unit vector 8k+u in poly
    uint64_t poly_to_tower[64]; // image of poly unit vector t in tower
    uint64_t cantor[64];        // v_i in the tower representation
    uint64_t iota[8][256];
    uint64_t enc[64];
    uint64_t dec[64];
    uint32_t enc32[32];         // m = 32: Encode rows r_j = prod over set bits k of j (k < 5) of v_{16-k}
    uint32_t dec32[32];         // m = 32: inverse of the Encode matrix
    Tower tw;
};

static inline uint64_t to_tower(const Tables &T, uint64_t p) { return apply64(T.poly_to_tower, p); }
static inline uint64_t to_poly(const Tables &T, uint64_t x) { return apply64(T.tower_to_poly, x); }

static inline uint64_t iota_of(const Tables &T, uint64_t cvec)
{
    uint64_t r = 0;
    for (int k = 0; k < 8; ++k) r ^= T.iota[k][(cvec >> (8 * k)) & 255u];
    return r;
}

// T must be heap-allocated (it holds the 64 KiB GF(2^8) table)
static inline void build_tables(Tables &T)
{
    uint64_t *v = T.cantor_poly;
    v[0] = 1;
    for (int i = 1; i < 64; ++i) v[i] = solve_x2_plus_x(v[i - 1]);
    // tower basis in poly coordinates: unit vector 8k+u <-> v_u * W_k
    for (int k = 0; k < 8; ++k) {
        uint64_t W = 1;
        if (k & 1) W = pmul(W, v[8]);
        if (k & 2) W = pmul(W, v[16]);
        if (k & 4) W = pmul(W, v[32]);
        for (int u = 0; u < 8; ++u) T.tower_to_poly[8 * k + u] = pmul(v[u], W);
    }
    invert64(T.tower_to_poly, T.poly_to_tower);
    for (int i = 0; i < 64; ++i) T.cantor[i] = to_tower(T, v[i]);
    // GF(2^8) products in Cantor coordinates
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) {
            uint64_t pa = 0, pb = 0;
            for (int u = 0; u < 8; ++u) {
                if ((a >> u) & 1) pa ^= v[u];
                if ((b >> u) & 1) pb ^= v[u];
            }
            uint64_t t = to_tower(T, pmul(pa, pb));
            if (t >> 8) throw std::runtime_error("V_8 is not closed");
            T.tw.mul8[a][b] = (uint8_t)t;
        }
    uint64_t v15 = T.cantor[15], v31 = T.cantor[31];
    if (v15 >> 16 || v31 >> 32) throw std::runtime_error("subfield check failed");
    T.tw.v15 = (uint16_t)v15;
    T.tw.v31 = (uint32_t)v31;
    // self-check: tower products agree with poly products
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int it = 0; it < 64; ++it) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        uint64_t a = s;
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        uint64_t b = s;
        if (T.tw.m64(a, b) != to_tower(T, pmul(to_poly(T, a), to_poly(T, b))))
            throw std::runtime_error("tower multiplication self-check failed");
    }
    for (int k = 0; k < 8; ++k)
        for (int e = 0; e < 256; ++e) {
            uint64_t r = 0;
            for (int t = 0; t < 8; ++t)
                if ((e >> t) & 1) r ^= T.cantor[8 * k + t];
            T.iota[k][e] = r;
        }
    for (int j = 0; j < 64; ++j) {
        uint64_t r = 1;
        for (int k = 0; k < 6; ++k)
            if ((j >> k) & 1) r = T.tw.m64(r, T.cantor[32 - k]);
        T.enc[j] = r;
    }
    invert64(T.enc, T.dec);
    // the same for m = 32 (Sec. 3, Eq. 9 with l_m = 5): the elements lie in
    // GF(2^32), the low half of the tower representation
    uint64_t e64[64], d64[64];
    for (int j = 0; j < 32; ++j) {
        uint32_t r = 1;
        for (int k = 0; k < 5; ++k)
            if ((j >> k) & 1) {
                if (T.cantor[16 - k] >> 32) throw std::runtime_error("v_{16-k} outside GF(2^32)");
                r = T.tw.m32(r, (uint32_t)T.cantor[16 - k]);
            }
        T.enc32[j] = r;
    }
    // invert the 32 x 32 matrix inside a 64 x 64 one (identity on the top half)
    for (int j = 0; j < 64; ++j) e64[j] = j < 32 ? (uint64_t)T.enc32[j] : 1ull << j;
    invert64(e64, d64);
    for (int j = 0; j < 32; ++j) {
        if (d64[j] >> 32) throw std::runtime_error("m = 32 Encode inverse leaves GF(2^32)");
        T.dec32[j] = (uint32_t)d64[j];
    }
}

// 8-bit window tables of multiplication by c: tab[k*256 + e] = c * (e at byte k)
static inline void window_table(const Tables &T, uint64_t c, uint64_t *tab)
{
    for (int k = 0; k < 8; ++k)
        for (int e = 0; e < 256; ++e) tab[k * 256 + e] = T.tw.m64(c, (uint64_t)e << (8 * k));
}

// ------------------------------------------------------- m = 128 field --
//
// GF(2^128) = GF(2^64)[y] / (y^2 + y + v_63).  v_63 lies outside the image
// of x -> x^2 + x on GF(2^64) (its equation has no root there: checked
// below), so the quadratic is irreducible, and y is a root of the next
// Cantor equation, v_64 = y (of the two roots y and y + 1 it is the one
// whose low half has bit 0 clear, the same rule as below 64).  An element
// is (x0, x1) = x0 + x1 y with both halves in the tower representation:
//   (a0 + a1 y)(b0 + b1 y) = (a0 b0 + a1 b1 v_63) + ((a0 + a1)(b0 + b1) + a0 b0) y.
// The Cantor basis continues with v_i^2 + v_i = v_{i-1} for 64 < i < 128,
// solved in GF(2^128).

struct E128 {
    uint64_t lo, hi;
};

static inline E128 mul128(const Tables &T, E128 a, E128 b)
{
    const uint64_t p0 = T.tw.m64(a.lo, b.lo), p2 = T.tw.m64(a.hi, b.hi);
    const uint64_t p1 = T.tw.m64(a.lo ^ a.hi, b.lo ^ b.hi);
    return {p0 ^ T.tw.m64(p2, T.cantor[63]), p1 ^ p0};
}

// root of x^2 + x = c in GF(2^128) with bit 0 of the low half clear
// (Gaussian elimination on the GF(2)-linear map x -> x^2 + x, kernel {0, 1})
static inline E128 solve_x2_plus_x_128(const Tables &T, E128 c)
{
    typedef unsigned __int128 u128;
    auto pack = [](E128 e) { return (u128)e.lo | ((u128)e.hi << 64); };
    u128 col[128];
    for (int t = 0; t < 128; ++t) {
        E128 e{t < 64 ? 1ull << t : 0, t < 64 ? 0 : 1ull << (t - 64)};
        E128 q = mul128(T, e, e);
        col[t] = pack(q) ^ pack(e);
    }
    u128 rowm[128];
    int rhs[128];
    const u128 cv = pack(c);
    for (int r = 0; r < 128; ++r) {
        u128 m = 0;
        for (int t = 0; t < 128; ++t)
            if ((col[t] >> r) & 1u) m |= (u128)1 << t;
        rowm[r] = m;
        rhs[r] = (int)((cv >> r) & 1u);
    }
    int pivrow[128];
    for (int t = 0; t < 128; ++t) pivrow[t] = -1;
    int rank = 0;
    for (int t = 0; t < 128 && rank < 128; ++t) {
        int p = -1;
        for (int r = rank; r < 128; ++r)
            if ((rowm[r] >> t) & 1u) { p = r; break; }
        if (p < 0) continue;
        std::swap(rowm[p], rowm[rank]);
        std::swap(rhs[p], rhs[rank]);
        for (int r = 0; r < 128; ++r)
            if (r != rank && ((rowm[r] >> t) & 1u)) {
                rowm[r] ^= rowm[rank];
                rhs[r] ^= rhs[rank];
            }
        pivrow[t] = rank++;
    }
    for (int r = rank; r < 128; ++r)
        if (rhs[r]) throw std::runtime_error("x^2 + x = c has no root in GF(2^128)");
    u128 x = 0;
    for (int t = 0; t < 128; ++t)
        if (pivrow[t] >= 0 && rhs[pivrow[t]]) x |= (u128)1 << t;
    if (x & 1u) x ^= 1u;
    E128 r{(uint64_t)x, (uint64_t)(x >> 64)};
    E128 chk = mul128(T, r, r);
    if ((chk.lo ^ r.lo) != c.lo || (chk.hi ^ r.hi) != c.hi) throw std::runtime_error("GF(2^128) root check failed");
    return r;
}

#define M128_MAXD 64

struct Tables128 {
    E128 v[128];                 // Cantor basis of GF(2^128), v_i for i < 64 in the low half
    uint64_t enc[64];            // P_t = prod over set bits k of t (k < 6) of v_{63-k}
    uint64_t dec[64];            // inverse of the P matrix
    uint64_t ktab[M128_MAXD][2][2048];   // window tables of H_d and H_d v_63 (v_{64+d} = L_d + H_d y)
};

// T128 must be heap-allocated (2 MiB of window tables)
static inline void build_tables128(const Tables &T, Tables128 &U)
{
    // x^2 + x = v_63 has no root in GF(2^64): the GF(2)-linear map x -> x^2 + x
    // has rank 63 there and v_63 lies outside its image
    bool has_root = true;
    try {
        (void)solve_x2_plus_x(T.cantor_poly[63]);
    } catch (const std::exception &) {
        has_root = false;
    }
    if (has_root) throw std::runtime_error("y^2 + y + v_63 is reducible over GF(2^64)");
    for (int i = 0; i < 64; ++i) U.v[i] = {T.cantor[i], 0};
    for (int i = 64; i < 128; ++i) U.v[i] = solve_x2_plus_x_128(T, U.v[i - 1]);
    if (U.v[64].lo != 0 || U.v[64].hi != 1) throw std::runtime_error("v_64 is not the tower generator");
    for (int t = 0; t < 64; ++t) {
        uint64_t r = 1;
        for (int k = 0; k < 6; ++k)
            if ((t >> k) & 1) r = T.tw.m64(r, T.cantor[63 - k]);
        U.enc[t] = r;
    }
    invert64(U.enc, U.dec);
    for (int d = 0; d < M128_MAXD; ++d) {
        const uint64_t h = U.v[64 + d].hi;
        window_table(T, h, U.ktab[d][0]);
        window_table(T, T.tw.m64(h, T.cantor[63]), U.ktab[d][1]);
    }
}

}  // namespace fpmul_host
