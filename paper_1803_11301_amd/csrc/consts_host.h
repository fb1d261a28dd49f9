// consts_host.h -- host-side construction of the constant tables the kernels use.
//
// Field: GF(2^64) = GF(2)[x] / (x^64 + x^4 + x^3 + x + 1), the representation
// the paper multiplies in (Sec. 4.3).  Elements are uint64_t, bit k = coefficient
// of x^k.  Only constants are converted into this representation; the input
// bits are 0/1 and need no conversion (Sec. 4.3).
//
// Cantor basis (Sec. 2.2, Eq. 2): v_0 = 1 and v_i^2 + v_i = v_{i-1}.  Each
// equation has the two roots v and v + 1; we take the root whose bit 0 is clear
// in the polynomial representation (the paper leaves the choice open; the
// product does not depend on it).
//
// Tables built here:
//   iota[8][256]  element with Cantor vector c = XOR_k iota[k][(c >> 8k) & 255]
//   enc[64]       Encode rows r_j = prod over set bits k of j (k < 6) of v_{32-k}
//                 (Eq. 9 with the layer index read as in the note below)
//   dec[64]       inverse of the Encode matrix: for f = XOR_{j in a} enc[j],
//                 a = XOR_{t in f} dec[t]  (the bits back, for Decode)
//
// Note on Eq. 9: the first l_m = 6 butterfly layers of the virtual length-n
// transform pair the offsets 2^(l+k), k = 0..5, and layer l+k multiplies by
// s_{l+k}(v_{l+32}) = v_{32-k} (Eq. 4).  The printed index 32-1-k would put
// every r_j in the subfield V_32 and make the 64 x 64 matrix singular.
#pragma once

#include <cstdint>
#include <cstring>
#include <stdexcept>

namespace fpmul_host {

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

static inline uint64_t gf_mul(uint64_t a, uint64_t b)
{
    uint64_t lo, hi;
    clmul64(a, b, lo, hi);
    return reduce(lo, hi);
}

// Solve x^2 + x = c over GF(2^64) (a GF(2)-linear system); root with bit 0 clear.
static inline uint64_t solve_x2_plus_x(uint64_t c)
{
    // column t of the map = image of x^t
    uint64_t col[64];
    for (int t = 0; t < 64; ++t) {
        uint64_t e = 1ull << t;
        col[t] = gf_mul(e, e) ^ e;
    }
    // rows of the augmented system: row r = (mask over unknowns t, rhs bit)
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
    if ((gf_mul(x, x) ^ x) != c) throw std::runtime_error("root check failed");
    return x;
}

struct Tables {
    uint64_t cantor[64];
    uint64_t iota[8][256];
    uint64_t enc[64];
    uint64_t dec[64];
};

static inline uint64_t iota_of(const Tables &T, uint64_t cvec)
{
    uint64_t r = 0;
    for (int k = 0; k < 8; ++k) r ^= T.iota[k][(cvec >> (8 * k)) & 255u];
    return r;
}

static inline void build_tables(Tables &T)
{
    T.cantor[0] = 1;
    for (int i = 1; i < 64; ++i) T.cantor[i] = solve_x2_plus_x(T.cantor[i - 1]);
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
            if ((j >> k) & 1) r = gf_mul(r, T.cantor[32 - k]);
        T.enc[j] = r;
    }
    // invert: Gaussian elimination on pairs (value, combination of rows)
    uint64_t val[64], comb[64];
    for (int j = 0; j < 64; ++j) { val[j] = T.enc[j]; comb[j] = 1ull << j; }
    for (int t = 0; t < 64; ++t) {
        int p = -1;
        for (int r = t; r < 64; ++r)
            if ((val[r] >> t) & 1u) { p = r; break; }
        if (p < 0) throw std::runtime_error("Encode matrix is singular");
        std::swap(val[p], val[t]);
        std::swap(comb[p], comb[t]);
        for (int r = 0; r < 64; ++r)
            if (r != t && ((val[r] >> t) & 1u)) { val[r] ^= val[t]; comb[r] ^= comb[t]; }
    }
    for (int t = 0; t < 64; ++t) {
        if (val[t] != (1ull << t)) throw std::runtime_error("Encode inverse failed");
        T.dec[t] = comb[t];
    }
}

}  // namespace fpmul_host
