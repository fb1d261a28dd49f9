// CPU checks of the host construction of the constant tables (consts_host.h),
// for the GF(2^64) tower and the GF(2^128) = GF(2^64)[y] / (y^2 + y + v_63)
// extension of the m = 128 variant.  Host code only; each check prints
// "ok <name>" and the program exits non-zero on the first failure.
#include <cstdio>
#include <cstdlib>
#include <memory>

#include "../../paper_1803_11301_amd/csrc/consts_host.h"

using namespace fpmul_host;

static int g_fail = 0;
#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond);  \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

static uint64_t g_s = 0x9E3779B97F4A7C15ull;
static uint64_t rnd()
{
    g_s ^= g_s << 13;
    g_s ^= g_s >> 7;
    g_s ^= g_s << 17;
    return g_s;
}

static bool eq(E128 a, E128 b) { return a.lo == b.lo && a.hi == b.hi; }
static E128 add(E128 a, E128 b) { return {a.lo ^ b.lo, a.hi ^ b.hi}; }

int main()
{
    std::unique_ptr<Tables> T(new Tables());
    std::unique_ptr<Tables128> U(new Tables128());
    build_tables(*T);
    build_tables128(*T, *U);

    // Cantor recursion v_i^2 + v_i = v_{i-1} through GF(2^128), v_0 = 1
    CHECK(U->v[0].lo == 1 && U->v[0].hi == 0);
    for (int i = 1; i < 128; ++i) CHECK(eq(add(mul128(*T, U->v[i], U->v[i]), U->v[i]), U->v[i - 1]));
    std::printf("ok basis_recursion\n");

    // the 128 basis vectors are independent over GF(2)
    {
        typedef unsigned __int128 u128;
        u128 rows[128];
        for (int i = 0; i < 128; ++i) rows[i] = (u128)U->v[i].lo | ((u128)U->v[i].hi << 64);
        int rank = 0;
        for (int b = 0; b < 128; ++b) {
            int p = -1;
            for (int r = rank; r < 128; ++r)
                if ((rows[r] >> b) & 1) { p = r; break; }
            if (p < 0) continue;
            std::swap(rows[p], rows[rank]);
            for (int r = 0; r < 128; ++r)
                if (r != rank && ((rows[r] >> b) & 1)) rows[r] ^= rows[rank];
            ++rank;
        }
        CHECK(rank == 128);
    }
    std::printf("ok basis_rank\n");

    // field axioms on random elements, and the order of the field: a^(2^128) = a,
    // while the generator y is moved to its conjugate y + 1 by x -> x^(2^64)
    for (int it = 0; it < 200; ++it) {
        E128 a{rnd(), rnd()}, b{rnd(), rnd()}, c{rnd(), rnd()};
        CHECK(eq(mul128(*T, mul128(*T, a, b), c), mul128(*T, a, mul128(*T, b, c))));
        CHECK(eq(mul128(*T, a, b), mul128(*T, b, a)));
        CHECK(eq(mul128(*T, a, add(b, c)), add(mul128(*T, a, b), mul128(*T, a, c))));
        CHECK(eq(mul128(*T, a, E128{1, 0}), a));
    }
    for (int it = 0; it < 8; ++it) {
        E128 a{rnd(), rnd()}, p = a;
        for (int k = 0; k < 128; ++k) p = mul128(*T, p, p);
        CHECK(eq(p, a));
    }
    {
        E128 y{0, 1}, p = y;
        for (int k = 0; k < 64; ++k) p = mul128(*T, p, p);
        CHECK(eq(p, E128{1, 1}));
    }
    std::printf("ok field_axioms\n");

    // Encode rows P_t and their inverse
    for (int t = 0; t < 64; ++t) {
        uint64_t r = 1;
        for (int k = 0; k < 6; ++k)
            if ((t >> k) & 1) r = T->tw.m64(r, T->cantor[63 - k]);
        CHECK(U->enc[t] == r);
    }
    for (int it = 0; it < 200; ++it) {
        uint64_t a = rnd();
        CHECK(apply64(U->dec, apply64(U->enc, a)) == a);
    }
    std::printf("ok encode_matrix\n");

    // the butterfly multiplier c = v_{64+d} + iota(2b) applied as the kernels
    // split it: (x0 + x1 y)(A + H y) = (x0 A + x1 H v_63) + ((x0 + x1) H + x1 A) y
    // with A = L_d + iota(2b), through the window tables of H and H v_63
    for (int it = 0; it < 400; ++it) {
        const int d = 1 + (int)(rnd() % 40);
        const uint64_t b = rnd() & ((1ull << (d - 1)) - 1);
        const E128 c = add(U->v[64 + d], E128{iota_of(*T, 2 * b), 0});
        const E128 x{rnd(), rnd()};
        const E128 want = mul128(*T, x, c);
        const uint64_t A = U->v[64 + d].lo ^ iota_of(*T, 2 * b);
        auto tab = [&](int which, uint64_t v) {
            uint64_t r = 0;
            for (int k = 0; k < 8; ++k) r ^= U->ktab[d][which][k * 256 + ((v >> (8 * k)) & 255u)];
            return r;
        };
        const uint64_t lo = T->tw.m64(x.lo, A) ^ tab(1, x.hi);
        const uint64_t hi = tab(0, x.lo ^ x.hi) ^ T->tw.m64(x.hi, A);
        CHECK(lo == want.lo && hi == want.hi);
    }
    std::printf("ok butterfly_split\n");

    // v_64 = y, so the d = 0 tables are those of 1 and of v_63
    for (int k = 0; k < 8; ++k)
        for (int e = 0; e < 256; e += 17) {
            CHECK(U->ktab[0][0][k * 256 + e] == ((uint64_t)e << (8 * k)));
            CHECK(U->ktab[0][1][k * 256 + e] == T->tw.m64(T->cantor[63], (uint64_t)e << (8 * k)));
        }
    std::printf("ok v63_table\n");
    return g_fail;
}
