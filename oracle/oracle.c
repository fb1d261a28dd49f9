/*
 * oracle.c -- CPU oracle for the product in GF(2)[x].
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this file: it is used by tests/, by the smoke check and by the
 * cpu_baseline leg of bench.py, and it shares no code with the HIP library.
 *
 * What it computes is the plain definition of the product of two bit
 * polynomials (Sec. 2.1, steps 0-3; Alg. 5 output):
 *     c_k = XOR over i + j = k of a_i * b_j,   0 <= k < len_a + len_b - 1.
 * The paper's method reaches exactly this result (Prop. 2: E_Sigma is a
 * bijection, so the interpolation is exact), so the definition is the oracle.
 *
 * Layout convention: bit k of a polynomial is bit (k % 64) of 64-bit word
 * (k / 64), little-endian words.  Bits at or above the stated length in the
 * last input word are ignored.
 *
 * Contents
 *   - 64x64 -> 128-bit carry-less word product: a software bit loop, and the
 *     x86 PCLMULQDQ instruction (Sec. 4.2 names it) used as a library
 *     primitive when the host has it; tests cross-check the two.
 *   - schoolbook word product, and Karatsuba above a threshold (a textbook
 *     recursion: (a0 + a1 y)(b0 + b1 y) with three half products).
 *   - GF(2^64) = GF(2)[x]/(x^64 + x^4 + x^3 + x + 1) multiply (Sec. 4.3 names
 *     this modulus) and Horner evaluation of a bit polynomial at a field
 *     point, for Schwartz-Zippel checks of products too large to recompute.
 *   - one output word of a product computed directly from the definition,
 *     for sampled checks at full size.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* 64x64 carry-less word product                                        */
/* ------------------------------------------------------------------ */

static inline void clmul_soft(uint64_t a, uint64_t b, uint64_t *lo, uint64_t *hi)
{
    uint64_t l = 0, h = 0;
    for (int i = 0; i < 64; i++) {
        if ((b >> i) & 1u) {
            l ^= a << i;
            if (i) h ^= a >> (64 - i);
        }
    }
    *lo = l;
    *hi = h;
}

#if defined(__x86_64__)
#include <immintrin.h>
__attribute__((target("pclmul,sse4.1")))
static inline void clmul_hw(uint64_t a, uint64_t b, uint64_t *lo, uint64_t *hi)
{
    __m128i x = _mm_set_epi64x(0, (long long)a);
    __m128i y = _mm_set_epi64x(0, (long long)b);
    __m128i z = _mm_clmulepi64_si128(x, y, 0x00);
    *lo = (uint64_t)_mm_cvtsi128_si64(z);
    *hi = (uint64_t)_mm_extract_epi64(z, 1);
}
#endif

/* 0 = software loop, 1 = PCLMULQDQ.  Chosen once from the host CPU. */
static int g_use_hw = -1;

static void pick_impl(void)
{
    if (g_use_hw >= 0) return;
#if defined(__x86_64__)
    __builtin_cpu_init();
    g_use_hw = __builtin_cpu_supports("pclmul") ? 1 : 0;
#else
    g_use_hw = 0;
#endif
}

int oracle_set_impl(int use_hw)
{
    pick_impl();
    if (use_hw < 0) return g_use_hw;
#if defined(__x86_64__)
    if (use_hw && !__builtin_cpu_supports("pclmul")) return -1;
#else
    if (use_hw) return -1;
#endif
    g_use_hw = use_hw ? 1 : 0;
    return g_use_hw;
}

static inline void clmul(uint64_t a, uint64_t b, uint64_t *lo, uint64_t *hi)
{
#if defined(__x86_64__)
    if (g_use_hw) { clmul_hw(a, b, lo, hi); return; }
#endif
    clmul_soft(a, b, lo, hi);
}

void oracle_clmul64(uint64_t a, uint64_t b, int use_hw, uint64_t out[2])
{
    pick_impl();
#if defined(__x86_64__)
    if (use_hw) { clmul_hw(a, b, &out[0], &out[1]); return; }
#endif
    (void)use_hw;
    clmul_soft(a, b, &out[0], &out[1]);
}

/* ------------------------------------------------------------------ */
/* word-array products                                                  */
/* ------------------------------------------------------------------ */

/* out[0 .. na+nb) ^= a * b  (schoolbook over words) */
static void school_acc(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out)
{
    for (size_t i = 0; i < na; i++) {
        uint64_t ai = a[i];
        if (!ai) continue;
        for (size_t j = 0; j < nb; j++) {
            uint64_t lo, hi;
            clmul(ai, b[j], &lo, &hi);
            out[i + j] ^= lo;
            out[i + j + 1] ^= hi;
        }
    }
}

#define KARA_MIN 32

/* out[0 .. 2n) = a * b, both n words.  tmp needs 4n words. */
static void kara(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *out, uint64_t *tmp, int par)
{
    if (n <= KARA_MIN) {
        memset(out, 0, 2 * n * sizeof(uint64_t));
        school_acc(a, n, b, n, out);
        return;
    }
    size_t h = n / 2, h2 = n - h;        /* low half h words, high half h2 >= h words */
    const uint64_t *a0 = a, *a1 = a + h, *b0 = b, *b1 = b + h;
    /* z0 = a0 b0 (2h words) into out[0..2h), z2 = a1 b1 (2 h2 words) into out[2h..2n) */
    uint64_t *z0 = out, *z2 = out + 2 * h;
    /* sums (h2 words each) and middle product (2 h2 words) in tmp */
    uint64_t *sa = tmp, *sb = tmp + h2, *zm = tmp + 2 * h2;
    uint64_t *rest = tmp + 4 * h2;       /* scratch for the recursion */
    for (size_t i = 0; i < h2; i++) {
        sa[i] = a1[i] ^ (i < h ? a0[i] : 0);
        sb[i] = b1[i] ^ (i < h ? b0[i] : 0);
    }
#ifdef _OPENMP
    if (par > 0) {
        uint64_t *r0 = (uint64_t *)malloc(4 * h2 * sizeof(uint64_t) * 2 + 64);
        uint64_t *r1 = (uint64_t *)malloc(4 * h2 * sizeof(uint64_t) * 2 + 64);
        uint64_t *r2 = (uint64_t *)malloc(4 * h2 * sizeof(uint64_t) * 2 + 64);
        #pragma omp task shared(a0, b0, z0) firstprivate(h, r0, par)
        kara(a0, b0, h, z0, r0, par - 1);
        #pragma omp task shared(a1, b1, z2) firstprivate(h2, r1, par)
        kara(a1, b1, h2, z2, r1, par - 1);
        #pragma omp task shared(sa, sb, zm) firstprivate(h2, r2, par)
        kara(sa, sb, h2, zm, r2, par - 1);
        #pragma omp taskwait
        free(r0); free(r1); free(r2);
    } else
#endif
    {
        (void)par;
        kara(a0, b0, h, z0, rest, 0);
        kara(a1, b1, h2, z2, rest, 0);
        kara(sa, sb, h2, zm, rest, 0);
    }
    /* middle term zm ^= z0 ^ z2, then out[h ..] ^= zm */
    for (size_t i = 0; i < 2 * h; i++) zm[i] ^= z0[i];
    for (size_t i = 0; i < 2 * h2; i++) zm[i] ^= z2[i];
    for (size_t i = 0; i < 2 * h2; i++) out[h + i] ^= zm[i];
}

/* scratch words kara() needs for size n (each level uses 4*h2 words, h2 <= n/2+1) */
static size_t kara_scratch(size_t n)
{
    size_t s = 0;
    while (n > KARA_MIN) {
        size_t h2 = n - n / 2;
        s += 4 * h2;
        n = h2;
    }
    return s + 16;
}

/* out[0 .. na+nb) = a * b for arbitrary word counts, Karatsuba on equal chunks */
static void mul_words(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out, int threads)
{
    memset(out, 0, (na + nb) * sizeof(uint64_t));
    if (!na || !nb) return;
    if (na < nb) { const uint64_t *t = a; a = b; b = t; size_t tn = na; na = nb; nb = tn; }
    /* a is the longer operand: cut it into chunks of nb words */
    if (nb <= KARA_MIN) { school_acc(a, na, b, nb, out); return; }
    size_t nch = (na + nb - 1) / nb;
    uint64_t *chunk = (uint64_t *)calloc(nb, sizeof(uint64_t));
    uint64_t *prod = (uint64_t *)malloc(2 * nb * sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)malloc(kara_scratch(nb) * sizeof(uint64_t));
    int par = 0;
#ifdef _OPENMP
    if (threads > 1) { par = 1; while ((1 << (par + 1)) < threads * 3 && par < 4) par++; }
#else
    (void)threads;
#endif
    for (size_t c = 0; c < nch; c++) {
        size_t off = c * nb, len = na - off < nb ? na - off : nb;
        memset(chunk, 0, nb * sizeof(uint64_t));
        memcpy(chunk, a + off, len * sizeof(uint64_t));
#ifdef _OPENMP
        if (par) {
            #pragma omp parallel num_threads(threads)
            #pragma omp single
            kara(chunk, b, nb, prod, tmp, par);
        } else
#endif
            kara(chunk, b, nb, prod, tmp, 0);
        size_t lim = na + nb - off < 2 * nb ? na + nb - off : 2 * nb;
        for (size_t i = 0; i < lim; i++) out[off + i] ^= prod[i];
    }
    free(chunk); free(prod); free(tmp);
}

static size_t words_of(uint64_t bits) { return (size_t)((bits + 63) / 64); }

/* copy len bits into a fresh zero-padded word array */
static uint64_t *masked_copy(const uint64_t *src, uint64_t len)
{
    size_t nw = words_of(len);
    uint64_t *d = (uint64_t *)calloc(nw ? nw : 1, sizeof(uint64_t));
    if (nw) {
        memcpy(d, src, nw * sizeof(uint64_t));
        if (len % 64) d[nw - 1] &= (~0ull) >> (64 - len % 64);
    }
    return d;
}

/*
 * Full product.  out must hold ceil((len_a + len_b - 1) / 64) words; exactly
 * len_a + len_b - 1 bits are written and the rest of the last word is zero.
 * Either length 0 gives an empty product (nothing written).
 * method: 0 = schoolbook only, 1 = Karatsuba.  threads: OpenMP threads (>=1).
 */
int oracle_polymul(const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                   uint64_t *out, int method, int threads)
{
    pick_impl();
    if (len_a == 0 || len_b == 0) return 0;
    uint64_t lc = len_a + len_b - 1;
    size_t na = words_of(len_a), nb = words_of(len_b), nc = words_of(lc);
    uint64_t *ma = masked_copy(a, len_a), *mb = masked_copy(b, len_b);
    uint64_t *full = (uint64_t *)calloc(na + nb, sizeof(uint64_t));
    if (method == 0) school_acc(ma, na, mb, nb, full);
    else mul_words(ma, na, mb, nb, full, threads < 1 ? 1 : threads);
    memcpy(out, full, nc * sizeof(uint64_t));
    if (lc % 64) out[nc - 1] &= (~0ull) >> (64 - lc % 64);
    free(ma); free(mb); free(full);
    return 0;
}

/*
 * Word w of the product, from the definition: the words of A and B are
 * polynomials A_i(x) x^{64 i}, B_j(x) x^{64 j}; word w of C collects the low
 * halves of A_i B_j with i + j = w and the high halves with i + j = w - 1.
 * Words at or beyond the product length read as the masked product.
 */
void oracle_product_words(const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                          const uint64_t *idx, uint64_t count, uint64_t *out)
{
    pick_impl();
    if (len_a == 0 || len_b == 0) { memset(out, 0, count * sizeof(uint64_t)); return; }
    size_t na = words_of(len_a), nb = words_of(len_b);
    uint64_t lc = len_a + len_b - 1;
    size_t nc = words_of(lc);
    uint64_t amask = len_a % 64 ? (~0ull) >> (64 - len_a % 64) : ~0ull;
    uint64_t bmask = len_b % 64 ? (~0ull) >> (64 - len_b % 64) : ~0ull;
    for (uint64_t q = 0; q < count; q++) {
        uint64_t w = idx[q], acc = 0;
        if (w >= nc) { out[q] = 0; continue; }
        for (size_t i = 0; i < na && i <= w; i++) {
            uint64_t ai = a[i] & (i == na - 1 ? amask : ~0ull);
            uint64_t lo, hi;
            size_t j = (size_t)(w - i);
            if (j < nb) {
                clmul(ai, b[j] & (j == nb - 1 ? bmask : ~0ull), &lo, &hi);
                acc ^= lo;
            }
            if (w >= i + 1 && (j = (size_t)(w - 1 - i)) < nb) {
                clmul(ai, b[j] & (j == nb - 1 ? bmask : ~0ull), &lo, &hi);
                acc ^= hi;
            }
        }
        if (w == nc - 1 && lc % 64) acc &= (~0ull) >> (64 - lc % 64);
        out[q] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* GF(2^64) = GF(2)[x] / (x^64 + x^4 + x^3 + x + 1)                     */
/* ------------------------------------------------------------------ */

/* reduce a 128-bit carry-less product hi:lo modulo x^64 + x^4 + x^3 + x + 1
   by plain long division, bit by bit from the top */
static uint64_t gf_reduce(uint64_t lo, uint64_t hi)
{
    for (int k = 63; k >= 0; k--) {
        if ((hi >> k) & 1u) {
            /* x^(64+k) = x^k (x^4 + x^3 + x + 1) */
            hi ^= 1ull << k;
            uint64_t t = 0x1Bull;               /* x^4 + x^3 + x + 1 */
            /* add t * x^k: bits k..k+4 */
            lo ^= t << k;
            if (k > 59) hi ^= t >> (64 - k);
        }
    }
    return lo;
}

uint64_t oracle_gf64_mul(uint64_t x, uint64_t y)
{
    uint64_t lo, hi;
    pick_impl();
    clmul(x, y, &lo, &hi);
    return gf_reduce(lo, hi);
}

/*
 * Evaluate the bit polynomial A (len bits) at the field point z:
 * A(z) = sum_k a_k z^k.  Horner over 64-bit words: word w contributes
 * W_w(z) = sum_{t<64} bit_t z^t, and A(z) = sum_w W_w(z) (z^64)^w.
 */
uint64_t oracle_eval(const uint64_t *a, uint64_t len, uint64_t z)
{
    pick_impl();
    if (len == 0) return 0;
    uint64_t pw[64];
    pw[0] = 1;
    for (int t = 1; t < 64; t++) pw[t] = oracle_gf64_mul(pw[t - 1], z);
    uint64_t z64 = oracle_gf64_mul(pw[63], z);
    size_t nw = words_of(len);
    uint64_t acc = 0;
    for (size_t w = nw; w-- > 0;) {
        uint64_t word = a[w];
        if (w == nw - 1 && len % 64) word &= (~0ull) >> (64 - len % 64);
        uint64_t ww = 0;
        while (word) {
            int t = __builtin_ctzll(word);
            ww ^= pw[t];
            word &= word - 1;
        }
        acc = oracle_gf64_mul(acc, z64) ^ ww;
    }
    return acc;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
