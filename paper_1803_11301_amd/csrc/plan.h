// plan.h -- host-side sizing of a product: which transform length a product
// of lc bits uses, and how many workspace words its launch needs.  Plain C++
// (no HIP), so that the sizing rules can be checked on the CPU; the library,
// the server's admission footprint and the no-allocation entry point all take
// their sizes from here.
#pragma once

#include <algorithm>
#include <cstdint>

namespace fpmul_plan {

constexpr int TAU_WORDS = 1024;          // tau = 2^16 bits: the row length of the fused BasisCvt
constexpr int M64_MAX_LOG2N = 37;        // m = 64 field bound: n <= (m/2) 2^(m/2) = 2^37
constexpr int FUSED_MIN_LOG2N = 22;      // the fused BasisCvt/Encode/Decode path: 2^22 <= n ...
constexpr int FUSED_MAX_LOG2N = 31;      // ... <= 2^31 bits
constexpr int SINGLE_VIA_BATCH_LOG2N = 17;   // polymul_ex of products up to 2^17 bits: a one-item batch

inline int ilog2(uint64_t x)   // ceil(log2 x), 0 for x <= 1
{
    int r = 0;
    while (r < 63 && (1ull << r) < x) ++r;
    if ((1ull << r) < x) ++r;
    return r;
}

inline uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// log2 of the transform length of a product of lc bits: n = max(64,
// 2^ceil(log2 lc)), except that a 2^21-bit transform is taken as 2^22 bits,
// which the fused path (from 2^22) computes faster than the per-step path;
// any n >= lc gives the same product (the transform is a bijection on
// polynomials of fewer than n bits)
inline int product_log2n(uint64_t lc)
{
    const int k = std::max(6, ilog2(lc));
    return k == 21 ? 22 : k;
}

// log2 of the transform length of a GF(2^128) product (m = 128: n >= 128)
inline int product128_log2n(uint64_t lc) { return std::max(7, ilog2(lc)); }

inline bool fast_path(int log2n) { return log2n >= FUSED_MIN_LOG2N && log2n <= FUSED_MAX_LOG2N; }

// words per skewed row of the fused BasisCvt: tau + R bits, the extension
// rounded up to 64 words
inline int bc_ew(int lgR)
{
    uint64_t R = 1ull << lgR, ext = (R + 63) / 64;
    ext = (ext + 63) / 64 * 64;
    return (int)(TAU_WORDS + ext);
}

// words one workspace buffer needs for transform length 2^log2n (m = 64)
inline uint64_t ws_words_for(int log2n)
{
    uint64_t nw = 1ull << (log2n - 6);
    if (!fast_path(log2n)) return nw;
    const int lgR = log2n - 16;
    return std::max<uint64_t>(nw, (1ull << lgR) * (uint64_t)bc_ew(lgR));
}

// true when the single-product path takes lc bits over GF(2^128)
inline bool routes_m128(uint64_t lc, int large_field_log2n)
{
    const int log2n = product_log2n(lc);
    return log2n >= large_field_log2n || log2n > M64_MAX_LOG2N;
}

// words per workspace buffer (four buffers) that the single-product path
// asks for when it multiplies operands of la and lb bits (both >= 1)
inline uint64_t product_ws_words(uint64_t la, uint64_t lb, int large_field_log2n)
{
    const uint64_t lc = la + lb - 1;
    if (routes_m128(lc, large_field_log2n)) return 1ull << (product128_log2n(lc) - 6);
    return ws_words_for(product_log2n(lc));
}

// device bytes the server reserves for one single-product launch of lc bits
// (it admits m = 64 products only)
inline uint64_t single_launch_bytes(uint64_t lc) { return 4 * ws_words_for(product_log2n(lc)) * 8; }

}  // namespace fpmul_plan
