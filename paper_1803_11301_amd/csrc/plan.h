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
constexpr int SINGLE_VIA_BATCH_LOG2N = 16;   // polymul_ex of products up to 2^16 bits: a one-item batch
constexpr int NOALLOC_MAX_LOG2N = 25;        // polymul_ex_noalloc: products up to 2^25 bits

constexpr int ilog2(uint64_t x)   // ceil(log2 x), 0 for x <= 1
{
    int r = 0;
    while (r < 63 && (1ull << r) < x) ++r;
    if ((1ull << r) < x) ++r;
    return r;
}

constexpr uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// log2 of the transform length of a product of lc bits: n = max(64,
// 2^ceil(log2 lc)), except that transforms of 2^17 .. 2^21 bits are taken as
// 2^22 bits, which the fused path (from 2^22) computes faster (its chain of
// launches spreads over the chip, about 0.13 ms for any of these products,
// where a one-workgroup batch item took 0.145 ms at 2^17 bits and a
// one-workgroup BasisCvt per operand 0.20 ms at 2^19 and 0.29 ms at 2^20);
// any n >= lc gives the same product (the transform is a bijection on
// polynomials of fewer than n bits)
constexpr int product_log2n(uint64_t lc)
{
    const int k = std::max(6, ilog2(lc));
    return (k >= 17 && k <= 21) ? 22 : k;
}

// log2 of the transform length of a GF(2^128) product (m = 128: n >= 128)
constexpr int product128_log2n(uint64_t lc) { return std::max(7, ilog2(lc)); }

constexpr bool fast_path(int log2n) { return log2n >= FUSED_MIN_LOG2N && log2n <= FUSED_MAX_LOG2N; }

// words per skewed row of the fused BasisCvt: tau + R bits, the extension
// rounded up to 64 words
constexpr int bc_ew(int lgR)
{
    uint64_t R = 1ull << lgR, ext = (R + 63) / 64;
    ext = (ext + 63) / 64 * 64;
    return (int)(TAU_WORDS + ext);
}

// words one workspace buffer needs for transform length 2^log2n (m = 64)
constexpr uint64_t ws_words_for(int log2n)
{
    uint64_t nw = 1ull << (log2n - 6);
    if (!fast_path(log2n)) return nw;
    const int lgR = log2n - 16;
    return std::max<uint64_t>(nw, (1ull << lgR) * (uint64_t)bc_ew(lgR));
}

// true when the single-product path takes lc bits over GF(2^128)
constexpr bool routes_m128(uint64_t lc, int large_field_log2n)
{
    const int log2n = product_log2n(lc);
    return log2n >= large_field_log2n || log2n > M64_MAX_LOG2N;
}

// words per workspace buffer (four buffers) that the single-product path
// asks for when it multiplies operands of la and lb bits (both >= 1)
constexpr uint64_t product_ws_words(uint64_t la, uint64_t lb, int large_field_log2n)
{
    const uint64_t lc = la + lb - 1;
    if (routes_m128(lc, large_field_log2n)) return 1ull << (product128_log2n(lc) - 6);
    return ws_words_for(product_log2n(lc));
}

// device bytes the server reserves for one single-product launch of lc bits
// (it admits m = 64 products only)
constexpr uint64_t single_launch_bytes(uint64_t lc) { return 4 * ws_words_for(product_log2n(lc)) * 8; }

}  // namespace fpmul_plan

namespace fpmul_plan {

// the device scratch of polymul_ex_noalloc: four workspace buffers for the
// largest product it takes, then the batch workspace of a one-item batch
// (grid 1, one slab of four 2^SINGLE_VIA_BATCH_LOG2N-bit buffers, the queue
// order and the counter, as the library's batch layout sizes them)
constexpr uint64_t NOALLOC_WS_WORDS = ws_words_for(NOALLOC_MAX_LOG2N);
constexpr uint64_t NOALLOC_BWS_BYTES = 4 * (1ull << (SINGLE_VIA_BATCH_LOG2N - 6)) * 8 + 256 + 256;
constexpr uint64_t NOALLOC_SCRATCH_WORDS = 4 * NOALLOC_WS_WORDS + NOALLOC_BWS_BYTES / 8;

}  // namespace fpmul_plan

// ---------------------------------------------------------------------------
// schedule choices of the fused path that the tuner searches
// ---------------------------------------------------------------------------
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace fpmul_plan {

constexpr int BOTTOM_LAYERS = 7;       // layers 0..6 in the bottom butterfly pass (the default)
constexpr int BOTTOM_LAYERS_MIN = 6;   // or layers 0..5, the upper passes taking layer 6
constexpr int UPPER_MAXK = 7;          // layers per upper pass at most
constexpr int TILE_LG = 12;            // 2^12 values per butterfly tile

// the lowest upper pass starts at the bottom pass's layer count b and needs
// K >= 12 - b layers (its tile's column bits lie below layer b)
constexpr int upper_low_mink(int bottom) { return TILE_LG - bottom; }

struct Schedule {
    std::vector<int> upper;   // layers per upper pass, lowest pass first; empty = the default split
    int rows_mult = 4;        // forward row-kernel workgroups per CU (the inverse takes four times as many)
    int zeta_mult = 16;       // zeta-kernel workgroups per CU (likewise)
};

// the default split of the U = l - 7 upper layers: as even as possible over
// ceil(U / 7) passes, the larger parts at the bottom
inline std::vector<int> default_upper(int l)
{
    std::vector<int> g;
    const int U = l - BOTTOM_LAYERS;
    if (U <= 0) return g;
    const int ng = (U + UPPER_MAXK - 1) / UPPER_MAXK, base = U / ng, extra = U % ng;
    for (int k = 0; k < ng; ++k) g.push_back(base + (k < extra ? 1 : 0));
    return g;
}

// the bottom pass's layer count under a split: the layers below the upper passes
inline int bottom_layers(int l, const std::vector<int> &g)
{
    int s = 0;
    for (int k : g) s += k;
    return g.empty() ? BOTTOM_LAYERS : l - s;
}

// a split is valid when its parts are 1..7 layers, they leave 6 or 7 layers
// to the bottom pass, and the lowest pass (from layer b) has at least 12 - b
inline bool upper_valid(int l, const std::vector<int> &g)
{
    if (l - BOTTOM_LAYERS <= 0) return g.empty();
    if (g.empty()) return false;
    for (int k : g)
        if (k < 1 || k > UPPER_MAXK) return false;
    const int b = bottom_layers(l, g);
    return b >= BOTTOM_LAYERS_MIN && b <= BOTTOM_LAYERS && g[0] >= upper_low_mink(b);
}

// every valid split into the fewest passes or one more, for either bottom pass
inline std::vector<std::vector<int>> upper_candidates(int l)
{
    std::vector<std::vector<int>> out;
    if (l - BOTTOM_LAYERS <= 0) return out;
    for (int b = BOTTOM_LAYERS; b >= BOTTOM_LAYERS_MIN; --b) {
        const int U = l - b;
        const int m0 = (U + UPPER_MAXK - 1) / UPPER_MAXK;
        for (int m = m0; m <= m0 + 1; ++m) {
            // enumerate compositions of U into m parts in [1, 7] (odometer)
            std::vector<int> c(m, 1);
            while (true) {
                int s = 0;
                for (int k : c) s += k;
                if (s == U && c[0] >= upper_low_mink(b)) out.push_back(c);
                int i = m - 1;
                while (i >= 0 && c[i] == UPPER_MAXK) c[i--] = 1;
                if (i < 0) break;
                ++c[i];
            }
        }
    }
    return out;
}

// one cache line: "<arch> cu=<n> log2n=<k> upper=a,b,c rows=<r> zeta=<z> ms=<t>"
inline std::string schedule_line(const char *arch, int cus, int log2n, const Schedule &s, double ms)
{
    std::string u;
    for (size_t i = 0; i < s.upper.size(); ++i) u += (i ? "," : "") + std::to_string(s.upper[i]);
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s cu=%d log2n=%d upper=%s rows=%d zeta=%d ms=%.4f", arch, cus, log2n,
                  u.empty() ? "-" : u.c_str(), s.rows_mult, s.zeta_mult, ms);
    return buf;
}

// parse one line; false when it is malformed, for another device, or invalid
inline bool schedule_parse(const char *line, const char *arch, int cus, int &log2n, Schedule &s)
{
    char a[64] = {0}, up[96] = {0};
    int cu = 0, lg = 0, rows = 0, zeta = 0;
    double ms = 0;
    if (std::sscanf(line, "%63s cu=%d log2n=%d upper=%95s rows=%d zeta=%d ms=%lf", a, &cu, &lg, up, &rows, &zeta,
                    &ms) != 7)
        return false;
    if (std::strcmp(a, arch) != 0 || cu != cus || !fast_path(lg)) return false;
    if (rows < 1 || rows > 16 || zeta < 1 || zeta > 64) return false;
    Schedule r;
    r.rows_mult = rows;
    r.zeta_mult = zeta;
    if (std::strcmp(up, "-") != 0) {
        const char *p = up;
        while (*p) {
            char *end = nullptr;
            const long k = std::strtol(p, &end, 10);
            if (end == p) return false;
            r.upper.push_back((int)k);
            p = *end == ',' ? end + 1 : end;
            if (*end && *end != ',') return false;
        }
        if (!upper_valid(lg - 6, r.upper)) return false;
    }
    log2n = lg;
    s = r;
    return true;
}

}  // namespace fpmul_plan
