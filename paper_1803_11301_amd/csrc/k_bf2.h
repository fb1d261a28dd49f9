// k_bf2.h -- butterfly passes (Alg. 2 and its inverse) with the values in
// registers across groups of three layers.
//
// A tile holds 2^11 values of a transform (per operand).  256 threads each
// hold 8 of them, differing in the three tile bits of the current layer
// group, so those layers run in registers; between groups the tile is
// exchanged through LDS.  Each multiplication x * (K + beta) (gf_device.h) is
//   tmul: 8 lookups in the 8-bit window table of K (one table per layer,
//         shared by the whole tile), and
//   pmul: beta in V_8 applied to all bytes at once with v_perm_b32 over the
//         byte tables of beta on its three bit groups {0,1,2}, {3,4,5}, {6,7}
//         (multiplication by beta is linear over GF(2)),
// combined with three-input XORs.
#pragma once

#include <type_traits>

#include "gf_device.h"
#include "k_butterfly.h"

#define B2_TILE_LG 11
#define B2_THREADS 256

// byte tables of beta * y on the bit groups of y: t0 (bits 0-2, 8 entries in
// two words), t1 (bits 3-5), t2 (bits 6-7, 4 entries); 32 bytes per entry
struct PermTab {
    uint32_t t0lo, t0hi, t1lo, t1hi, t2, pad0, pad1, pad2;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ int b2_pad(int e) { return e + (e >> 3); }

// acc XOR x * (K + beta): tab = window table of K (compile-time LDS address in
// the callers), (t01, t2) = byte tables of beta
__device__ __forceinline__ uint64_t b2_mul_acc(const uint64_t *__restrict__ tab, uint4 t01, uint32_t t2, uint64_t x,
                                               uint64_t acc)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint64_t v0 = tab[lo & 255u], v1 = tab[256 + ((lo >> 8) & 255u)];
    const uint64_t v2 = tab[512 + ((lo >> 16) & 255u)], v3 = tab[768 + (lo >> 24)];
    const uint64_t v4 = tab[1024 + (hi & 255u)], v5 = tab[1280 + ((hi >> 8) & 255u)];
    const uint64_t v6 = tab[1536 + ((hi >> 16) & 255u)], v7 = tab[1792 + (hi >> 24)];
    const uint32_t sl0 = lo & 0x07070707u, sl1 = (lo >> 3) & 0x07070707u, sl2 = (lo >> 6) & 0x03030303u;
    const uint32_t sh0 = hi & 0x07070707u, sh1 = (hi >> 3) & 0x07070707u, sh2 = (hi >> 6) & 0x03030303u;
    const uint32_t pl = xor3(__builtin_amdgcn_perm(t01.y, t01.x, sl0), __builtin_amdgcn_perm(t01.w, t01.z, sl1),
                             __builtin_amdgcn_perm(t2, t2, sl2));
    const uint32_t ph = xor3(__builtin_amdgcn_perm(t01.y, t01.x, sh0), __builtin_amdgcn_perm(t01.w, t01.z, sh1),
                             __builtin_amdgcn_perm(t2, t2, sh2));
    const uint32_t rl = xor3(xor3((uint32_t)v0, (uint32_t)v1, (uint32_t)v2), xor3((uint32_t)v3, (uint32_t)v4,
                             (uint32_t)v5), xor3((uint32_t)v6, (uint32_t)v7, pl)) ^ (uint32_t)acc;
    const uint32_t rh = xor3(xor3((uint32_t)(v0 >> 32), (uint32_t)(v1 >> 32), (uint32_t)(v2 >> 32)),
                             xor3((uint32_t)(v3 >> 32), (uint32_t)(v4 >> 32), (uint32_t)(v5 >> 32)),
                             xor3((uint32_t)(v6 >> 32), (uint32_t)(v7 >> 32), ph)) ^ (uint32_t)(acc >> 32);
    return (uint64_t)rl | ((uint64_t)rh << 32);
}

// One layer on the registers: the layer bit is register bit M; the block
// index of a pair is b_t | (register bits above M) * bw, beta = iota(2 (b mod 128)).
template <int M, bool INV>
__device__ __forceinline__ void b2_layer(uint64_t (&xa)[8], const uint64_t *__restrict__ tab,
                                         const PermTab *__restrict__ s_pt, const DevTables *__restrict__ T,
                                         uint32_t bl_t, uint32_t bw1, uint32_t bw2)
{
    // tables of the thread's beta from LDS; those of the blocks that differ in
    // register bits above M follow by linearity: tab(beta + beta') = tab(beta) +
    // tab(beta'), with beta' = iota(2 bw) the same for the whole workgroup
    const PermTab *P = s_pt + (bl_t & 127u);
    const uint4 b01 = *reinterpret_cast<const uint4 *>(P);
    const uint32_t b2 = P->t2;
    uint4 c01[2] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0)};
    uint32_t c2[2] = {0, 0};
    if (M == 0) {
        const uint32_t *q1 = T->pt_beta8[bw1], *q2 = T->pt_beta8[bw2];
        c01[0] = make_uint4(q1[0], q1[1], q1[2], q1[3]);
        c2[0] = q1[4];
        c01[1] = make_uint4(q2[0], q2[1], q2[2], q2[3]);
        c2[1] = q2[4];
    } else if (M == 1) {
        const uint32_t *q2 = T->pt_beta8[bw2];
        c01[0] = make_uint4(q2[0], q2[1], q2[2], q2[3]);
        c2[0] = q2[4];
    }
#pragma unroll
    for (int u = 0; u < (1 << (2 - M)); ++u) {
        uint4 t01 = b01;
        uint32_t t2 = b2;
#pragma unroll
        for (int q = 0; q < 2 - M; ++q)
            if ((u >> q) & 1) {
                t01.x ^= c01[q].x;
                t01.y ^= c01[q].y;
                t01.z ^= c01[q].z;
                t01.w ^= c01[q].w;
                t2 ^= c2[q];
            }
#pragma unroll
        for (int low = 0; low < (1 << M); ++low) {
            const int r0 = low | (u << (M + 1)), r1 = r0 | (1 << M);
            if (!INV) {
                const uint64_t h0 = b2_mul_acc(tab, t01, t2, xa[r1], xa[r0]);
                xa[r1] ^= h0;
                xa[r0] = h0;
            } else {
                const uint64_t p1 = xa[r0] ^ xa[r1];
                xa[r0] = b2_mul_acc(tab, t01, t2, p1, xa[r0]);
                xa[r1] = p1;
            }
        }
    }
}

// ------------------------------------------------------------ upper pass ---
//
// Layers i_lo .. i_lo + K - 1 on tiles of 2^K rows (global bits i_lo ..) by
// 2^(11-K) columns (global bits 0 ..).  Tile bits: columns 0 .. LGW-1, rows
// LGW .. 10.  The rows are taken in groups of three from the top (forward)
// or from the bottom (inverse); a group of fewer than three rows is padded
// with the highest other tile bits, on which no layer runs.

template <int K, int TLG = B2_TILE_LG>
struct B2Upper {
    static constexpr int LGW = TLG - K;
    static constexpr int NC = (K + 2) / 3;
    // rows of group c (forward order): [lo, hi]
    static constexpr int lo_row(int c) { return K - 3 * c - 3 < 0 ? 0 : K - 3 * c - 3; }
    static constexpr int hi_row(int c) { return K - 3 * c - 1; }
};

// register bits (tile bits s0 < s1 < s2) of group c and which are layers
struct B2Group {
    int s[3];
    int layer[3];   // 1 if a layer runs on register bit m
};

template <int K, int TLG = B2_TILE_LG>
__device__ __forceinline__ B2Group b2_upper_group(int c)
{
    using U = B2Upper<K, TLG>;
    const int lo = U::lo_row(c), hi = U::hi_row(c), n = hi - lo + 1;
    int bits[3], lay[3], cnt = 0;
    for (int r = lo; r <= hi; ++r) {
        bits[cnt] = U::LGW + r;
        lay[cnt++] = 1;
    }
    for (int b = TLG - 1; cnt < 3 && b >= 0; --b) {
        if (b >= U::LGW + lo && b <= U::LGW + hi) continue;
        bits[cnt] = b;
        lay[cnt++] = 0;
    }
    (void)n;
    // sort ascending (three elements)
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (bits[b] < bits[a]) {
                int t = bits[a];
                bits[a] = bits[b];
                bits[b] = t;
                t = lay[a];
                lay[a] = lay[b];
                lay[b] = t;
            }
    B2Group g;
    for (int m = 0; m < 3; ++m) {
        g.s[m] = bits[m];
        g.layer[m] = lay[m];
    }
    return g;
}

// tile index of thread t's value with register bits zero: the thread bits
// fill the tile bits outside the group, lowest first
template <int TLG = B2_TILE_LG>
__device__ __forceinline__ int b2_thread_base(const B2Group &g, int t)
{
    int e = 0, q = 0;
    for (int b = 0; b < TLG; ++b) {
        if (b == g.s[0] || b == g.s[1] || b == g.s[2]) continue;
        e |= ((t >> q) & 1) << b;
        ++q;
    }
    return e;
}

template <int K, int TLG = B2_TILE_LG>
__device__ __forceinline__ uint64_t b2_upper_global(int e, uint64_t gbase, int i_lo)
{
    constexpr int LGW = B2Upper<K, TLG>::LGW;
    return gbase | (uint64_t)(e & ((1 << LGW) - 1)) | ((uint64_t)(e >> LGW) << i_lo);
}

// The 64 basis images of a K table: K = 2^(32+d) + bh << 8 in Cantor
// coordinates, so the images are those of v_{32+d} plus the rows of the set
// bits of bh (gf_device.h); the rows come from an LDS copy of the table.
__device__ __forceinline__ void b2_basis(uint64_t *img, int d, uint32_t bh, const uint64_t (*s_pb)[64],
                                         const DevTables *__restrict__ T, int t64)
{
    uint64_t v = T->gbasis[d][t64];
#pragma unroll
    for (int b = 0; b < 24; ++b)
        if ((bh >> b) & 1u) v ^= s_pb[b][t64];
    img[t64] = v;
}

__device__ __forceinline__ void b2_load_pbasis(uint64_t (*s_pb)[64], const DevTables *__restrict__ T, int tid, int nth)
{
    for (int q = tid; q < 24 * 64; q += nth) (&s_pb[0][0])[q] = (&T->pbasis[0][0])[q];
}

// the images of register bit m's layer are cached in slot[m] of s_img; they
// are recomputed (threads 64 m .. 64 m + 63) only when that layer's K changes
__device__ __forceinline__ void b2_fill(const B2Group &g, uint64_t (*s_tab)[2048], const uint64_t (*s_img)[64],
                                        const int (&slot)[3], int tid, int nth)
{
    for (int item = tid; item < 3 * 256; item += nth) {
        const int m = item >> 8;
        if (g.layer[m]) ktable_fill_item(s_tab[m], s_img[slot[m]], item & 255);
    }
}

// ----------------------------------------------------------- bottom pass ---
//
// Layers 10 .. 0 on contiguous tiles of 2^11 values (tile bits = global bits
// 0 .. 10).  Groups of register bits, forward order: {8,9,10}, {5,6,7},
// {2,3,4}, {0,1} with bit 10 carried.  In layers 0, 1, 2 the 1024 blocks of
// a tile would need several K tables with beta in V_8, so there the split is
// K16 + beta16 with beta16 = iota(2 (b mod 2^15)) in V_16:
//   x * beta16 = beta0 * x + beta1 * (x * v8)   (beta16 = beta1 v8 + beta0),
// and x * v8 acts on each tower pair (y1 v8 + y0) as
//   (y0 + y1) v8 + v7 y1      (v8^2 = v8 + v7, Eq. 2).

struct B2Bottom {
    static constexpr int NC = 4;
};

__device__ __forceinline__ B2Group b2_bottom_group(int c)
{
    B2Group g;
    if (c < 3) {
        const int lo = 8 - 3 * c;
        g.s[0] = lo;
        g.s[1] = lo + 1;
        g.s[2] = lo + 2;
        g.layer[0] = g.layer[1] = g.layer[2] = 1;
    } else {
        g.s[0] = 0;
        g.s[1] = 1;
        g.s[2] = 10;
        g.layer[0] = g.layer[1] = 1;
        g.layer[2] = 0;
    }
    return g;
}

// layers below 3 use the V_16 split
__device__ __forceinline__ bool b2_wide(int i) { return i < 3; }

// v_perm multiply of the four bytes of w by the byte with tables P
__device__ __forceinline__ uint32_t b2_pmul32(const uint4 &t01, uint32_t t2, uint32_t w)
{
    const uint32_t s0 = w & 0x07070707u, s1 = (w >> 3) & 0x07070707u, s2 = (w >> 6) & 0x03030303u;
    return xor3(__builtin_amdgcn_perm(t01.y, t01.x, s0), __builtin_amdgcn_perm(t01.w, t01.z, s1),
                __builtin_amdgcn_perm(t2, t2, s2));
}

// x * beta16 on the two tower pairs a0 + a1 y of a 32-bit word, with y^2 =
// y + c (c = v_7, Cantor byte 0x80) and beta16 = b0 + b1 y: the low byte of a
// pair becomes a0 b0 + a1 (b1 c), the high byte a0 b1 + a1 (b0 + b1).  The
// three byte products (by b0, b1 and b1 c; tables P0, P1, PC) share one set of
// selectors, and one byte permutation places the cross terms.
__device__ __forceinline__ uint32_t b2_mulv16(const uint4 &p0, uint32_t p02, const uint4 &p1, uint32_t p12,
                                              const uint4 &pc, uint32_t pc2, uint32_t w)
{
    const uint32_t s0 = w & 0x07070707u, s1 = (w >> 3) & 0x07070707u, s2 = (w >> 6) & 0x03030303u;
    auto pm = [&](const uint4 &t01, uint32_t t2) {
        return xor3(__builtin_amdgcn_perm(t01.y, t01.x, s0), __builtin_amdgcn_perm(t01.w, t01.z, s1),
                    __builtin_amdgcn_perm(t2, t2, s2));
    };
    const uint32_t a = pm(p0, p02), b = pm(p1, p12), bc = pm(pc, pc2);
    // bytes (bc[1], b[0], bc[3], b[2]): a1 b1 c to the low byte, a0 b1 to the high byte
    return xor3(a, __builtin_amdgcn_perm(bc, b, 0x02070005u), b & 0xFF00FF00u);
}

// acc XOR x * (K16 + beta16): tab = window table of K16, (P0, P1, PC) = byte
// tables of b0, b1 and b1 c
__device__ __forceinline__ uint64_t b2_mul_acc16(const uint64_t *__restrict__ tab, const uint4 &p0, uint32_t p02,
                                                 const uint4 &p1, uint32_t p12, const uint4 &pc, uint32_t pc2,
                                                 uint64_t x, uint64_t acc)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint64_t v0 = tab[lo & 255u], v1 = tab[256 + ((lo >> 8) & 255u)];
    const uint64_t v2 = tab[512 + ((lo >> 16) & 255u)], v3 = tab[768 + (lo >> 24)];
    const uint64_t v4 = tab[1024 + (hi & 255u)], v5 = tab[1280 + ((hi >> 8) & 255u)];
    const uint64_t v6 = tab[1536 + ((hi >> 16) & 255u)], v7 = tab[1792 + (hi >> 24)];
    const uint32_t al = b2_mulv16(p0, p02, p1, p12, pc, pc2, lo), ah = b2_mulv16(p0, p02, p1, p12, pc, pc2, hi);
    const uint32_t rl = xor3(xor3((uint32_t)v0, (uint32_t)v1, (uint32_t)v2), xor3((uint32_t)v3, (uint32_t)v4,
                             (uint32_t)v5), xor3((uint32_t)v6, (uint32_t)v7, al)) ^ (uint32_t)acc;
    const uint32_t rh = xor3(xor3((uint32_t)(v0 >> 32), (uint32_t)(v1 >> 32), (uint32_t)(v2 >> 32)),
                             xor3((uint32_t)(v3 >> 32), (uint32_t)(v4 >> 32), (uint32_t)(v5 >> 32)),
                             xor3((uint32_t)(v6 >> 32), (uint32_t)(v7 >> 32), ah)) ^ (uint32_t)(acc >> 32);
    return (uint64_t)rl | ((uint64_t)rh << 32);
}

// byte tables of beta16 = b0 + b1 y: those of b0, b1 and b1 c.  They are
// linear in beta16, so the tables of beta16 + d are those of beta16 XOR those of d.
struct B16Tabs {
    uint4 p0, p1, pc;
    uint32_t p02, p12, pc2;
};

__device__ __forceinline__ B16Tabs b16_tabs(const PermTab *__restrict__ pt, uint32_t beta)
{
    B16Tabs t;
    const PermTab *P0 = pt + (beta & 255u), *P1 = pt + (beta >> 8);
    t.p0 = *reinterpret_cast<const uint4 *>(P0);
    t.p1 = *reinterpret_cast<const uint4 *>(P1);
    t.p02 = P0->t2;
    t.p12 = P1->t2;
    const PermTab *PC = pt + ((t.p12 >> 16) & 255u);   // b1 c: entry 2 of P1's bit-6/7 table
    t.pc = *reinterpret_cast<const uint4 *>(PC);
    t.pc2 = PC->t2;
    return t;
}

__device__ __forceinline__ uint4 b16_xor4(const uint4 &a, const uint4 &b)
{
    return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
}

__device__ __forceinline__ B16Tabs b16_xor(const B16Tabs &a, const B16Tabs &b)
{
    B16Tabs t;
    t.p0 = b16_xor4(a.p0, b.p0);
    t.p1 = b16_xor4(a.p1, b.p1);
    t.pc = b16_xor4(a.pc, b.pc);
    t.p02 = a.p02 ^ b.p02;
    t.p12 = a.p12 ^ b.p12;
    t.pc2 = a.pc2 ^ b.pc2;
    return t;
}

// one V_16 layer on register bit M: block of a pair = b_t | register bits
// above M times bw; beta16 = iota(2 (b mod 2^15)).  The thread's own beta16
// comes through the iota tables of the low two Cantor bytes (s_io16) and its
// byte tables from LDS; the blocks that differ in register bits above M add
// iota(2 bw), the same for the whole workgroup, whose tables are read from T.
template <int M, bool INV>
__device__ __forceinline__ void b2_layer16(uint64_t (&xa)[8], const uint64_t *__restrict__ tab,
                                           const PermTab *__restrict__ s_pt8, const uint16_t (*s_io16)[256],
                                           const DevTables *__restrict__ T, uint32_t b_t, uint32_t bw1,
                                           uint32_t bw2)
{
    const uint32_t v = (2u * b_t) & 0xFFFFu;
    const B16Tabs base = b16_tabs(s_pt8, (uint32_t)s_io16[0][v & 255u] ^ (uint32_t)s_io16[1][v >> 8]);
    auto delta = [&](uint32_t bw) {   // bw < 2^15
        const uint32_t w = 2u * bw;
        const uint32_t d = (uint32_t)(T->iota[0][w & 255u] ^ T->iota[1][w >> 8]) & 0xFFFFu;
        return b16_tabs(reinterpret_cast<const PermTab *>(T->pt8), d);
    };
    B16Tabs d1 = base, d2 = base, d3 = base;
    if (M == 0) {
        d1 = delta(bw1);
        d2 = delta(bw2);
        d3 = b16_xor(d1, d2);
    } else if (M == 1) {
        d1 = delta(bw2);
    }
#pragma unroll
    for (int u = 0; u < (1 << (2 - M)); ++u) {
        const B16Tabs t = u == 0 ? base : b16_xor(base, u == 1 ? d1 : u == 2 ? d2 : d3);
#pragma unroll
        for (int low = 0; low < (1 << M); ++low) {
            const int r0 = low | (u << (M + 1)), r1 = r0 | (1 << M);
            if (!INV) {
                const uint64_t h0 = b2_mul_acc16(tab, t.p0, t.p02, t.p1, t.p12, t.pc, t.pc2, xa[r1], xa[r0]);
                xa[r1] ^= h0;
                xa[r0] = h0;
            } else {
                const uint64_t p = xa[r0] ^ xa[r1];
                xa[r0] = b2_mul_acc16(tab, t.p0, t.p02, t.p1, t.p12, t.pc, t.pc2, p, xa[r0]);
                xa[r1] = p;
            }
        }
    }
}

// images for the layers of group g: slot = layer index i, key = its bh
__device__ __forceinline__ void b2_bottom_images(const B2Group &g, uint64_t (*s_img)[64], uint32_t (&key)[11],
                                                 const uint64_t (*s_pb)[64], uint64_t gbase, int l,
                                                 const DevTables *__restrict__ T, int tid)
{
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        if (!g.layer[m]) continue;
        const int i = g.s[m];
        // K = 2^(32+d) + (b >> 7) << 8 (V_8 split) or 2^(32+d) + (b >> 15) << 16 (V_16 split)
        const uint32_t bh = b2_wide(i) ? (uint32_t)(gbase >> (i + 16)) << 8 : (uint32_t)(gbase >> (i + 8));
        if (key[i] != bh) {
            if ((tid >> 6) == m) b2_basis(s_img[i], l - i, bh, s_pb, T, tid & 63);
            key[i] = bh;
        }
    }
}

template <bool INV>
__device__ __forceinline__ void b2_bottom_compute(const B2Group &g, uint64_t (&xa)[8],
                                                  uint64_t (*s_tab)[2048], const PermTab *s_ptb,
                                                  const PermTab *s_pt8, const uint16_t (*s_io16)[256],
                                                  uint64_t gb_t, const DevTables *__restrict__ T)
{
    auto run = [&](auto Mc) {
        constexpr int M = decltype(Mc)::value;
        if (!g.layer[M]) return;
        const int i = g.s[M];
        if (b2_wide(i)) {
            const uint32_t b_t = (uint32_t)(gb_t >> (i + 1)) & 0x7FFFu;
            const uint32_t bw1 = (1u << g.s[1]) >> (i + 1), bw2 = (1u << g.s[2]) >> (i + 1);
            b2_layer16<M, INV>(xa, s_tab[M], s_pt8, s_io16, T, b_t, bw1 & 0x7FFFu, bw2 & 0x7FFFu);
        } else {
            const uint32_t bl_t = (uint32_t)(gb_t >> (i + 1)) & 127u;
            const uint32_t bw1 = ((1u << g.s[1]) >> (i + 1)) & 127u, bw2 = ((1u << g.s[2]) >> (i + 1)) & 127u;
            b2_layer<M, INV>(xa, s_tab[M], s_ptb, T, bl_t, bw1, bw2);
        }
    };
    if (!INV) {
        run(std::integral_constant<int, 2>());
        run(std::integral_constant<int, 1>());
        run(std::integral_constant<int, 0>());
    } else {
        run(std::integral_constant<int, 0>());
        run(std::integral_constant<int, 1>());
        run(std::integral_constant<int, 2>());
    }
}

// MODE: BF_FWD or BF_INV; l >= 11; grid <= 2^(l-11).  A grid of two rows
// takes A (y = 0) and B (y = 1), each tile of each transform on a workgroup
// of its own (a workgroup taking the same tile of both shares its K tables
// between them but leaves half the workgroups: 7 us slower per product).
template <int MODE>
__global__ __launch_bounds__(B2_THREADS, 2) void k_bf2_bottom(uint64_t *A0, uint64_t *B0, int l,
                                                                           const DevTables *__restrict__ T)
{
    constexpr bool INV = MODE == BF_INV;
    uint64_t *__restrict__ A = blockIdx.y ? B0 : A0;
    constexpr int NC = B2Bottom::NC;
    __shared__ __align__(16) uint64_t s_tab[3][2048];   // K tables; the exchange area aliases them
    __shared__ __align__(16) PermTab s_ptb[128];        // tables of iota(2 bl), bl < 128
    __shared__ __align__(16) PermTab s_pt8[256];        // tables of every byte of V_8
    __shared__ uint16_t s_io16[2][256];                 // iota of the low two Cantor bytes (V_16)
    __shared__ uint64_t s_pb[24][64];                   // basis rows of the bits of bh
    __shared__ uint64_t s_img[B2_TILE_LG][64];          // basis images of each layer's K, cached
    uint64_t *stA = &s_tab[0][0];
    const int tid = threadIdx.x, nth = blockDim.x;

    for (int q = tid; q < 128 * 8; q += nth)
        reinterpret_cast<uint32_t *>(s_ptb)[q] = reinterpret_cast<const uint32_t *>(T->pt_beta8)[q];
    for (int q = tid; q < 256 * 8; q += nth)
        reinterpret_cast<uint32_t *>(s_pt8)[q] = reinterpret_cast<const uint32_t *>(T->pt8)[q];
    for (int q = tid; q < 2 * 256; q += nth) (&s_io16[0][0])[q] = (uint16_t)(&T->iota[0][0])[q];
    b2_load_pbasis(s_pb, T, tid, nth);
    __syncthreads();

    const uint64_t ntiles = 1ull << (l - B2_TILE_LG);
    // contiguous runs of tiles keep most layers' K (and the cached images) unchanged
    const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t_beg = (uint64_t)blockIdx.x * per, t_end = t_beg + per < ntiles ? t_beg + per : ntiles;
    uint32_t key[B2_TILE_LG];
#pragma unroll
    for (int i = 0; i < B2_TILE_LG; ++i) key[i] = 0xFFFFFFFFu;
    uint64_t xa[8];
    for (uint64_t tile = t_beg; tile < t_end; ++tile) {
        const uint64_t gbase = tile << B2_TILE_LG;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const int c = INV ? NC - 1 - cc : cc;
            const B2Group g = b2_bottom_group(c);
            const int e_t = b2_thread_base(g, tid);
            const uint64_t gb_t = gbase | (uint64_t)e_t;
            if (cc == 0) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    xa[r] = A[gbase | (uint64_t)e];
                }
                __syncthreads();   // the previous tile is done with the tables
                b2_bottom_images(g, s_img, key, s_pb, gbase, l, T, tid);
                __syncthreads();
            } else {
                const B2Group gp = b2_bottom_group(INV ? c + 1 : c - 1);
                const int ep = b2_thread_base(gp, tid);
                __syncthreads();   // done with the previous tables (the exchange area aliases them)
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = ep | ((r & 1) << gp.s[0]) | (((r >> 1) & 1) << gp.s[1]) | ((r >> 2) << gp.s[2]);
                    stA[b2_pad(e)] = xa[r];
                }
                b2_bottom_images(g, s_img, key, s_pb, gbase, l, T, tid);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    xa[r] = stA[b2_pad(e)];
                }
                __syncthreads();   // exchange area free for the tables
            }
            int slot[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) slot[m] = g.layer[m] ? g.s[m] : 0;
            b2_fill(g, s_tab, s_img, slot, tid, nth);
            __syncthreads();
            b2_bottom_compute<INV>(g, xa, s_tab, s_ptb, s_pt8, s_io16, gb_t, T);
            if (cc == NC - 1) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    A[gbase | (uint64_t)e] = xa[r];
                }
            }
        }
    }
}

// ------------------------------------------------------------ pointwise ---
// A[j] = A[j] * B[j] (Alg. 5, the pointwise step), tower Karatsuba with the
// GF(2^8) pair table in LDS (MulPairView layout); one workgroup per CU
__global__ __launch_bounds__(1024) void k_pointwise(uint64_t *__restrict__ A, const uint64_t *__restrict__ B,
                                                    uint64_t n, const DevTables *__restrict__ T)
{
    __shared__ __align__(16) uint8_t s_mp[MPV_BYTES];
    const int tid = threadIdx.x, nth = blockDim.x;
    const uint4 *src = reinterpret_cast<const uint4 *>(&T->mulp[0][0]);
    uint4 *dst = reinterpret_cast<uint4 *>(s_mp);
    for (int idx = tid; idx < 131072 / 16; idx += nth) dst[idx] = src[idx];
    for (int q = tid; q < 512; q += nth) reinterpret_cast<uint16_t *>(s_mp + MPV_OFF_C15)[q] = (&T->c15[0][0])[q];
    for (int q = tid; q < 1024; q += nth) reinterpret_cast<uint32_t *>(s_mp + MPV_OFF_C31)[q] = (&T->c31[0][0])[q];
    __syncthreads();
    const MulPairView mv{s_mp};
    // PW_ILP independent products per thread and iteration, so that their
    // lookups overlap (one workgroup per CU leaves few waves to hide them)
    constexpr int PW_ILP = 4;
    const uint64_t G = (uint64_t)gridDim.x * nth;
    uint64_t j = (uint64_t)blockIdx.x * nth + tid;
    for (; j + (PW_ILP - 1) * G < n; j += PW_ILP * G) {
        uint64_t a[PW_ILP], b[PW_ILP];
#pragma unroll
        for (int k = 0; k < PW_ILP; ++k) {
            a[k] = A[j + k * G];
            b[k] = B[j + k * G];
        }
#pragma unroll
        for (int k = 0; k < PW_ILP; ++k) A[j + k * G] = mv.m64(a[k], b[k]);
    }
    for (; j < n; j += G) A[j] = mv.m64(A[j], B[j]);
}

// A[j] = A[j]^2: the pointwise step of a square (Alg. 5 with both transforms
// equal).  Squaring is GF(2)-linear in characteristic 2, so a value's square
// is the XOR of its eight byte windows' squares, one lookup each in a 16 KiB
// table in LDS; the kernel streams the transform once.
#define SQ_THREADS 256
__global__ __launch_bounds__(SQ_THREADS) void k_square(uint64_t *__restrict__ A, uint64_t n,
                                                       const DevTables *__restrict__ T)
{
    __shared__ uint64_t s_sq[8][256];
    for (int q = threadIdx.x; q < 8 * 256; q += blockDim.x) (&s_sq[0][0])[q] = (&T->sq_win[0][0])[q];
    __syncthreads();
    const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += G) {
        const uint64_t x = A[j];
        uint64_t r = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) r ^= s_sq[k][(x >> (8 * k)) & 255u];
        A[j] = r;
    }
}
