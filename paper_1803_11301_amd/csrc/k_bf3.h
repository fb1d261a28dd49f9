// k_bf3.h -- butterfly passes (Alg. 2 and its inverse) with every layer's K
// table resident in LDS: upper passes (layers from 7, or from 11 for
// transforms below 2^20 values) and the bottom pass of layers 0 .. 6.
//
// A workgroup of 512 threads owns a tile of 2^12 values: the K <= 7 layers of
// the pass (tile rows) times 2^(12-K) consecutive columns.  Each thread holds
// 8 values that differ in the three tile bits of the current layer group
// (the arrangement of the k_bf2.h passes), and the multiplications are the
// same tmul + pmul of x * (K + beta).
//
// Unlike the 2^11-value passes of k_bf2.h, the K tables of all layers of the
// pass stay in LDS for the whole run of tiles (up to 7 x 16 KiB) beside a
// separate exchange area, so a table is rebuilt only when its K changes
// (layer i: once per 2^(i-4) tiles or less) instead of for every layer group
// of every tile.  The price is one workgroup per CU, so
// the next tile's values are loaded into registers while the current tile
// is computed.  The two operands of a product are taken by the two halves of
// the grid.
#pragma once

#include "k_bf2.h"

#define B3_TILE_LG 12
#define B3_THREADS 512
#define B3_STAGE_WORDS (4096 + 512)   // one padded tile in the exchange area

template <int K>
constexpr size_t bf3_upper_lds()
{
    return sizeof(uint64_t) * (size_t)(K * 2048 + B3_STAGE_WORDS + 64) + sizeof(PermTab) * 128;
}

template <int K, bool INV>
__device__ __forceinline__ void bf3_upper_compute(const B2Group &g, uint64_t (&x)[8], uint64_t (*s_tab)[2048],
                                                  const PermTab *s_pt, uint64_t gb_t, int i_lo,
                                                  const DevTables *__restrict__ T)
{
    constexpr int LGW = B2Upper<K, B3_TILE_LG>::LGW;
    uint64_t gw[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) gw[m] = b2_upper_global<K, B3_TILE_LG>(1 << g.s[m], 0, i_lo);
    auto run = [&](auto Mc) {
        constexpr int M = decltype(Mc)::value;
        if (!g.layer[M]) return;
        const int row = g.s[M] - LGW, i = i_lo + row;
        const uint32_t bl_t = (uint32_t)(gb_t >> (i + 1)) & 127u;
        const uint32_t bw1 = (uint32_t)(gw[1] >> (i + 1)) & 127u, bw2 = (uint32_t)(gw[2] >> (i + 1)) & 127u;
        b2_layer<M, INV>(x, s_tab[row], s_pt, T, bl_t, bw1, bw2);
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

// Layers i_lo .. i_lo + K - 1 of A (and of B when B is not null: the second
// half of the grid takes B; the grid is then even).  l >= 12, i_lo >= 12 - K.
template <bool INV, int K>
__global__ __launch_bounds__(B3_THREADS, 1) void k_bf3_upper(uint64_t *__restrict__ A, uint64_t *__restrict__ B,
                                                               int l, int i_lo, const DevTables *__restrict__ T)
{
    using U = B2Upper<K, B3_TILE_LG>;
    constexpr int NC = U::NC, LGW = U::LGW;
    __shared__ __align__(16) uint64_t s_tab[K][2048];       // K table of tile row r (layer i_lo + r)
    __shared__ __align__(16) uint64_t s_x[B3_STAGE_WORDS];  // exchange between layer groups
    __shared__ __align__(16) PermTab s_pt[128];
    __shared__ uint64_t s_img[64];                          // basis images of the table being built
    const int tid = threadIdx.x, nth = blockDim.x;

    for (int q = tid; q < 128 * 8; q += nth)
        reinterpret_cast<uint32_t *>(s_pt)[q] = reinterpret_cast<const uint32_t *>(T->pt_beta8)[q];

    const unsigned nops = B ? 2u : 1u, per_op = gridDim.x / nops;
    const unsigned op = blockIdx.x / per_op;
    if (op >= nops) return;   // uniform per workgroup
    uint64_t *__restrict__ X = op ? B : A;
    const uint64_t bid = blockIdx.x - (uint64_t)op * per_op;
    const int nlo = i_lo - LGW;
    const uint64_t ntiles = 1ull << (l - B3_TILE_LG);
    const uint64_t per = (ntiles + per_op - 1) / per_op;
    const uint64_t t_beg = bid * per, t_end = t_beg + per < ntiles ? t_beg + per : ntiles;
    if (t_beg >= t_end) return;   // uniform per workgroup

    auto gbase_of = [&](uint64_t tile) -> uint64_t {
        return ((tile >> nlo) << (i_lo + K)) | ((tile & ((1ull << nlo) - 1)) << LGW);
    };
    const B2Group g0 = b2_upper_group<K, B3_TILE_LG>(INV ? NC - 1 : 0);
    const int e0 = b2_thread_base<B3_TILE_LG>(g0, tid);
    auto load = [&](uint64_t tile, uint64_t(&v)[8]) {
        const uint64_t gbase = gbase_of(tile);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = e0 | ((r & 1) << g0.s[0]) | (((r >> 1) & 1) << g0.s[1]) | ((r >> 2) << g0.s[2]);
            v[r] = X[b2_upper_global<K, B3_TILE_LG>(e, gbase, i_lo)];
        }
    };

    uint32_t key[K];
#pragma unroll
    for (int r = 0; r < K; ++r) key[r] = 0xFFFFFFFFu;
    uint64_t x[8], nx[8];
    load(t_beg, nx);
    for (uint64_t tile = t_beg; tile < t_end; ++tile) {
        const uint64_t gbase = gbase_of(tile);
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = nx[r];
        if (tile + 1 < t_end) load(tile + 1, nx);   // in flight during this tile

        // rebuild the tables whose K changed (every table on the first tile);
        // K of row r depends only on bits of gbase above the tile, so the
        // test is uniform over the workgroup
        bool changed = false;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int i = i_lo + r;
            const uint32_t bh = (uint32_t)(gbase >> (i + 8));
            if (key[r] != bh) {
                key[r] = bh;
                changed = true;
                __syncthreads();   // s_tab[r] and s_img no longer read
                ktable_basis(s_img, l - i, bh, T, tid);
                __syncthreads();
                for (int item = tid; item < 256; item += nth) ktable_fill_item(s_tab[r], s_img, item);
            }
        }
        if (changed) __syncthreads();

#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const int c = INV ? NC - 1 - cc : cc;
            const B2Group g = b2_upper_group<K, B3_TILE_LG>(c);
            const int e_t = b2_thread_base<B3_TILE_LG>(g, tid);
            if (cc > 0) {
                const B2Group gp = b2_upper_group<K, B3_TILE_LG>(INV ? c + 1 : c - 1);
                const int ep = b2_thread_base<B3_TILE_LG>(gp, tid);
                __syncthreads();   // the previous exchange has been read
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = ep | ((r & 1) << gp.s[0]) | (((r >> 1) & 1) << gp.s[1]) | ((r >> 2) << gp.s[2]);
                    s_x[b2_pad(e)] = x[r];
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    x[r] = s_x[b2_pad(e)];
                }
            }
            bf3_upper_compute<K, INV>(g, x, s_tab, s_pt, b2_upper_global<K, B3_TILE_LG>(e_t, gbase, i_lo), i_lo,
                                      T);
            if (cc == NC - 1) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    X[b2_upper_global<K, B3_TILE_LG>(e, gbase, i_lo)] = x[r];
                }
            }
        }
    }
}

// ----------------------------------------------------------- bottom pass ---
//
// Layers 0 .. 6 (or 0 .. 5) on contiguous tiles of 2^12 values, every
// layer's K table resident.  Register groups (forward order) {4,5,6}, {1,2,3}
// and {0} (with two tile bits on which no layer runs), or {3,4,5} and {0,1,2}
// for six layers; an exchange between groups.  Every layer uses the V_16
// split of k_bf2.h: K16 = 2^(32+d) + (b >> 15) << 16 changes once per 2^(i+4)
// tiles, so the tables are rebuilt almost never (with the V_8 split, K of the
// lowest layers would change every tile or two and vary inside a 2^12 tile
// below layer 4).  With six bottom layers the lowest upper pass takes layer 6.

#define B3_BOT_LAYERS 7   // the default; a schedule may give the bottom pass 6 layers (two register groups)

// NL bottom layers in ceil(NL / 3) register groups
template <int NL>
__device__ __forceinline__ B2Group bf3_bottom_group(int c)
{
    // layers hi .. lo of group c, counted from the top, then padding bits from
    // the highest tile bits outside the group
    const int hi = NL - 1 - 3 * c, lo = hi - 2 < 0 ? 0 : hi - 2;
    int bits[3], lay[3], cnt = 0;
    for (int r = lo; r <= hi; ++r) {
        bits[cnt] = r;
        lay[cnt++] = 1;
    }
    for (int b = B3_TILE_LG - 1; cnt < 3; --b) {
        if (b >= lo && b <= hi) continue;
        bits[cnt] = b;
        lay[cnt++] = 0;
    }
    for (int x = 0; x < 3; ++x)
        for (int y = x + 1; y < 3; ++y)
            if (bits[y] < bits[x]) {
                int t = bits[x];
                bits[x] = bits[y];
                bits[y] = t;
                t = lay[x];
                lay[x] = lay[y];
                lay[y] = t;
            }
    B2Group g;
    for (int m = 0; m < 3; ++m) {
        g.s[m] = bits[m];
        g.layer[m] = lay[m];
    }
    return g;
}

template <bool INV>
__device__ __forceinline__ void bf3_bottom_compute(const B2Group &g, uint64_t (&x)[8], uint64_t (*s_tab)[2048],
                                                   const PermTab *s_pt8, const uint16_t (*s_io16)[256], uint64_t gb_t,
                                                   const DevTables *__restrict__ T)
{
    auto run = [&](auto Mc) {
        constexpr int M = decltype(Mc)::value;
        if (!g.layer[M]) return;
        const int i = g.s[M];
        const uint32_t b_t = (uint32_t)(gb_t >> (i + 1)) & 0x7FFFu;
        const uint32_t bw1 = ((1u << g.s[1]) >> (i + 1)) & 0x7FFFu, bw2 = ((1u << g.s[2]) >> (i + 1)) & 0x7FFFu;
        b2_layer16<M, INV>(x, s_tab[i], s_pt8, s_io16, T, b_t, bw1, bw2);
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

// Layers 0 .. NL - 1 (NL = 6 or 7) of A (and of B when B is not null: the
// second half of the grid takes B; the grid is then even).  l >= 12.
template <bool INV, int NL>
__global__ __launch_bounds__(B3_THREADS, 1) void k_bf3_bottom(uint64_t *__restrict__ A, uint64_t *__restrict__ B,
                                                                int l, const DevTables *__restrict__ T)
{
    static_assert(NL == 6 || NL == 7, "bottom pass of 6 or 7 layers");
    constexpr int NG = (NL + 2) / 3;   // register groups
    __shared__ __align__(16) uint64_t s_tab[NL][2048];   // K16 table of layer i
    __shared__ __align__(16) uint64_t s_x[B3_STAGE_WORDS];
    __shared__ __align__(16) PermTab s_pt8[256];        // tables of every byte of V_8
    __shared__ uint16_t s_io16[2][256];                 // iota of the low two Cantor bytes
    __shared__ uint64_t s_img[64];
    const int tid = threadIdx.x, nth = blockDim.x;

    for (int q = tid; q < 256 * 8; q += nth)
        reinterpret_cast<uint32_t *>(s_pt8)[q] = reinterpret_cast<const uint32_t *>(T->pt8)[q];
    for (int q = tid; q < 2 * 256; q += nth) (&s_io16[0][0])[q] = (uint16_t)(&T->iota[0][0])[q];
    __syncthreads();

    const unsigned nops = B ? 2u : 1u, per_op = gridDim.x / nops;
    const unsigned op = blockIdx.x / per_op;
    if (op >= nops) return;   // uniform per workgroup
    uint64_t *__restrict__ X = op ? B : A;
    const uint64_t bid = blockIdx.x - (uint64_t)op * per_op;
    const uint64_t ntiles = 1ull << (l - B3_TILE_LG);
    const uint64_t per = (ntiles + per_op - 1) / per_op;
    const uint64_t t_beg = bid * per, t_end = t_beg + per < ntiles ? t_beg + per : ntiles;
    if (t_beg >= t_end) return;   // uniform per workgroup

    const B2Group g0 = bf3_bottom_group<NL>(INV ? NG - 1 : 0);
    auto load = [&](uint64_t tile, uint64_t(&v)[8], int tid_t) {
        const uint64_t gbase = tile << B3_TILE_LG;
        const int e0 = b2_thread_base<B3_TILE_LG>(g0, tid_t);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = e0 | ((r & 1) << g0.s[0]) | (((r >> 1) & 1) << g0.s[1]) | ((r >> 2) << g0.s[2]);
            v[r] = X[gbase | (uint64_t)e];
        }
    };

    uint32_t key[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) key[i] = 0xFFFFFFFFu;
    uint64_t x[8], nx[8];
    load(t_beg, nx, tid);
    for (uint64_t tile = t_beg; tile < t_end; ++tile) {
        const uint64_t gbase = tile << B3_TILE_LG;
        // every address below depends on the thread index only; in the
        // forward pass, taking it through an opaque copy per tile keeps the
        // compiler from holding the offsets live (and spilled) across the loop
        // (the inverse pass has the registers, and runs faster without)
        int tid_t = tid;
        if constexpr (!INV) asm volatile("" : "+v"(tid_t));
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = nx[r];
        if (tile + 1 < t_end) load(tile + 1, nx, tid_t);   // in flight during this tile

        // rebuild the tables whose K16 changed; uniform over the workgroup
        bool changed = false;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const uint32_t bh = (uint32_t)(gbase >> (i + 16)) << 8;
            if (key[i] != bh) {
                key[i] = bh;
                changed = true;
                __syncthreads();   // s_tab[i] and s_img no longer read
                ktable_basis(s_img, l - i, bh, T, tid_t);
                __syncthreads();
                for (int item = tid_t; item < 256; item += nth) ktable_fill_item(s_tab[i], s_img, item);
            }
        }
        if (changed) __syncthreads();

#pragma unroll
        for (int cc = 0; cc < NG; ++cc) {
            const int c = INV ? NG - 1 - cc : cc;
            const B2Group g = bf3_bottom_group<NL>(c);
            const int e_t = b2_thread_base<B3_TILE_LG>(g, tid_t);
            if (cc > 0) {
                const B2Group gp = bf3_bottom_group<NL>(INV ? c + 1 : c - 1);
                const int ep = b2_thread_base<B3_TILE_LG>(gp, tid_t);
                __syncthreads();   // the previous exchange has been read
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = ep | ((r & 1) << gp.s[0]) | (((r >> 1) & 1) << gp.s[1]) | ((r >> 2) << gp.s[2]);
                    s_x[b2_pad(e)] = x[r];
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    x[r] = s_x[b2_pad(e)];
                }
            }
            bf3_bottom_compute<INV>(g, x, s_tab, s_pt8, s_io16, gbase | (uint64_t)e_t, T);
            if (cc == NG - 1) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = e_t | ((r & 1) << g.s[0]) | (((r >> 1) & 1) << g.s[1]) | ((r >> 2) << g.s[2]);
                    X[gbase | (uint64_t)e] = x[r];
                }
            }
        }
    }
}
