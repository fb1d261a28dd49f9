// k_bf3.h -- upper butterfly passes (Alg. 2 and its inverse, layers at or
// above 11) with every layer's K table resident in LDS.
//
// A workgroup of 512 threads owns a tile of 2^12 values: the K <= 7 layers of
// the pass (tile rows) times 2^(12-K) consecutive columns.  Each thread holds
// 8 values that differ in the three tile bits of the current layer group
// (the arrangement of the k_bf2.h passes), and the multiplications are the
// same tmul + pmul of x * (K + beta).
//
// What differs from k_bf2_upper: the K tables of all layers of the pass stay
// in LDS for the whole run of tiles (up to 7 x 16 KiB) beside a separate
// exchange area, so a table is rebuilt only when its K changes -- once per
// 2^(r + 1 + i_lo - 5) tiles for row r, i.e. almost never -- instead of for
// every layer group of every tile.  The price is one workgroup per CU, so
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
        b2_layer<M, INV, false>(x, x, s_tab[row], s_pt, T, bl_t, bw1, bw2);
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
