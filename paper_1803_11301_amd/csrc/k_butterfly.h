// k_butterfly.h -- Butterfly (Alg. 2) and its inverse as LDS-resident tile
// passes, for small transforms (l < 11) and the batch kernel.
//
// Layer i pairs indices j and j + 2^i inside blocks of 2^(i+1); the block
// b = j >> (i+1) fixes the multiplier s_i(v_{l+32} + b 2^(i+1)) whose Cantor
// vector is 2^(32+d) XOR 2b, d = l - i.
//
// The bottom pass runs layers R-1 .. 0 on contiguous tiles of 2^R values.
// For a product it runs the forward layers of A and B, the pointwise
// products and the inverse layers of C on the same tile (the low layers of
// the forward transforms, the pointwise step and the low layers of the
// inverse transform of Alg. 5), so those steps cost one HBM round trip.
//
// Each multiplication is x * (K + beta) = tmul(T_K, x) ^ bmul(beta, x) with K
// shared by 128 consecutive blocks (window table built in LDS) and beta in V_8
// (gf_device.h); the low layers of a tile need up to 2^(R-8) tables.
#pragma once

#include "gf_device.h"

#define BF_THREADS 1024       // bottom pass (one workgroup per CU)
#define BF_SLOTS 4            // K tables resident in LDS at once (16 KiB each)
#define BF_BOTTOM_R 11        // log2 of the bottom tile
#define BF_UPPER_MAXK 7       // layers per upper pass

enum { BF_FWD = 0, BF_INV = 1, BF_PRODUCT = 2 };

// LDS layout shared by both kernels (bytes)
#define BF_OFF_MUL8 0
#define BF_OFF_TAB (32 * 1024)
#define BF_OFF_BASIS (BF_OFF_TAB + BF_SLOTS * 2048 * 8)
#define BF_OFF_DATA (BF_OFF_BASIS + BF_SLOTS * 64 * 8)

__device__ __forceinline__ void bf_load_mul8_even(uint8_t *s_mul8e, const DevTables *__restrict__ T, int tid, int nth)
{
    // row a = 2r of the GF(2^8) table -> s_mul8e[r * 256 ..]
    const uint4 *src = reinterpret_cast<const uint4 *>(&T->mul8[0][0]);
    uint4 *dst = reinterpret_cast<uint4 *>(s_mul8e);
    for (int idx = tid; idx < 128 * 16; idx += nth) {
        int r = idx >> 4, c = idx & 15;
        dst[idx] = src[(2 * r) * 16 + c];
    }
}

// build the K tables for `cnt` consecutive values bh0 .. bh0+cnt-1 at depth d
__device__ __forceinline__ void bf_build(uint64_t *s_tab, uint64_t *s_basis, int d, uint32_t bh0, int cnt,
                                         const DevTables *__restrict__ T, int tid, int nth)
{
    int slot = tid >> 6;
    if (slot < cnt) ktable_basis(s_basis + slot * 64, d, bh0 + slot, T, tid & 63);
    // (tid >> 6 < cnt <= BF_SLOTS needs at least 64 * BF_SLOTS threads)
    __syncthreads();
    for (int item = tid; item < 256 * cnt; item += nth)
        ktable_fill_item(s_tab + (item >> 8) * 2048, s_basis + (item >> 8) * 64, item & 255);
    __syncthreads();
}

__device__ __forceinline__ void bf_fwd_pair(uint64_t *X, uint32_t p0, uint32_t p1, const uint64_t *tab,
                                            const uint8_t *row)
{
    uint64_t x0 = X[p0], x1 = X[p1];
    uint64_t h0 = x0 ^ tmul(tab, x1) ^ bmul(row, x1);
    X[p0] = h0;
    X[p1] = h0 ^ x1;
}

__device__ __forceinline__ void bf_inv_pair(uint64_t *X, uint32_t p0, uint32_t p1, const uint64_t *tab,
                                            const uint8_t *row)
{
    uint64_t h0 = X[p0], h1 = X[p1];
    uint64_t q1 = h0 ^ h1;
    X[p0] = h0 ^ tmul(tab, q1) ^ bmul(row, q1);
    X[p1] = q1;
}

// one layer i of the bottom tile (tile index H, 2^R values), on X (and Y if set)
__device__ void bf_bottom_layer(int i, bool inverse, uint64_t *X, uint64_t *Y, int l, int R, uint64_t H,
                                uint8_t *s_mul8e, uint64_t *s_tab, uint64_t *s_basis,
                                const DevTables *__restrict__ T, int tid, int nth)
{
    const int d = l - i;
    const int lgb = R - 1 - i;                      // log2 of the blocks in the tile
    const int lgpg = lgb < 7 ? lgb : 7;             // log2 of the blocks per K
    const int ngroups = 1 << (lgb - lgpg);
    const uint64_t bfirst = H << lgb;               // global block index of the first block
    const uint32_t bh_first = (uint32_t)(bfirst >> 7);
    const int per_group = 1 << (lgpg + i);          // butterflies per K group
    for (int g0 = 0; g0 < ngroups; g0 += BF_SLOTS) {
        const int cnt = ngroups - g0 < BF_SLOTS ? ngroups - g0 : BF_SLOTS;
        bf_build(s_tab, s_basis, d, bh_first + g0, cnt, T, tid, nth);
        const int total = cnt * per_group;
        for (int q = tid; q < total; q += nth) {
            const uint32_t qq = (uint32_t)(q + g0 * per_group);
            const uint32_t tb = qq >> i, off = qq & ((1u << i) - 1u);
            const uint32_t p0 = (tb << (i + 1)) | off, p1 = p0 | (1u << i);
            const int slot = (int)(tb >> lgpg) - g0;
            const uint32_t bl = (uint32_t)((bfirst + tb) & 127u);
            const uint64_t *tab = s_tab + slot * 2048;
            const uint8_t *row = s_mul8e + bl * 256;
            if (!inverse) {
                bf_fwd_pair(X, p0, p1, tab, row);
                if (Y) bf_fwd_pair(Y, p0, p1, tab, row);
            } else {
                bf_inv_pair(X, p0, p1, tab, row);
            }
        }
        __syncthreads();
    }
}

// One bottom tile H (2^R values at H * 2^R) on the LDS layout above, the even
// rows of the GF(2^8) table already in place.  MODE: BF_FWD / BF_INV on A, or
// BF_PRODUCT: forward A and B, pointwise A*B, inverse; result written to A.
template <int MODE>
__device__ void bf_bottom_tile(uint64_t *__restrict__ A, const uint64_t *__restrict__ B, int l, int R, uint64_t H,
                               uint8_t *smem, const DevTables *__restrict__ T, int tid, int nth)
{
    uint8_t *s_mul8e = smem + BF_OFF_MUL8;
    uint64_t *s_tab = reinterpret_cast<uint64_t *>(smem + BF_OFF_TAB);
    uint64_t *s_basis = reinterpret_cast<uint64_t *>(smem + BF_OFF_BASIS);
    uint64_t *s_A = reinterpret_cast<uint64_t *>(smem + BF_OFF_DATA);
    uint64_t *s_B = s_A + (1u << R);
    const uint64_t TT = 1ull << R;
    const uint64_t base = H << R;
    for (uint32_t e = tid; e < TT; e += nth) {
        s_A[e] = A[base + e];
        if (MODE == BF_PRODUCT) s_B[e] = B[base + e];
    }
    __syncthreads();

    if (MODE != BF_INV)
        for (int i = R - 1; i >= 0; --i)
            bf_bottom_layer(i, false, s_A, MODE == BF_PRODUCT ? s_B : nullptr, l, R, H, s_mul8e, s_tab, s_basis, T,
                            tid, nth);

    if (MODE == BF_PRODUCT) {
        // the odd rows of the GF(2^8) table and the v_15 / v_31 tables go to the
        // slot area, which follows the even rows (the Mul8View layout)
        static_assert(BF_OFF_TAB == BF_OFF_MUL8 + 32768, "odd rows must follow the even rows");
        static_assert(BF_OFF_DATA - BF_OFF_MUL8 >= M8V_BYTES, "slot area too small for the product tables");
        uint8_t *s_odd = smem + BF_OFF_TAB;
        uint16_t *s_c15 = reinterpret_cast<uint16_t *>(smem + BF_OFF_MUL8 + M8V_OFF_C15);
        uint32_t *s_c31 = reinterpret_cast<uint32_t *>(smem + BF_OFF_MUL8 + M8V_OFF_C31);
        const uint4 *src = reinterpret_cast<const uint4 *>(&T->mul8[0][0]);
        uint4 *dst = reinterpret_cast<uint4 *>(s_odd);
        for (int idx = tid; idx < 128 * 16; idx += nth) dst[idx] = src[(2 * (idx >> 4) + 1) * 16 + (idx & 15)];
        for (int idx = tid; idx < 512; idx += nth) s_c15[idx] = (&T->c15[0][0])[idx];
        for (int idx = tid; idx < 1024; idx += nth) s_c31[idx] = (&T->c31[0][0])[idx];
        __syncthreads();
        const Mul8View mv{smem + BF_OFF_MUL8};
        for (uint32_t e = tid; e < TT; e += nth) s_A[e] = mv.m64(s_A[e], s_B[e]);
        __syncthreads();
    }

    if (MODE != BF_FWD)
        for (int i = 0; i < R; ++i)
            bf_bottom_layer(i, true, s_A, nullptr, l, R, H, s_mul8e, s_tab, s_basis, T, tid, nth);

    for (uint32_t e = tid; e < TT; e += nth) A[base + e] = s_A[e];
    __syncthreads();
}

// Bottom pass.  grid <= 2^(l-R) persistent workgroups over the tiles.
template <int MODE>
__global__ __launch_bounds__(BF_THREADS) void k_bfly_bottom(uint64_t *__restrict__ A, const uint64_t *__restrict__ B,
                                                            int l, int R, const DevTables *__restrict__ T)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, nth = blockDim.x;
    const uint64_t ntiles = 1ull << (l - R);
    bf_load_mul8_even(smem + BF_OFF_MUL8, T, tid, nth);
    for (uint64_t H = blockIdx.x; H < ntiles; H += gridDim.x) bf_bottom_tile<MODE>(A, B, l, R, H, smem, T, tid, nth);
}

static inline size_t bf_bottom_lds(int R, bool product)
{
    return BF_OFF_DATA + ((size_t)1 << R) * 8 * (product ? 2 : 1);
}


