// k_m128.h -- the m = 128 variant of the method (Sec. 3 with m = 128, l_m = 7;
// the field-size bound after Prop. 2 then allows transforms far beyond the
// 2^37 bits of m = 64).
//
// Field: GF(2^128) = GF(2^64)[y] / (y^2 + y + v_63), y = v_64 (the Cantor
// equation of v_64).  A value is two words (x0, x1) = x0 + x1 y, each half in
// the tower representation of gf_device.h, stored at words 2i and 2i + 1 of
// the transform buffer: n_p = n / 128 values take n bits, as for m = 64.
//
// Encode (Alg. 4, Eq. 9 with m = 128): row j of the m x n_p bit matrix goes
// to r_j = prod over set bits k of j (k < 7) of v_{64-k}.  Bit 0 of j selects
// v_64 = y, so r_j = y^(j & 1) P_{j >> 1} with P_t = prod over set bits k of t
// of v_{63-k} in GF(2^64): the even rows give the low half and the odd rows
// the high half, each through the same 64 x 64 map P.  Decode applies P^-1 to
// both halves and returns the bits to their rows.
//
// Butterfly (Alg. 2 at alpha = v_{l+64}): layer i, block b multiplies by the
// element with Cantor vector 2^(64+d) XOR 2b, d = l - i.  With
// v_{64+d} = L_d + H_d y and A = L_d + iota(2b) (2b < 2^63 stays in the low
// half):
//   (x0 + x1 y) (A + H_d y) = (x0 A + x1 (H_d v_63)) + ((x0 + x1) H_d + x1 A) y,
// two GF(2^64) products by A and two by the layer constants H_d and H_d v_63
// through their 8-bit window tables.
#pragma once

#include "gf_device.h"

#define M128_MAXD 64

struct DevTables128 {
    uint64_t enc_win[8][256];            // Encode: byte window k of a 64-row column -> sum of P_t
    uint64_t dec_win[8][256];            // Decode: byte window k of a half -> its 64 row bits
    uint64_t lo[M128_MAXD];              // L_d
    uint64_t ktab[M128_MAXD][2][2048];   // window tables of H_d and H_d v_63 (d = 0: 1 and v_63)
    uint64_t gbase[33][64];              // L_d unit_t (basis images of L_d), d <= 32
};

// the GF(2^8) table and the two reduction tables into LDS (Mul8View layout)
__device__ __forceinline__ void m128_load_mul8(uint8_t *s_m8, const DevTables *__restrict__ T, int tid, int nth)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(&T->mul8[0][0]);
    uint4 *dst = reinterpret_cast<uint4 *>(s_m8);
    for (int idx = tid; idx < 256 * 16; idx += nth) {
        const int a = idx >> 4, c = idx & 15;   // row a, 16-byte column c
        dst[((a & 1) << 11) | ((a >> 1) << 4) | c] = src[idx];
    }
    for (int q = tid; q < 512; q += nth) reinterpret_cast<uint16_t *>(s_m8 + M8V_OFF_C15)[q] = (&T->c15[0][0])[q];
    for (int q = tid; q < 1024; q += nth) reinterpret_cast<uint32_t *>(s_m8 + M8V_OFF_C31)[q] = (&T->c31[0][0])[q];
}

__device__ __forceinline__ uint64_t m128_win(const uint64_t (*__restrict__ win)[256], uint64_t x)
{
    uint64_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= win[k][(x >> (8 * k)) & 255u];
    return r;
}

// Encode: value i gathers bit i of each of the 128 rows of n_p bits
__global__ void k_encode128(const uint64_t *__restrict__ bits, int l, const DevTables128 *__restrict__ U,
                            uint64_t *__restrict__ vals)
{
    const uint64_t n_p = 1ull << l, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_p; i += stride) {
        uint64_t c0 = 0, c1 = 0;
        for (int t = 0; t < 64; ++t) {
            const uint64_t p0 = ((uint64_t)(2 * t) << l) + i, p1 = p0 + n_p;
            c0 |= ((bits[p0 >> 6] >> (p0 & 63)) & 1ull) << t;
            c1 |= ((bits[p1 >> 6] >> (p1 & 63)) & 1ull) << t;
        }
        vals[2 * i] = m128_win(U->enc_win, c0);
        vals[2 * i + 1] = m128_win(U->enc_win, c1);
    }
}

// The same with 64 x 64 bit transposes across the wave (l >= 9): one wave
// per 8 blocks of 64 consecutive values.  Lane t loads the words of rows 2t
// and 2t + 1 over those columns, each row as one 64-byte run; bit t of value
// k's halves is bit k of lane t's words, so the transposes of the even and
// the odd words give lane k its two columns.  Rows at or above nzrows are zero (the operand's bits end
// below nzrows n_p) and are not read.
#define M128_NB 8
__global__ __launch_bounds__(256) void k_encode128_w8(const uint64_t *__restrict__ bits, int l, int nzrows,
                                                      const DevTables128 *__restrict__ U, uint64_t *__restrict__ vals)
{
    __shared__ uint64_t s_win[8][256];
    for (int q = threadIdx.x; q < 8 * 256; q += blockDim.x) (&s_win[0][0])[q] = (&U->enc_win[0][0])[q];
    __syncthreads();
    const uint64_t rw = 1ull << (l - 6), ngrp = rw / M128_NB;
    const int lane = threadIdx.x & 63;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const bool le = 2 * lane < nzrows, lo = 2 * lane + 1 < nzrows;
    for (uint64_t grp = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; grp < ngrp; grp += nwaves) {
        const uint64_t b0 = grp * M128_NB;
        ulonglong2 we[M128_NB / 2], wo[M128_NB / 2];
        const ulonglong2 *re = reinterpret_cast<const ulonglong2 *>(bits + (uint64_t)(2 * lane) * rw + b0);
        const ulonglong2 *ro = reinterpret_cast<const ulonglong2 *>(bits + (uint64_t)(2 * lane + 1) * rw + b0);
#pragma unroll
        for (int h = 0; h < M128_NB / 2; ++h) {
            we[h] = le ? re[h] : make_ulonglong2(0, 0);
            wo[h] = lo ? ro[h] : make_ulonglong2(0, 0);
        }
#pragma unroll
        for (int bb = 0; bb < M128_NB; ++bb) {
            const uint64_t e = (bb & 1) ? we[bb / 2].y : we[bb / 2].x, o = (bb & 1) ? wo[bb / 2].y : wo[bb / 2].x;
            const uint64_t c0 = bc_wave_transpose64(e, lane), c1 = bc_wave_transpose64(o, lane);
            reinterpret_cast<ulonglong2 *>(vals)[(b0 + bb) * 64 + lane] =
                make_ulonglong2(m128_win(s_win, c0), m128_win(s_win, c1));
        }
    }
}

// Decode part 1: both halves of every value -> their row bits, in place
__global__ void k_decode128_vec(uint64_t *__restrict__ vals, uint64_t nwords, const DevTables128 *__restrict__ U)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride)
        vals[w] = m128_win(U->dec_win, vals[w]);
}

// Decode part 2: bit t of half e of value i is row 2t + e, column i
__global__ void k_decode128_scatter(const uint64_t *__restrict__ vecs, int l, uint64_t *__restrict__ bits)
{
    const uint64_t nw = 2ull << l, mask = (1ull << l) - 1, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t W = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; W < nw; W += stride) {
        uint64_t r = 0;
        for (int t = 0; t < 64; ++t) {
            const uint64_t p = 64 * W + t, j = p >> l, i = p & mask;
            r |= ((vecs[2 * i + (j & 1)] >> (j >> 1)) & 1ull) << t;
        }
        bits[W] = r;
    }
}

// Decode, both parts, with wave transposes (l >= 9): lane k holds value
// i0 + k of a block of 64; P^-1 on both halves, then the transpose of half e
// gives lane t the word of row 2t + e over the block's columns.  8 blocks per
// wave, so every row is written as one 64-byte run.
__global__ __launch_bounds__(256) void k_decode128_w8(const uint64_t *__restrict__ vecs, int l,
                                                      const DevTables128 *__restrict__ U, uint64_t *__restrict__ bits)
{
    __shared__ uint64_t s_win[8][256];
    for (int q = threadIdx.x; q < 8 * 256; q += blockDim.x) (&s_win[0][0])[q] = (&U->dec_win[0][0])[q];
    __syncthreads();
    const uint64_t rw = 1ull << (l - 6), ngrp = rw / M128_NB;
    const int lane = threadIdx.x & 63;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t grp = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; grp < ngrp; grp += nwaves) {
        const uint64_t b0 = grp * M128_NB;
        uint64_t r0[M128_NB], r1[M128_NB];
#pragma unroll
        for (int bb = 0; bb < M128_NB; ++bb) {
            const ulonglong2 v = reinterpret_cast<const ulonglong2 *>(vecs)[(b0 + bb) * 64 + lane];
            const ulonglong2 h = make_ulonglong2(m128_win(s_win, v.x), m128_win(s_win, v.y));
            r0[bb] = bc_wave_transpose64(h.x, lane);
            r1[bb] = bc_wave_transpose64(h.y, lane);
        }
        ulonglong2 *we = reinterpret_cast<ulonglong2 *>(bits + (uint64_t)(2 * lane) * rw + b0);
        ulonglong2 *wo = reinterpret_cast<ulonglong2 *>(bits + (uint64_t)(2 * lane + 1) * rw + b0);
#pragma unroll
        for (int h = 0; h < M128_NB / 2; ++h) {
            we[h] = make_ulonglong2(r0[2 * h], r0[2 * h + 1]);
            wo[h] = make_ulonglong2(r1[2 * h], r1[2 * h + 1]);
        }
    }
}

// x beta for beta in V_8, every byte by byte permutes (b2_pmul32 with the
// v_perm tables t01, t2 of beta) instead of GF(2^8) table lookups
__device__ __forceinline__ uint64_t m128_pmul(const uint4 &t01, uint32_t t2, uint64_t x)
{
    return (uint64_t)b2_pmul32(t01, t2, (uint32_t)x) | ((uint64_t)b2_pmul32(t01, t2, (uint32_t)(x >> 32)) << 32);
}

// forward butterfly on (u, v): u += c v, v += u; inverse: v += u, u += c v,
// for c = A + H_d y with A = K + beta (T_K = tk; beta's v_perm tables t01,
// t2), th / thv the window tables of H_d and H_d v_63:
// (x0 + x1 y)(A + H_d y) = (x0 A + x1 H_d v_63) + ((x0 + x1) H_d + x1 A) y
template <bool INV>
__device__ __forceinline__ void m128_bfly(const uint64_t *__restrict__ tk, const uint4 &t01, uint32_t t2,
                                          const uint64_t *__restrict__ th, const uint64_t *__restrict__ thv,
                                          ulonglong2 &u, ulonglong2 &v)
{
    if (INV) {
        v.x ^= u.x;
        v.y ^= u.y;
    }
    const uint64_t a0 = tmul(tk, v.x) ^ m128_pmul(t01, t2, v.x), a1 = tmul(tk, v.y) ^ m128_pmul(t01, t2, v.y);
    u.x ^= a0 ^ tmul(thv, v.y);
    u.y ^= tmul(th, v.x ^ v.y) ^ a1;
    if (!INV) {
        v.x ^= u.x;
        v.y ^= u.y;
    }
}

// One butterfly layer i of the transforms of A (and of B when given):
// forward h0 = p0 + c p1, h1 = h0 + p1; inverse p1 = h0 + h1, p0 = h0 + c p1.
// The pairs of both operands form one range of 1024-pair tiles, one pair per
// thread; each workgroup takes a contiguous run of tiles.
//
// The products by A = L_d + iota(2b) split as for m = 64: with b = 128 bh + bl,
// A = K + beta, K = L_d + iota(bh << 8) and beta = iota(2 bl) in V_8, so
// x A = tmul(T_K, x) + bmul(beta, x).  T_K is rebuilt in LDS whenever bh
// changes (every 2^(i+7) pairs) from its basis images K unit_t =
// L_d unit_t + the v_{8+v} unit_t of the set bits v of bh.  This needs a
// tile inside one block range of bh (i >= 3, whole tiles: l >= 11) and
// bh < 2^24 (d <= 32).  The layers below 3 split b at bit 11 instead:
// beta = iota(2 (b mod 2^11)) lies in V_16 and is applied as
// beta0 x + beta1 (x v_8) with byte permutes.  Transforms with l < 11 or
// d > 32 take general products by A.
#define M128_TILE 1024

template <bool INV>
__global__ __launch_bounds__(1024) void k_bfly128_layer(uint64_t *__restrict__ A, uint64_t *__restrict__ B, int l,
                                                        int i, const DevTables *__restrict__ T,
                                                        const DevTables128 *__restrict__ U)
{
    __shared__ __align__(16) uint8_t s_m8[M8V_BYTES];
    __shared__ __align__(16) uint64_t s_tab[2][2048];
    __shared__ __align__(16) uint64_t s_k[2048];
    __shared__ __align__(16) uint32_t s_pt8[256][8];
    __shared__ uint64_t s_img[64];
    const int tid = threadIdx.x, nth = blockDim.x, d = l - i;
    m128_load_mul8(s_m8, T, tid, nth);
    for (int q = tid; q < 2 * 2048; q += nth) (&s_tab[0][0])[q] = (&U->ktab[d][0][0])[q];
    for (int q = tid; q < 256 * 8; q += nth) (&s_pt8[0][0])[q] = (&T->pt8[0][0])[q];
    __syncthreads();
    const Mul8View mv{s_m8};
    const uint64_t Ld = U->lo[d];
    const uint64_t half = 1ull << (l - 1), total = B ? 2 * half : half, omask = (1ull << i) - 1;
    // tabled: K from the bits of b above 7 (beta in V_8); for i < 3 a tile
    // spans more than 128 blocks, so K takes the bits above 11 and beta the
    // 12-bit rest, an element of V_16 applied as beta0 x + beta1 (x v_8)
    const bool tabled = l >= 11 && d <= 32;
    const int kshift = i >= 3 ? 7 : 11;
    const uint64_t ntiles = (total + M128_TILE - 1) / M128_TILE;
    const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t_end = min(ntiles, (uint64_t)(blockIdx.x + 1) * per);
    uint64_t key = ~0ull;
    for (uint64_t tile = (uint64_t)blockIdx.x * per; tile < t_end; ++tile) {
        if (tabled) {
            const uint64_t bh = ((tile * M128_TILE) & (half - 1)) >> (i + kshift);
            if (bh != key) {   // uniform: one tile lies in one block range of bh
                __syncthreads();   // the previous tile is done with T_K
                if (tid < 64) {
                    // K = L_d + iota(bh << (kshift + 1)); pbasis[k] is v_{8+k} unit_t
                    const int off = kshift - 7;
                    uint64_t v = U->gbase[d][tid];
                    for (int k = 0; k + off < 24; ++k) v ^= ((bh >> k) & 1u) ? T->pbasis[k + off][tid] : 0ull;
                    s_img[tid] = v;
                }
                __syncthreads();
                if (tid < 256) ktable_fill_item(s_k, s_img, tid);
                __syncthreads();
                key = bh;
            }
        }
        const uint64_t q = tile * M128_TILE + tid;
        if (q >= total) continue;
        uint64_t *X = q < half ? A : B;
        const uint64_t r = q & (half - 1), b = r >> i;
        const uint64_t j0 = (b << (i + 1)) | (r & omask), j1 = j0 + (1ull << i);
        const ulonglong2 u = reinterpret_cast<const ulonglong2 *>(X)[j0];
        const ulonglong2 v = reinterpret_cast<const ulonglong2 *>(X)[j1];
        uint64_t x0, x1;
        if (!INV) {
            x0 = v.x;
            x1 = v.y;
        } else {
            x0 = u.x ^ v.x;
            x1 = u.y ^ v.y;
        }
        uint64_t a0, a1;   // x0 A, x1 A
        if (tabled && i >= 3) {
            const uint8_t *row = s_m8 + ((b & 127u) << 8);   // GF(2^8) row of beta = 2 bl (even)
            a0 = tmul(s_k, x0) ^ bmul(row, x0);
            a1 = tmul(s_k, x1) ^ bmul(row, x1);
        } else if (tabled) {
            const uint64_t cb = 2 * (b & 2047u);   // beta = iota(cb), cb < 2^12: V_16
            const uint32_t b16 = (uint32_t)(T->iota[0][cb & 255u] ^ T->iota[1][cb >> 8]);
            const uint4 p0 = *reinterpret_cast<const uint4 *>(s_pt8[b16 & 255u]);
            const uint4 p1 = *reinterpret_cast<const uint4 *>(s_pt8[b16 >> 8]);
            const uint32_t p02 = s_pt8[b16 & 255u][4], p12 = s_pt8[b16 >> 8][4];
            const uint32_t bc = (p12 >> 16) & 255u;   // beta1 v_7
            const uint4 pc = *reinterpret_cast<const uint4 *>(s_pt8[bc]);
            const uint32_t pc2 = s_pt8[bc][4];
            auto mul16 = [&](uint64_t x) {
                const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
                const uint32_t rl = b2_mulv16(p0, p02, p1, p12, pc, pc2, lo);
                const uint32_t rh = b2_mulv16(p0, p02, p1, p12, pc, pc2, hi);
                return (uint64_t)rl | ((uint64_t)rh << 32);
            };
            a0 = tmul(s_k, x0) ^ mul16(x0);
            a1 = tmul(s_k, x1) ^ mul16(x1);
        } else {
            const uint64_t cb = 2 * b;
            uint64_t Ab = Ld;
#pragma unroll
            for (int k = 0; k < 8; ++k) Ab ^= T->iota[k][(cb >> (8 * k)) & 255u];
            a0 = mv.m64(x0, Ab);
            a1 = mv.m64(x1, Ab);
        }
        // (x0 + x1 y)(A + H_d y) = (x0 A + x1 H_d v_63) + ((x0 + x1) H_d + x1 A) y
        const uint64_t m0 = a0 ^ tmul(s_tab[1], x1), m1 = tmul(s_tab[0], x0 ^ x1) ^ a1;
        if (!INV) {
            const uint64_t h0 = u.x ^ m0, h1 = u.y ^ m1;
            reinterpret_cast<ulonglong2 *>(X)[j0] = make_ulonglong2(h0, h1);
            reinterpret_cast<ulonglong2 *>(X)[j1] = make_ulonglong2(h0 ^ v.x, h1 ^ v.y);
        } else {
            reinterpret_cast<ulonglong2 *>(X)[j0] = make_ulonglong2(u.x ^ m0, u.y ^ m1);
            reinterpret_cast<ulonglong2 *>(X)[j1] = make_ulonglong2(x0, x1);
        }
    }
}

// Layers i + 1 and i in one pass (forward: i + 1 first), one group of four
// values j + k 2^i (k < 4) per thread.  Layer i + 1 pairs (0, 2) and (1, 3) in
// block b1 = j >> (i + 2); layer i pairs (0, 1) in block 2 b1 and (2, 3) in
// block 2 b1 + 1, which share K (2 b1 is even) and differ in beta by 2.
// With 512 groups per tile (one per thread) both K keys are uniform over a
// tile when i >= 3; needs l >= 11 (whole tiles) and d = l - i <= 32.  512
// threads keep the four values and the products in registers (256 VGPRs).
// LDS: the v_perm tables of
// the betas, the window tables of H and H v_63 of both layers and the two K
// tables.
#define M128_TILE2 512

template <bool INV>
__global__ __launch_bounds__(M128_TILE2) void k_bfly128_2layer(uint64_t *__restrict__ A, uint64_t *__restrict__ B, int l,
                                                         int i, const DevTables *__restrict__ T,
                                                         const DevTables128 *__restrict__ U)
{
    __shared__ __align__(16) uint32_t s_ptb[128][8];
    __shared__ __align__(16) uint64_t s_h[4][2048];
    __shared__ __align__(16) uint64_t s_k[2][2048];
    __shared__ uint64_t s_img[2][64];
    const int tid = threadIdx.x, nth = blockDim.x, d0 = l - i, d1 = d0 - 1;
    {
        for (int q = tid; q < 128 * 8; q += nth) (&s_ptb[0][0])[q] = (&T->pt_beta8[0][0])[q];
        for (int q = tid; q < 2 * 2048; q += nth) {
            (&s_h[0][0])[q] = (&U->ktab[d1][0][0])[q];
            (&s_h[2][0])[q] = (&U->ktab[d0][0][0])[q];
        }
    }
    __syncthreads();
    const uint64_t quarter = 1ull << (l - 2), total = B ? 2 * quarter : quarter, imask = (1ull << i) - 1;
    const uint64_t ntiles = total / M128_TILE2, per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t_end = min(ntiles, (uint64_t)(blockIdx.x + 1) * per);
    uint64_t key1 = ~0ull, key0 = ~0ull;
    // group of this thread in a tile: operand, first value j, block b1
    auto where = [&](uint64_t tile, ulonglong2 *&P, uint64_t &j, uint64_t &b1) {
        const uint64_t q = tile * M128_TILE2 + tid, g = q & (quarter - 1);
        P = reinterpret_cast<ulonglong2 *>(q < quarter ? A : B);
        b1 = g >> i;
        j = (b1 << (i + 2)) | (g & imask);
    };
    const uint64_t s = 1ull << i;
    uint64_t tile = (uint64_t)blockIdx.x * per;
    ulonglong2 *P = nullptr;
    uint64_t j = 0, b1 = 0;
    ulonglong2 x0{}, x1{}, x2{}, x3{};
    if (tile < t_end) {
        where(tile, P, j, b1);
        x0 = P[j], x1 = P[j + s], x2 = P[j + 2 * s], x3 = P[j + 3 * s];
    }
    for (; tile < t_end; ++tile) {
        // the next tile's values are loaded while this one computes
        ulonglong2 *Pn = P;
        uint64_t jn = j, b1n = b1;
        ulonglong2 y0{}, y1{}, y2{}, y3{};
        if (tile + 1 < t_end) {
            where(tile + 1, Pn, jn, b1n);
            y0 = Pn[jn], y1 = Pn[jn + s], y2 = Pn[jn + 2 * s], y3 = Pn[jn + 3 * s];
        }
        const uint64_t g0 = (tile * M128_TILE2) & (quarter - 1);
        const uint64_t bh1 = g0 >> (i + 7), bh0 = g0 >> (i + 6);
        if (bh1 != key1 || bh0 != key0) {   // uniform over the tile
            __syncthreads();   // the previous tile is done with the K tables
            if (tid < 128) {
                const int t = tid & 63, which = tid >> 6;
                const uint64_t bh = which ? bh0 : bh1;
                uint64_t v = U->gbase[which ? d0 : d1][t];
#pragma unroll
                for (int k = 0; k < 24; ++k) v ^= ((bh >> k) & 1u) ? T->pbasis[k][t] : 0ull;
                s_img[which][t] = v;
            }
            __syncthreads();
            for (int it = tid; it < 512; it += nth) ktable_fill_item(s_k[it >> 8], s_img[it >> 8], it & 255);
            __syncthreads();
            key1 = bh1;
            key0 = bh0;
        }
        const int r1 = (int)(b1 & 127u), r0 = (int)((2 * b1) & 127u);   // beta = 2 r (r0 even)
        const uint4 p1 = *reinterpret_cast<const uint4 *>(s_ptb[r1]);
        const uint4 p0a = *reinterpret_cast<const uint4 *>(s_ptb[r0]);
        const uint4 p0b = *reinterpret_cast<const uint4 *>(s_ptb[r0 + 1]);
        const uint32_t p1e = s_ptb[r1][4], p0ae = s_ptb[r0][4], p0be = s_ptb[r0 + 1][4];
        if (!INV) {
            m128_bfly<false>(s_k[0], p1, p1e, s_h[0], s_h[1], x0, x2);
            m128_bfly<false>(s_k[0], p1, p1e, s_h[0], s_h[1], x1, x3);
            m128_bfly<false>(s_k[1], p0a, p0ae, s_h[2], s_h[3], x0, x1);
            m128_bfly<false>(s_k[1], p0b, p0be, s_h[2], s_h[3], x2, x3);
        } else {
            m128_bfly<true>(s_k[1], p0a, p0ae, s_h[2], s_h[3], x0, x1);
            m128_bfly<true>(s_k[1], p0b, p0be, s_h[2], s_h[3], x2, x3);
            m128_bfly<true>(s_k[0], p1, p1e, s_h[0], s_h[1], x0, x2);
            m128_bfly<true>(s_k[0], p1, p1e, s_h[0], s_h[1], x1, x3);
        }
        P[j] = x0;
        P[j + s] = x1;
        P[j + 2 * s] = x2;
        P[j + 3 * s] = x3;
        P = Pn;
        j = jn;
        b1 = b1n;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
}

// Layers i + 2, i + 1 and i in one pass (forward: i + 2 first), eight values
// j0 + k 2^i (k < 8) per thread, 512 threads.  Layer i + 2 pairs (k, k + 4) in
// block b = j0 >> (i + 3); layer i + 1 pairs (k, k + 2) in blocks 2b and
// 2b + 1; layer i pairs (k, k + 1) in blocks 4b .. 4b + 3.  K and beta as in
// the two-layer pass (beta in V_8 by byte permutes); the three K keys are
// uniform over a tile of 512 groups when i >= 4.  Needs l >= 12 and
// d = l - i <= 32.
template <bool INV>
__global__ __launch_bounds__(M128_TILE2) void k_bfly128_3layer(uint64_t *__restrict__ A, uint64_t *__restrict__ B, int l,
                                                               int i, const DevTables *__restrict__ T,
                                                               const DevTables128 *__restrict__ U)
{
    __shared__ __align__(16) uint32_t s_ptb[128][8];
    __shared__ __align__(16) uint64_t s_h[3][2][2048];   // [m] tables of H, H v_63 of layer i + m
    __shared__ __align__(16) uint64_t s_k[3][2048];      // [m] T_K of layer i + m
    __shared__ uint64_t s_img[3][64];
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int q = tid; q < 128 * 8; q += nth) (&s_ptb[0][0])[q] = (&T->pt_beta8[0][0])[q];
    for (int q = tid; q < 3 * 2 * 2048; q += nth) {
        const int m = q / 4096, r = q - m * 4096;
        (&s_h[m][0][0])[r] = (&U->ktab[l - i - m][0][0])[r];
    }
    __syncthreads();
    const uint64_t eighth = 1ull << (l - 3), total = B ? 2 * eighth : eighth, imask = (1ull << i) - 1;
    const uint64_t ntiles = total / M128_TILE2, per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t_end = min(ntiles, (uint64_t)(blockIdx.x + 1) * per);
    uint64_t key[3] = {~0ull, ~0ull, ~0ull};
    for (uint64_t tile = (uint64_t)blockIdx.x * per; tile < t_end; ++tile) {
        const uint64_t g0 = (tile * M128_TILE2) & (eighth - 1);
        // bh of layer i + m: (block >> 7) with block = (g >> i) << (2 - m) (+ lower bits)
        bool changed = false;
#pragma unroll
        for (int m = 0; m < 3; ++m) changed |= (g0 >> (i + 5 + m)) != key[m];
        if (changed) {   // uniform over the tile
            __syncthreads();   // the previous tile is done with the K tables
            if (tid < 192) {
                const int m = tid >> 6, t = tid & 63;
                const uint64_t bh = g0 >> (i + 5 + m);
                uint64_t v = U->gbase[l - i - m][t];
#pragma unroll
                for (int k = 0; k < 24; ++k) v ^= ((bh >> k) & 1u) ? T->pbasis[k][t] : 0ull;
                s_img[m][t] = v;
            }
            __syncthreads();
            for (int it = tid; it < 3 * 256; it += nth) ktable_fill_item(s_k[it >> 8], s_img[it >> 8], it & 255);
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 3; ++m) key[m] = g0 >> (i + 5 + m);
        }
        const uint64_t q = tile * M128_TILE2 + tid;
        ulonglong2 *P = reinterpret_cast<ulonglong2 *>(q < eighth ? A : B);
        const uint64_t g = q & (eighth - 1), b = g >> i;
        const uint64_t j0 = (b << (i + 3)) | (g & imask), s = 1ull << i;
        ulonglong2 x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = P[j0 + k * s];
        const int r2 = (int)(b & 127u), r1 = (int)((2 * b) & 127u), r0 = (int)((4 * b) & 127u);
        auto pt = [&](int r, uint4 &t01, uint32_t &t2) {
            t01 = *reinterpret_cast<const uint4 *>(s_ptb[r]);
            t2 = s_ptb[r][4];
        };
        uint4 p2, p1a, p1b, p0a, p0b, p0c, p0d;
        uint32_t e2, e1a, e1b, e0a, e0b, e0c, e0d;
        pt(r2, p2, e2);
        pt(r1, p1a, e1a);
        pt(r1 + 1, p1b, e1b);
        pt(r0, p0a, e0a);
        pt(r0 + 1, p0b, e0b);
        pt(r0 + 2, p0c, e0c);
        pt(r0 + 3, p0d, e0d);
        if (!INV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) m128_bfly<false>(s_k[2], p2, e2, s_h[2][0], s_h[2][1], x[k], x[k + 4]);
            m128_bfly<false>(s_k[1], p1a, e1a, s_h[1][0], s_h[1][1], x[0], x[2]);
            m128_bfly<false>(s_k[1], p1a, e1a, s_h[1][0], s_h[1][1], x[1], x[3]);
            m128_bfly<false>(s_k[1], p1b, e1b, s_h[1][0], s_h[1][1], x[4], x[6]);
            m128_bfly<false>(s_k[1], p1b, e1b, s_h[1][0], s_h[1][1], x[5], x[7]);
            m128_bfly<false>(s_k[0], p0a, e0a, s_h[0][0], s_h[0][1], x[0], x[1]);
            m128_bfly<false>(s_k[0], p0b, e0b, s_h[0][0], s_h[0][1], x[2], x[3]);
            m128_bfly<false>(s_k[0], p0c, e0c, s_h[0][0], s_h[0][1], x[4], x[5]);
            m128_bfly<false>(s_k[0], p0d, e0d, s_h[0][0], s_h[0][1], x[6], x[7]);
        } else {
            m128_bfly<true>(s_k[0], p0a, e0a, s_h[0][0], s_h[0][1], x[0], x[1]);
            m128_bfly<true>(s_k[0], p0b, e0b, s_h[0][0], s_h[0][1], x[2], x[3]);
            m128_bfly<true>(s_k[0], p0c, e0c, s_h[0][0], s_h[0][1], x[4], x[5]);
            m128_bfly<true>(s_k[0], p0d, e0d, s_h[0][0], s_h[0][1], x[6], x[7]);
            m128_bfly<true>(s_k[1], p1a, e1a, s_h[1][0], s_h[1][1], x[0], x[2]);
            m128_bfly<true>(s_k[1], p1a, e1a, s_h[1][0], s_h[1][1], x[1], x[3]);
            m128_bfly<true>(s_k[1], p1b, e1b, s_h[1][0], s_h[1][1], x[4], x[6]);
            m128_bfly<true>(s_k[1], p1b, e1b, s_h[1][0], s_h[1][1], x[5], x[7]);
#pragma unroll
            for (int k = 0; k < 4; ++k) m128_bfly<true>(s_k[2], p2, e2, s_h[2][0], s_h[2][1], x[k], x[k + 4]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) P[j0 + k * s] = x[k];
    }
}

// Layers 2, 1 and 0 in one pass (forward: 2 first), eight consecutive values
// j0 + e (e < 8, j0 = 8 g) per thread, 512 threads: layer 2 pairs (e, e + 4)
// in block g, layer 1 pairs (e, e + 2) in blocks 2g and 2g + 1, layer 0 pairs
// (e, e + 1) in blocks 4g .. 4g + 3.  Each layer splits its block index b at
// bit 11 as k_bfly128_layer does below layer 3: K = L_d + iota((b >> 11) << 12)
// from a window table rebuilt when a 4096-value tile starts a new range of
// b >> 11, and beta = iota(2 (b mod 2^11)) in V_16 by byte permutes.  Needs
// l >= 12 (whole tiles) and d = l <= 32.
#define M128_LOW_THREADS 512

// x (K + beta16) with T_K = tk, beta16 = beta0 + beta1 v_8 given by the v_perm
// tables (p0, p02) of beta0, (p1, p12) of beta1 and (pc, pc2) of beta1 v_7
__device__ __forceinline__ uint64_t m128_kb16(const uint64_t *__restrict__ tk, const uint4 &p0, uint32_t p02,
                                              const uint4 &p1, uint32_t p12, const uint4 &pc, uint32_t pc2,
                                              uint64_t x)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint32_t rl = b2_mulv16(p0, p02, p1, p12, pc, pc2, lo);
    const uint32_t rh = b2_mulv16(p0, p02, p1, p12, pc, pc2, hi);
    return tmul(tk, x) ^ ((uint64_t)rl | ((uint64_t)rh << 32));
}

template <bool INV>
__device__ __forceinline__ void m128_bfly16(const uint64_t *__restrict__ tk, const uint32_t (*__restrict__ pt8)[8],
                                            uint32_t b16, const uint64_t *__restrict__ th,
                                            const uint64_t *__restrict__ thv, ulonglong2 &u, ulonglong2 &v)
{
    const uint4 p0 = *reinterpret_cast<const uint4 *>(pt8[b16 & 255u]);
    const uint4 p1 = *reinterpret_cast<const uint4 *>(pt8[b16 >> 8]);
    const uint32_t p02 = pt8[b16 & 255u][4], p12 = pt8[b16 >> 8][4];
    const uint32_t bc = (p12 >> 16) & 255u;   // beta1 v_7: entry 2 of beta1's bit-6/7 table
    const uint4 pc = *reinterpret_cast<const uint4 *>(pt8[bc]);
    const uint32_t pc2 = pt8[bc][4];
    if (INV) {
        v.x ^= u.x;
        v.y ^= u.y;
    }
    const uint64_t a0 = m128_kb16(tk, p0, p02, p1, p12, pc, pc2, v.x);
    const uint64_t a1 = m128_kb16(tk, p0, p02, p1, p12, pc, pc2, v.y);
    u.x ^= a0 ^ tmul(thv, v.y);
    u.y ^= tmul(th, v.x ^ v.y) ^ a1;
    if (!INV) {
        v.x ^= u.x;
        v.y ^= u.y;
    }
}

template <bool INV>
__global__ __launch_bounds__(M128_LOW_THREADS) void k_bfly128_low3(uint64_t *__restrict__ A, uint64_t *__restrict__ B,
                                                                   int l, const DevTables *__restrict__ T,
                                                                   const DevTables128 *__restrict__ U)
{
    __shared__ __align__(16) uint64_t s_h[3][2][2048];   // [i] window tables of H_{l-i}, H_{l-i} v_63
    __shared__ __align__(16) uint64_t s_k[3][2048];      // [i] T_K of layer i
    __shared__ __align__(16) uint32_t s_pt8[256][8];
    __shared__ uint64_t s_img[3][64];
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int q = tid; q < 3 * 2 * 2048; q += nth) {
        const int i = q / 4096, r = q - i * 4096;
        (&s_h[i][0][0])[r] = (&U->ktab[l - i][0][0])[r];
    }
    for (int q = tid; q < 256 * 8; q += nth) (&s_pt8[0][0])[q] = (&T->pt8[0][0])[q];
    __syncthreads();
    const uint64_t quarter8 = 1ull << (l - 3);   // groups of 8 per operand
    const uint64_t total = B ? 2 * quarter8 : quarter8;
    const uint64_t ntiles = total / M128_LOW_THREADS, per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t_end = min(ntiles, (uint64_t)(blockIdx.x + 1) * per);
    uint64_t key[3] = {~0ull, ~0ull, ~0ull};
    for (uint64_t tile = (uint64_t)blockIdx.x * per; tile < t_end; ++tile) {
        const uint64_t j00 = ((tile * M128_LOW_THREADS) & (quarter8 - 1)) << 3;   // tile's first value
        bool changed = false;
#pragma unroll
        for (int i = 0; i < 3; ++i) changed |= (j00 >> (i + 12)) != key[i];
        if (changed) {   // uniform over the tile
            __syncthreads();   // the previous tile is done with the K tables
            if (tid < 192) {
                const int i = tid >> 6, t = tid & 63;
                const uint64_t bh = j00 >> (i + 12);   // (b >> 11) for b = j >> (i + 1)
                uint64_t v = U->gbase[l - i][t];
                for (int k = 0; k < 20; ++k) v ^= ((bh >> k) & 1u) ? T->pbasis[k + 4][t] : 0ull;
                s_img[i][t] = v;
            }
            __syncthreads();
            for (int it = tid; it < 3 * 256; it += nth) ktable_fill_item(s_k[it >> 8], s_img[it >> 8], it & 255);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 3; ++i) key[i] = j00 >> (i + 12);
        }
        const uint64_t q = tile * M128_LOW_THREADS + tid;
        ulonglong2 *P = reinterpret_cast<ulonglong2 *>(q < quarter8 ? A : B);
        const uint64_t g = q & (quarter8 - 1), j0 = g << 3;
        ulonglong2 x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = P[j0 + e];
        // beta of block b at layer i: iota(2 (b mod 2^11)), a V_16 element
        auto beta = [&](uint64_t b) {
            const uint32_t cb = (uint32_t)(2 * (b & 2047u));
            return (uint32_t)(T->iota[0][cb & 255u] ^ T->iota[1][cb >> 8]);
        };
        const uint32_t b2 = beta(g), b1a = beta(2 * g), b1b = beta(2 * g + 1);
        const uint32_t b0a = beta(4 * g), b0b = beta(4 * g + 1), b0c = beta(4 * g + 2), b0d = beta(4 * g + 3);
        if (!INV) {
#pragma unroll
            for (int e = 0; e < 4; ++e) m128_bfly16<false>(s_k[2], s_pt8, b2, s_h[2][0], s_h[2][1], x[e], x[e + 4]);
            m128_bfly16<false>(s_k[1], s_pt8, b1a, s_h[1][0], s_h[1][1], x[0], x[2]);
            m128_bfly16<false>(s_k[1], s_pt8, b1a, s_h[1][0], s_h[1][1], x[1], x[3]);
            m128_bfly16<false>(s_k[1], s_pt8, b1b, s_h[1][0], s_h[1][1], x[4], x[6]);
            m128_bfly16<false>(s_k[1], s_pt8, b1b, s_h[1][0], s_h[1][1], x[5], x[7]);
            m128_bfly16<false>(s_k[0], s_pt8, b0a, s_h[0][0], s_h[0][1], x[0], x[1]);
            m128_bfly16<false>(s_k[0], s_pt8, b0b, s_h[0][0], s_h[0][1], x[2], x[3]);
            m128_bfly16<false>(s_k[0], s_pt8, b0c, s_h[0][0], s_h[0][1], x[4], x[5]);
            m128_bfly16<false>(s_k[0], s_pt8, b0d, s_h[0][0], s_h[0][1], x[6], x[7]);
        } else {
            m128_bfly16<true>(s_k[0], s_pt8, b0a, s_h[0][0], s_h[0][1], x[0], x[1]);
            m128_bfly16<true>(s_k[0], s_pt8, b0b, s_h[0][0], s_h[0][1], x[2], x[3]);
            m128_bfly16<true>(s_k[0], s_pt8, b0c, s_h[0][0], s_h[0][1], x[4], x[5]);
            m128_bfly16<true>(s_k[0], s_pt8, b0d, s_h[0][0], s_h[0][1], x[6], x[7]);
            m128_bfly16<true>(s_k[1], s_pt8, b1a, s_h[1][0], s_h[1][1], x[0], x[2]);
            m128_bfly16<true>(s_k[1], s_pt8, b1a, s_h[1][0], s_h[1][1], x[1], x[3]);
            m128_bfly16<true>(s_k[1], s_pt8, b1b, s_h[1][0], s_h[1][1], x[4], x[6]);
            m128_bfly16<true>(s_k[1], s_pt8, b1b, s_h[1][0], s_h[1][1], x[5], x[7]);
#pragma unroll
            for (int e = 0; e < 4; ++e) m128_bfly16<true>(s_k[2], s_pt8, b2, s_h[2][0], s_h[2][1], x[e], x[e + 4]);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) P[j0 + e] = x[e];
    }
}

// A[j] = A[j] B[j] over GF(2^128) (Alg. 5, the pointwise step)
__global__ __launch_bounds__(1024) void k_pointwise128(uint64_t *__restrict__ A, const uint64_t *__restrict__ B,
                                                       uint64_t n_p, const DevTables *__restrict__ T,
                                                       const DevTables128 *__restrict__ U)
{
    __shared__ __align__(16) uint8_t s_m8[M8V_BYTES];
    __shared__ __align__(16) uint64_t s_v63[2048];   // window table of v_63 (H_0 v_63, H_0 = 1)
    const int tid = threadIdx.x, nth = blockDim.x;
    m128_load_mul8(s_m8, T, tid, nth);
    for (int q = tid; q < 2048; q += nth) s_v63[q] = U->ktab[0][1][q];
    __syncthreads();
    const Mul8View mv{s_m8};
    const uint64_t stride = (uint64_t)gridDim.x * nth;
    for (uint64_t j = (uint64_t)blockIdx.x * nth + tid; j < n_p; j += stride) {
        const ulonglong2 a = reinterpret_cast<const ulonglong2 *>(A)[j];
        const ulonglong2 b = reinterpret_cast<const ulonglong2 *>(B)[j];
        const uint64_t p0 = mv.m64(a.x, b.x), p2 = mv.m64(a.y, b.y), p1 = mv.m64(a.x ^ a.y, b.x ^ b.y);
        reinterpret_cast<ulonglong2 *>(A)[j] = make_ulonglong2(p0 ^ tmul(s_v63, p2), p1 ^ p0);
    }
}
