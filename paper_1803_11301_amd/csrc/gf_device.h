// gf_device.h -- GF(2^64) arithmetic on gfx950 in the tower representation
// (bytes of GF(2^8) = V_8 in Cantor coordinates, towered by v_8, v_16, v_32;
// see consts_host.h).
//
// Multiplications the kernels use:
//   tmul  -- by a constant K through its 8-bit window table in LDS
//            (tab[k*256 + e] = K * (e at byte k)): 8 lookups, 7 XORs.
//   bmul  -- by an element beta of V_8: every byte is multiplied by beta on
//            its own (the tower is V_8-linear), one GF(2^8) table row.
//   gmul  -- general product (pointwise step of Alg. 5): Karatsuba over the
//            tower, 27 GF(2^8) products plus the three reductions
//            v_8^2 = v_8 + v_7, v_16^2 = v_16 + v_15, v_32^2 = v_32 + v_31.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

struct DevTables {
    uint64_t iota[8][256];       // Cantor vector -> tower element, by bytes
    uint64_t enc_win[8][256];    // Encode: byte window k of the bit column -> sum of r_j
    uint64_t dec_win[8][256];    // Decode: byte window k of the value -> bits
    uint64_t gbasis[32][64];     // v_{32+d} * unit_{8k+u}
    uint64_t pbasis[24][64];     // v_{8+v} * unit_{8k+u}
    uint8_t mul8[256][256];      // GF(2^8) products, Cantor coordinates
    uint16_t c15[2][256];        // v_15 * (byte at position p) in GF(2^16)
    uint32_t c31[4][256];        // v_31 * (byte at position p) in GF(2^32)
    // v_perm byte tables of beta = iota(2 bl), bl < 128, on the bit groups
    // {0,1,2}, {3,4,5}, {6,7} of a byte: t0lo t0hi t1lo t1hi t2 (3 words pad)
    uint32_t pt_beta8[128][8];
    uint32_t pt8[256][8];        // the same tables for every byte of V_8
    // m = 32 (GF(2^32), the low half of the tower representation)
    uint32_t enc32_win[4][256];  // Encode: byte window k of the 32-bit column -> sum of r_j
    uint32_t dec32_win[4][256];  // Decode: byte window k of the value -> bits
    uint32_t kt32[16][1024];     // window tables of v_{16+d}: [d][256 k + e] = v_{16+d} * (e at byte k)
    uint16_t mulp[256][256];     // GF(2^8) products with their v_7 multiples: p | (v_7 p) << 8, p = a b
    uint64_t sq_win[8][256];     // squares: byte window k of a value -> (e << 8k)^2
};

// ----------------------------------------------------------------- tmul ----

__device__ __forceinline__ uint64_t tmul(const uint64_t *__restrict__ tab, uint64_t x)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    uint64_t r0 = tab[lo & 255u] ^ tab[256 + ((lo >> 8) & 255u)];
    uint64_t r1 = tab[512 + ((lo >> 16) & 255u)] ^ tab[768 + (lo >> 24)];
    uint64_t r2 = tab[1024 + (hi & 255u)] ^ tab[1280 + ((hi >> 8) & 255u)];
    uint64_t r3 = tab[1536 + ((hi >> 16) & 255u)] ^ tab[1792 + (hi >> 24)];
    return (r0 ^ r1) ^ (r2 ^ r3);
}

// ----------------------------------------------------------------- bmul ----

// row = 256-byte GF(2^8) table row of beta
__device__ __forceinline__ uint64_t bmul(const uint8_t *__restrict__ row, uint64_t x)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    uint32_t a = (uint32_t)row[lo & 255u] | ((uint32_t)row[(lo >> 8) & 255u] << 8) |
                 ((uint32_t)row[(lo >> 16) & 255u] << 16) | ((uint32_t)row[lo >> 24] << 24);
    uint32_t b = (uint32_t)row[hi & 255u] | ((uint32_t)row[(hi >> 8) & 255u] << 8) |
                 ((uint32_t)row[(hi >> 16) & 255u] << 16) | ((uint32_t)row[hi >> 24] << 24);
    return (uint64_t)a | ((uint64_t)b << 32);
}

// ----------------------------------------------------------------- gmul ----

// LDS view of the full GF(2^8) table and the reduction tables, all at fixed
// offsets from one base: row a of the GF(2^8) table at
// (a & 1) * 32768 + (a >> 1) * 256 (even rows first, then odd rows), the
// v_15 table (u16[2][256]) at 65536 and the v_31 table (u32[4][256]) at 66560.
#define M8V_OFF_C15 65536
#define M8V_OFF_C31 (65536 + 1024)
#define M8V_BYTES (65536 + 1024 + 4096)
struct Mul8View {
    const uint8_t *base;
    __device__ __forceinline__ uint32_t m8(uint32_t a, uint32_t b) const
    {
        return base[((a & 1u) << 15) | ((a >> 1) << 8) | b];
    }
    __device__ __forceinline__ uint32_t m16(uint32_t a, uint32_t b) const
    {
        uint32_t a0 = a & 255u, a1 = a >> 8, b0 = b & 255u, b1 = b >> 8;
        uint32_t p0 = m8(a0, b0), p2 = m8(a1, b1), p1 = m8(a0 ^ a1, b0 ^ b1);
        uint32_t hi = p1 ^ p0, lo = p0 ^ m8(0x80u, p2);    // v_7 = Cantor byte 0x80
        return lo | (hi << 8);
    }
    __device__ __forceinline__ uint32_t mv15(uint32_t x) const
    {
        const uint16_t *c15 = reinterpret_cast<const uint16_t *>(base + M8V_OFF_C15);
        return c15[x & 255u] ^ c15[256 + (x >> 8)];
    }
    __device__ __forceinline__ uint32_t m32(uint32_t a, uint32_t b) const
    {
        uint32_t a0 = a & 0xFFFFu, a1 = a >> 16, b0 = b & 0xFFFFu, b1 = b >> 16;
        uint32_t p0 = m16(a0, b0), p2 = m16(a1, b1), p1 = m16(a0 ^ a1, b0 ^ b1);
        uint32_t hi = p1 ^ p0, lo = p0 ^ mv15(p2);
        return lo | (hi << 16);
    }
    __device__ __forceinline__ uint32_t mv31(uint32_t x) const
    {
        const uint32_t *c31 = reinterpret_cast<const uint32_t *>(base + M8V_OFF_C31);
        return c31[x & 255u] ^ c31[256 + ((x >> 8) & 255u)] ^ c31[512 + ((x >> 16) & 255u)] ^ c31[768 + (x >> 24)];
    }
    __device__ __forceinline__ uint64_t m64(uint64_t a, uint64_t b) const
    {
        uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
        uint32_t p0 = m32(a0, b0), p2 = m32(a1, b1), p1 = m32(a0 ^ a1, b0 ^ b1);
        uint32_t hi = p1 ^ p0, lo = p0 ^ mv31(p2);
        return (uint64_t)lo | ((uint64_t)hi << 32);
    }
};

// The same tower products from the pair table (DevTables::mulp) in LDS: a
// GF(2^16) product takes three lookups instead of four, the v_7 multiple of
// a1 b1 coming with it.  Layout: the pair table (128 KiB), then the v_15 and
// v_31 tables as in Mul8View.
#define MPV_OFF_C15 131072
#define MPV_OFF_C31 (131072 + 1024)
#define MPV_BYTES (131072 + 1024 + 4096)
struct MulPairView {
    const uint8_t *base;
    __device__ __forceinline__ uint32_t mp(uint32_t a, uint32_t b) const
    {
        return reinterpret_cast<const uint16_t *>(base)[(a << 8) | b];
    }
    __device__ __forceinline__ uint32_t m16(uint32_t a, uint32_t b) const
    {
        const uint32_t a0 = a & 255u, a1 = a >> 8, b0 = b & 255u, b1 = b >> 8;
        const uint32_t p0 = mp(a0, b0) & 255u, q2 = mp(a1, b1), p1 = mp(a0 ^ a1, b0 ^ b1) & 255u;
        const uint32_t hi = p1 ^ p0, lo = p0 ^ (q2 >> 8);   // q2 >> 8 = v_7 a1 b1
        return lo | (hi << 8);
    }
    __device__ __forceinline__ uint32_t mv15(uint32_t x) const
    {
        const uint16_t *c15 = reinterpret_cast<const uint16_t *>(base + MPV_OFF_C15);
        return c15[x & 255u] ^ c15[256 + (x >> 8)];
    }
    __device__ __forceinline__ uint32_t m32(uint32_t a, uint32_t b) const
    {
        uint32_t a0 = a & 0xFFFFu, a1 = a >> 16, b0 = b & 0xFFFFu, b1 = b >> 16;
        uint32_t p0 = m16(a0, b0), p2 = m16(a1, b1), p1 = m16(a0 ^ a1, b0 ^ b1);
        uint32_t hi = p1 ^ p0, lo = p0 ^ mv15(p2);
        return lo | (hi << 16);
    }
    __device__ __forceinline__ uint32_t mv31(uint32_t x) const
    {
        const uint32_t *c31 = reinterpret_cast<const uint32_t *>(base + MPV_OFF_C31);
        return c31[x & 255u] ^ c31[256 + ((x >> 8) & 255u)] ^ c31[512 + ((x >> 16) & 255u)] ^ c31[768 + (x >> 24)];
    }
    __device__ __forceinline__ uint64_t m64(uint64_t a, uint64_t b) const
    {
        uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
        uint32_t p0 = m32(a0, b0), p2 = m32(a1, b1), p1 = m32(a0 ^ a1, b0 ^ b1);
        uint32_t hi = p1 ^ p0, lo = p0 ^ mv31(p2);
        return (uint64_t)lo | ((uint64_t)hi << 32);
    }
};

// ------------------------------------------------------ K window tables ----
//
// Butterfly layer i of block b multiplies by the element with Cantor vector
// 2^(32+d) XOR 2b, d = l - i (Eq. 4 applied to the base points of Alg. 2).
// With b = bh * 128 + bl this is K + beta, K = Cantor(2^(32+d) XOR bh << 8)
// and beta = Cantor(2 bl) in V_8, so x * (K + beta) = tmul(T_K, x) ^ bmul(beta, x).
// T_K is built in LDS from its 64 basis images K * unit_{8k+u}, which are
// linear in bh: gbasis[d] XOR the pbasis rows of the set bits of bh.

// one thread per basis image (tid < 64); the 24 row loads are independent so
// they are all in flight together
__device__ __forceinline__ void ktable_basis(uint64_t *basis, int d, uint32_t bh, const DevTables *__restrict__ T,
                                             int tid)
{
    if (tid < 64) {
        uint64_t v = T->gbasis[d][tid];
#pragma unroll
        for (int b = 0; b < 24; ++b) {
            uint64_t r = T->pbasis[b][tid];
            v ^= ((bh >> b) & 1u) ? r : 0ull;
        }
        basis[tid] = v;
    }
}

// one work item = 8 entries of window k = item / 32: with m = item mod 32 the
// entry pairs 32 j + m, j < 4 (entries 64 j + 2 m and 64 j + 2 m + 1).  Work
// items m, m + 1 write adjacent 16-byte pairs, so the lanes of a wave store one
// contiguous run and the LDS writes are free of bank conflicts.
__device__ __forceinline__ void ktable_fill_item(uint64_t *tab, const uint64_t *basis, int item)
{
    const int k = item >> 5, m = item & 31;
    const uint64_t *bs = basis + 8 * k;
    uint64_t base = 0;
#pragma unroll
    for (int v = 0; v < 5; ++v)
        if ((m >> v) & 1) base ^= bs[1 + v];
    const uint64_t b0 = bs[0], b6 = bs[6], b7 = bs[7];
    ulonglong2 *t = reinterpret_cast<ulonglong2 *>(tab + k * 256) + m;
    const uint64_t c1 = base ^ b6, c2 = base ^ b7, c3 = c1 ^ b7;
    t[0] = make_ulonglong2(base, base ^ b0);
    t[32] = make_ulonglong2(c1, c1 ^ b0);
    t[64] = make_ulonglong2(c2, c2 ^ b0);
    t[96] = make_ulonglong2(c3, c3 ^ b0);
}
