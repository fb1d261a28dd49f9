// k_batch.h -- many independent products (Alg. 5 each) in one persistent launch.
//
// Each workgroup takes whole products from a size-sorted queue and runs
// every step of FP_Polymul for that product on its own slab of device
// memory: BasisCvt (Alg. 1) of both operands as Taylor steps, Encode (Alg. 4,
// Eq. 9) through 64 x 64 wave transposes, the butterfly layers above the
// bottom tile streamed through the slab (Alg. 2), the bottom tiles with the
// pointwise products fused (the bottom pass of k_butterfly.h), the inverse
// layers, Decode and the inverse BasisCvt.  The transform depth l of every
// product is computed on the device from its two lengths.
#pragma once

#include "gf_device.h"
#include "k_basiscvt.h"
#include "k_bf2.h"
#include "k_butterfly.h"
#include "k_steps.h"

#define BT_THREADS 1024
#define BT_MAX_LOG2N 22      // largest transform of a batch item: 2^22 bits (products below 2^22 bits)
#define BT_MIN_LOG2N 6
#define BT_MAX_STEPS 1024    // BasisCvt steps of all sizes 2^6 .. 2^22 together
#define BT_NBINS (BT_MAX_LOG2N - BT_MIN_LOG2N + 2)

// layers above the bottom tile must share one K table (block index < 128)
static_assert(BT_MAX_LOG2N - 6 - BF_BOTTOM_R <= 7, "upper batch layers need one K table per layer");

// Taylor steps of BasisCvt(2^k) for k in [6, 22]: entries first[k] .. first[k] + count[k] - 1
struct BatchStep {
    uint64_t S, d;   // segment length and shift in bits
    uint64_t L, D;   // for S <= 64: low-half and low-d masks of every segment in a word
};
struct BatchSteps {
    int first[BT_MAX_LOG2N + 1];
    int count[BT_MAX_LOG2N + 1];
    BatchStep st[BT_MAX_STEPS];
};

// one item given by pointers (the server's batched launches) instead of pool
// offsets
struct BtDesc {
    const uint64_t *a, *b;
    uint64_t *out;
    uint64_t la, lb;
};

// writes a descriptor passed by value (a single product through the batch path)
__global__ void k_bt_put_desc(BtDesc d, BtDesc *__restrict__ dst)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
}

__device__ __forceinline__ int bt_ceil_log2(uint64_t x) { return x <= 1 ? 0 : 64 - __clzll(x - 1); }

// transform log2 of a product, or -1 if it has no bits, or BT_MAX_LOG2N + 1
// if it is longer than max_bits
__device__ __forceinline__ int bt_log2n(uint64_t la, uint64_t lb, uint64_t max_bits)
{
    if (la == 0 || lb == 0) return -1;
    if (la > max_bits || lb > max_bits || la + lb - 1 > max_bits) return BT_MAX_LOG2N + 1;
    const int k = bt_ceil_log2(la + lb - 1);
    return k < BT_MIN_LOG2N ? BT_MIN_LOG2N : k;
}

// lengths of item q: from the descriptors when given, else from the arrays
__device__ __forceinline__ void bt_lengths(const BtDesc *desc, const uint64_t *len_a, const uint64_t *len_b,
                                           uint32_t q, uint64_t &la, uint64_t &lb)
{
    if (desc) {
        la = desc[q].la;
        lb = desc[q].lb;
    } else {
        la = len_a[q];
        lb = len_b[q];
    }
}

// queue order: larger transforms first, empty and rejected items last; also
// resets the queue counter.  One workgroup.
__global__ __launch_bounds__(1024) void k_batch_plan(uint32_t count, const uint64_t *__restrict__ len_a,
                                                     const uint64_t *__restrict__ len_b,
                                                     const BtDesc *__restrict__ desc, uint64_t max_bits,
                                                     uint32_t *__restrict__ order, uint32_t *__restrict__ counter)
{
    __shared__ uint32_t hist[BT_NBINS];
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int k = tid; k < BT_NBINS; k += nth) hist[k] = 0;
    __syncthreads();
    for (uint32_t q = tid; q < count; q += nth) {
        uint64_t la, lb;
        bt_lengths(desc, len_a, len_b, q, la, lb);
        const int lg = bt_log2n(la, lb, max_bits);
        const int key = (lg < 0 || lg > BT_MAX_LOG2N) ? BT_NBINS - 1 : BT_MAX_LOG2N - lg;
        atomicAdd(&hist[key], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int k = 0; k < BT_NBINS; ++k) {
            const uint32_t c = hist[k];
            hist[k] = run;
            run += c;
        }
        counter[0] = 0;
    }
    __syncthreads();
    for (uint32_t q = tid; q < count; q += nth) {
        uint64_t la, lb;
        bt_lengths(desc, len_a, len_b, q, la, lb);
        const int lg = bt_log2n(la, lb, max_bits);
        const int key = (lg < 0 || lg > BT_MAX_LOG2N) ? BT_NBINS - 1 : BT_MAX_LOG2N - lg;
        order[atomicAdd(&hist[key], 1u)] = q;
    }
}

// dst[0, nw) = src bits [0, len), zero-padded
__device__ __forceinline__ void bt_load(const uint64_t *__restrict__ src, uint64_t len, uint64_t *__restrict__ dst,
                                        uint64_t nw, int tid, int nth)
{
    const uint64_t inw = (len + 63) / 64;
    for (uint64_t w = tid; w < nw; w += nth) {
        uint64_t v = 0;
        if (w < inw) {
            v = src[w];
            if (w == inw - 1 && (len & 63)) v &= (~0ull) >> (64 - (len & 63));
        }
        dst[w] = v;
    }
}

// BasisCvt(2^lgN) (or its inverse) on words [0, 2^lgN / 64) of X, ping-pong
// with Y; returns the buffer that holds the result
__device__ uint64_t *bt_basiscvt(uint64_t *X, uint64_t *Y, int lgN, bool inverse, const BatchSteps *__restrict__ BS,
                                 int tid, int nth)
{
    const uint64_t nw = (1ull << lgN) / 64;
    const int first = BS->first[lgN], cnt = BS->count[lgN];
    for (int k = 0; k < cnt; ++k) {
        const BatchStep st = BS->st[first + (inverse ? cnt - 1 - k : k)];
        if (st.S >= 128) {
            for (uint64_t w = tid; w < nw; w += nth) Y[w] = bcvt_wide_word(X, w, st.S, st.d, inverse ? 1 : 0);
        } else {
            const int H = (int)(st.S / 2), d = (int)st.d;
            for (uint64_t w = tid; w < nw; w += nth) Y[w] = bcvt_in_word(X[w], H, d, st.L, st.D, inverse ? 1 : 0);
        }
        __syncthreads();
        uint64_t *t = X;
        X = Y;
        Y = t;
    }
    return X;
}

// Steps [k0, k1) in execution order of BasisCvt(2^lgN) (steps st0[0, cnt),
// reversed for the inverse) on nw words held in LDS, in place.  Every step
// must have segments of at most 64 nw bits.  A wide step (S >= 128) runs as
// its two updates with a barrier between them (hi[0, d) ^= hi[H-d, H) and
// lo[d, H) ^= hi[0, H-d), in that order forward and the other order
// inverse); consecutive in-word steps run together in one pass.
__device__ void bt_lds_steps(uint64_t *v, int nw, const BatchStep *__restrict__ st0, int cnt, bool inverse, int k0,
                             int k1, int tid, int nth)
{
    auto step = [&](int k) { return st0[inverse ? cnt - 1 - k : k]; };
    for (int k = k0; k < k1;) {
        const BatchStep s = step(k);
        if (s.S <= 64) {
            int e = k + 1;
            while (e < k1 && step(e).S <= 64) ++e;
            for (int w = tid; w < nw; w += nth) {
                uint64_t x = v[w];
                for (int j = k; j < e; ++j) {
                    const BatchStep t = step(j);
                    x = bcvt_in_word(x, (int)(t.S / 2), (int)t.d, t.L, t.D, inverse ? 1 : 0);
                }
                v[w] = x;
            }
            __syncthreads();
            k = e;
            continue;
        }
        const int SW = (int)(s.S / 64), HW = SW / 2, lgHW = 31 - __clz(HW), nseg = nw / SW;
        const int d = (int)s.d;
        for (int ph = 0; ph < 2; ++ph) {
            const bool fix_hi = (ph == 0) != inverse;
            if (fix_hi) {
                if (d >= 64) {
                    // hi word k ^= hi word k + HW - dw, k < dw
                    const int dw = d / 64, lgdw = 31 - __clz(dw);
                    for (int t = tid; t < nseg * dw; t += nth) {
                        uint64_t *hp = v + (t >> lgdw) * SW + HW;
                        const int k2 = t & (dw - 1);
                        hp[k2] ^= hp[k2 + HW - dw];
                    }
                } else {
                    for (int sg = tid; sg < nseg; sg += nth) {
                        uint64_t *hp = v + sg * SW + HW;
                        hp[0] ^= hp[HW - 1] >> (64 - d);
                    }
                }
            } else {
                for (int t = tid; t < nseg * HW; t += nth) {
                    const int q = t & (HW - 1);
                    uint64_t *lp = v + (t >> lgHW) * SW, *hp = lp + HW;
                    if (d >= 64) {
                        const int dw = d / 64;
                        if (q >= dw) lp[q] ^= hp[q - dw];
                    } else {
                        lp[q] ^= (hp[q] << d) | (q ? hp[q - 1] >> (64 - d) : 0ull);
                    }
                }
            }
            __syncthreads();
        }
        ++k;
    }
}

#define BT_LDS_WORDS (1 << 14)   // 2^20 bits of BasisCvt in LDS at a time (128 KiB)
static_assert(BF_OFF_DATA + (2 << BF_BOTTOM_R) * 8 >= BT_LDS_WORDS * 8, "the batch kernel's LDS holds the chunk");

// BasisCvt(2^lgN) (or its inverse) on words [0, 2^lgN / 64) of X, ping-pong
// with Y for the steps whose segments exceed LDS; runs of the other steps
// are applied chunk by chunk in LDS (lds: BT_LDS_WORDS words).  Returns the
// buffer that holds the result.
__device__ uint64_t *bt_basiscvt_lds(uint64_t *X, uint64_t *Y, int lgN, bool inverse, const BatchSteps *__restrict__ BS,
                                     uint64_t *lds, int tid, int nth)
{
    const int nw = (int)((1ull << lgN) / 64);
    const int first = BS->first[lgN], cnt = BS->count[lgN];
    const BatchStep *st0 = BS->st + first;
    auto step = [&](int k) { return st0[inverse ? cnt - 1 - k : k]; };
    for (int k = 0; k < cnt;) {
        const BatchStep s = step(k);
        if (s.S <= 64ull * BT_LDS_WORDS) {
            int e = k + 1;
            while (e < cnt && step(e).S <= 64ull * BT_LDS_WORDS) ++e;
            const int chw = nw < BT_LDS_WORDS ? nw : BT_LDS_WORDS;
            for (int c0 = 0; c0 < nw; c0 += chw) {
                for (int w = tid; w < chw; w += nth) lds[w] = X[c0 + w];
                __syncthreads();
                bt_lds_steps(lds, chw, st0, cnt, inverse, k, e, tid, nth);
                for (int w = tid; w < chw; w += nth) X[c0 + w] = lds[w];
                __syncthreads();
            }
            k = e;
        } else {
            for (int w = tid; w < nw; w += nth) Y[w] = bcvt_wide_word(X, w, s.S, s.d, inverse ? 1 : 0);
            __syncthreads();
            uint64_t *t = X;
            X = Y;
            Y = t;
            ++k;
        }
    }
    return X;
}

// Encode (Alg. 4): vals[i] = sum_j bit (j n_p + i) of `bits` times r_j, n_p = 2^l
// (bits: n_p words, or only the first nwv of them with the rest zero)
__device__ void bt_encode(const uint64_t *__restrict__ bits, int l, uint64_t *__restrict__ vals,
                          const DevTables *__restrict__ T, int tid, int nth, uint64_t nwv = ~0ull)
{
    const uint64_t n_p = 1ull << l;
    if (l >= 6) {
        const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
        const uint64_t groups = n_p >> 6;
        for (uint64_t g = wave; g < groups; g += nwave) {
            // lane j: bits j n_p + 64 g .. + 63, one word; after the transpose lane t
            // holds the column of element 64 g + t
            const uint64_t iw = ((uint64_t)lane << (l - 6)) + g;
            uint64_t x = iw < nwv ? bits[iw] : 0ull;
            x = bc_wave_transpose64(x, lane);
            uint64_t f = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) f ^= T->enc_win[k][(x >> (8 * k)) & 255u];
            vals[64 * g + lane] = f;
        }
    } else {
        for (uint64_t i = tid; i < n_p; i += nth) {
            uint64_t col = 0;
            for (int j = 0; j < 64; ++j) {
                const uint64_t p = ((uint64_t)j << l) + i;
                if ((p >> 6) < nwv) col |= ((bits[p >> 6] >> (p & 63)) & 1ull) << j;
            }
            uint64_t f = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) f ^= T->enc_win[k][(col >> (8 * k)) & 255u];
            vals[i] = f;
        }
    }
}

// Decode: bit j of R^-1 vals[i] goes to bit j n_p + i of `bits` (n_p words);
// tmp (n_p words) is scratch for l < 6
__device__ void bt_decode(const uint64_t *__restrict__ vals, int l, uint64_t *__restrict__ bits,
                          uint64_t *__restrict__ tmp, const DevTables *__restrict__ T, int tid, int nth)
{
    const uint64_t n_p = 1ull << l;
    if (l >= 6) {
        const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
        const uint64_t groups = n_p >> 6;
        for (uint64_t g = wave; g < groups; g += nwave) {
            const uint64_t h = vals[64 * g + lane];
            uint64_t a = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) a ^= T->dec_win[k][(h >> (8 * k)) & 255u];
            // lane j then holds bit j of the 64 vectors: bits j n_p + 64 g .. + 63
            a = bc_wave_transpose64(a, lane);
            bits[((uint64_t)lane << (l - 6)) + g] = a;
        }
    } else {
        for (uint64_t i = tid; i < n_p; i += nth) {
            const uint64_t h = vals[i];
            uint64_t a = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) a ^= T->dec_win[k][(h >> (8 * k)) & 255u];
            tmp[i] = a;
        }
        __syncthreads();
        const uint64_t mask = n_p - 1;
        for (uint64_t W = tid; W < n_p; W += nth) {
            uint64_t r = 0;
            for (int t = 0; t < 64; ++t) {
                const uint64_t p = 64 * W + t;
                r |= ((tmp[p & mask] >> (p >> l)) & 1ull) << t;
            }
            bits[W] = r;
        }
    }
}

// one butterfly layer i >= the bottom tile, streamed through X (and Y, with
// the same multipliers, for the forward pair); every block index is below
// 128, so one K table serves the layer
__device__ void bt_upper_layer(uint64_t *__restrict__ X, uint64_t *__restrict__ Y, int l, int i, bool inverse,
                               uint8_t *smem, const DevTables *__restrict__ T, int tid, int nth)
{
    const uint8_t *s_mul8e = smem + BF_OFF_MUL8;
    uint64_t *s_tab = reinterpret_cast<uint64_t *>(smem + BF_OFF_TAB);
    uint64_t *s_basis = reinterpret_cast<uint64_t *>(smem + BF_OFF_BASIS);
    bf_build(s_tab, s_basis, l - i, 0u, 1, T, tid, nth);
    const uint32_t half = 1u << (l - 1);
    for (uint32_t q = tid; q < half; q += nth) {
        const uint32_t tb = q >> i, off = q & ((1u << i) - 1u);
        const uint32_t p0 = (tb << (i + 1)) | off, p1 = p0 | (1u << i);
        const uint8_t *row = s_mul8e + (tb & 127u) * 256;
        if (inverse) {
            bf_inv_pair(X, p0, p1, s_tab, row);
        } else {
            bf_fwd_pair(X, p0, p1, s_tab, row);
            if (Y) bf_fwd_pair(Y, p0, p1, s_tab, row);
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------ m = 32 -----
//
// Small products over GF(2^32) (Sec. 3 with m = 32): n = 2^log2n <= 2^20 bits
// ((m/2) 2^(m/2) = 2^20), n_p = n/32 values of 32 bits, l = log2n - 5 < 16.
// GF(2^32) is the low half of the tower representation, so its elements are
// 32-bit words.  Encode and Decode use 32 x 32 half-wave transposes and the
// 32 x 32 matrix R (rows r_j = product of v_{16-k} over the set bits k of
// j).  Butterfly layer i of block b multiplies by the element with Cantor
// vector 2^(16+d) XOR 2b, d = l - i; since 2b < 2^15 this is
//   x * v_{16+d}  (four 8-bit window lookups in its fixed table)
// + x * beta16    (beta16 = iota(2b) in V_16: v_perm byte products as in the
//                  V_16 split of the large passes).
#define BT32_MAX_LOG2N 20
#define BT32_OFF_K BF_OFF_DATA                        // window table of v_{16+d}, 4 KiB
#define BT32_OFF_PT8 (BF_OFF_DATA + 4096)              // v_perm tables of every byte of V_8, 8 KiB
#define BT32_OFF_IO16 (BF_OFF_DATA + 4096 + 8192)      // iota of the low two Cantor bytes, 1 KiB

__device__ __forceinline__ uint32_t bt32_enc(const DevTables *__restrict__ T, uint32_t x)
{
    return T->enc32_win[0][x & 255u] ^ T->enc32_win[1][(x >> 8) & 255u] ^ T->enc32_win[2][(x >> 16) & 255u] ^
           T->enc32_win[3][x >> 24];
}

__device__ __forceinline__ uint32_t bt32_dec(const DevTables *__restrict__ T, uint32_t h)
{
    return T->dec32_win[0][h & 255u] ^ T->dec32_win[1][(h >> 8) & 255u] ^ T->dec32_win[2][(h >> 16) & 255u] ^
           T->dec32_win[3][h >> 24];
}

// 32 x 32 bit transpose in each half-wave: lane i holds row i, afterwards
// lane t holds column t (bit i = bit t of row i); every lane takes part
__device__ __forceinline__ uint32_t bt32_transpose(uint32_t x, int lane)
{
    x = bc_tstage<16>(x, 0x0000FFFFu, lane);
    x = bc_tstage<8>(x, 0x00FF00FFu, lane);
    x = bc_tstage<4>(x, 0x0F0F0F0Fu, lane);
    x = bc_tstage<2>(x, 0x33333333u, lane);
    return bc_tstage<1>(x, 0x55555555u, lane);
}

// Encode, m = 32: vals[i] = sum over j < 32 of bit (j n_p + i) of `bits` times r_j
__device__ void bt_encode32(const uint64_t *__restrict__ bits, int l, uint32_t *__restrict__ vals,
                            const DevTables *__restrict__ T, int tid, int nth)
{
    const uint32_t n_p = 1u << l;
    if (l >= 5) {
        const uint32_t *b32 = reinterpret_cast<const uint32_t *>(bits);
        const int lane = tid & 63, t = lane & 31, half = lane >> 5, wave = tid >> 6, nwave = nth >> 6;
        const uint32_t groups = n_p >> 5;
        for (uint32_t g0 = 2 * wave; g0 < groups; g0 += 2 * nwave) {
            // lane (half, j): bits j n_p + 32 g .. + 31 of row j, one 32-bit word
            const uint32_t g = g0 + half;
            uint32_t x = g < groups ? b32[((uint32_t)t << (l - 5)) + g] : 0u;
            x = bt32_transpose(x, lane);
            if (g < groups) vals[32 * g + t] = bt32_enc(T, x);
        }
    } else {
        for (uint32_t i = tid; i < n_p; i += nth) {
            uint32_t col = 0;
            for (int j = 0; j < 32; ++j) {
                const uint32_t p = ((uint32_t)j << l) + i;
                col |= (uint32_t)((bits[p >> 6] >> (p & 63)) & 1ull) << j;
            }
            vals[i] = bt32_enc(T, col);
        }
    }
}

// Decode, m = 32: bit j of R^-1 vals[i] goes to bit j n_p + i of `bits` (n/64
// words); tmp (n_p words of 32 bits) is scratch for l < 5
__device__ void bt_decode32(const uint32_t *__restrict__ vals, int l, uint64_t *__restrict__ bits,
                            uint32_t *__restrict__ tmp, const DevTables *__restrict__ T, int tid, int nth)
{
    const uint32_t n_p = 1u << l;
    uint32_t *b32 = reinterpret_cast<uint32_t *>(bits);
    if (l >= 5) {
        const int lane = tid & 63, t = lane & 31, half = lane >> 5, wave = tid >> 6, nwave = nth >> 6;
        const uint32_t groups = n_p >> 5;
        for (uint32_t g0 = 2 * wave; g0 < groups; g0 += 2 * nwave) {
            const uint32_t g = g0 + half;
            uint32_t a = g < groups ? bt32_dec(T, vals[32 * g + t]) : 0u;
            // lane (half, j) then holds bit j of the 32 vectors: bits j n_p + 32 g .. + 31
            a = bt32_transpose(a, lane);
            if (g < groups) b32[((uint32_t)t << (l - 5)) + g] = a;
        }
    } else {
        for (uint32_t i = tid; i < n_p; i += nth) tmp[i] = bt32_dec(T, vals[i]);
        __syncthreads();
        // 32 n_p bits, i.e. n_p words of 32 bits: bit p is bit (p >> l) of tmp[p mod n_p]
        for (uint32_t W = tid; W < n_p; W += nth) {
            uint32_t r = 0;
            for (int t = 0; t < 32; ++t) {
                const uint32_t p = 32 * W + t;
                r |= ((tmp[p & (n_p - 1)] >> (p >> l)) & 1u) << t;
            }
            b32[W] = r;
        }
    }
}

// v_perm tables and iota tables of the m = 32 layers into LDS
__device__ __forceinline__ void bt32_load_tables(uint8_t *smem, const DevTables *__restrict__ T, int tid, int nth)
{
    uint32_t *s_pt8 = reinterpret_cast<uint32_t *>(smem + BT32_OFF_PT8);
    uint16_t *s_io16 = reinterpret_cast<uint16_t *>(smem + BT32_OFF_IO16);
    for (int q = tid; q < 256 * 8; q += nth) s_pt8[q] = (&T->pt8[0][0])[q];
    for (int q = tid; q < 2 * 256; q += nth) s_io16[q] = (uint16_t)(&T->iota[0][0])[q];
}

// one butterfly layer, m = 32, streamed through X (and Y with the same
// multipliers, forward only)
__device__ void bt_bfly32_layer(uint32_t *__restrict__ X, uint32_t *__restrict__ Y, int l, int i, bool inverse,
                                uint8_t *smem, const DevTables *__restrict__ T, int tid, int nth)
{
    uint32_t *s_k = reinterpret_cast<uint32_t *>(smem + BT32_OFF_K);
    const PermTab *s_pt8 = reinterpret_cast<const PermTab *>(smem + BT32_OFF_PT8);
    const uint16_t *s_io16 = reinterpret_cast<const uint16_t *>(smem + BT32_OFF_IO16);
    const int d = l - i;
    for (int q = tid; q < 1024; q += nth) s_k[q] = T->kt32[d][q];
    __syncthreads();
    const uint32_t half = 1u << (l - 1);
    for (uint32_t q = tid; q < half; q += nth) {
        const uint32_t tb = q >> i, off = q & ((1u << i) - 1u);
        const uint32_t p0 = (tb << (i + 1)) | off, p1 = p0 | (1u << i);
        const uint32_t v = 2u * tb;   // below 2^15
        const uint32_t beta = (uint32_t)s_io16[v & 255u] ^ (uint32_t)s_io16[256 + (v >> 8)];
        const PermTab *P0 = s_pt8 + (beta & 255u), *P1 = s_pt8 + (beta >> 8);
        const uint4 t0 = *reinterpret_cast<const uint4 *>(P0), t1 = *reinterpret_cast<const uint4 *>(P1);
        const uint32_t t02 = P0->t2, t12 = P1->t2;
        const PermTab *PC = s_pt8 + ((t12 >> 16) & 255u);   // beta1 v_7: entry 2 of beta1's bit-6/7 table
        const uint4 tc = *reinterpret_cast<const uint4 *>(PC);
        const uint32_t tc2 = PC->t2;
        auto mul = [&](uint32_t x) {
            const uint32_t k = s_k[x & 255u] ^ s_k[256 + ((x >> 8) & 255u)] ^ s_k[512 + ((x >> 16) & 255u)] ^
                               s_k[768 + (x >> 24)];
            return k ^ b2_mulv16(t0, t02, t1, t12, tc, tc2, x);
        };
        if (!inverse) {
            const uint32_t b = X[p1], h0 = X[p0] ^ mul(b);
            X[p0] = h0;
            X[p1] = h0 ^ b;
            if (Y) {
                const uint32_t bb = Y[p1], g0 = Y[p0] ^ mul(bb);
                Y[p0] = g0;
                Y[p1] = g0 ^ bb;
            }
        } else {
            const uint32_t h0 = X[p0], pp = h0 ^ X[p1];
            X[p0] = h0 ^ mul(pp);
            X[p1] = pp;
        }
    }
    __syncthreads();
}

// A[i] = A[i] * B[i] in GF(2^32) for i < n_p (Mul8View tables set up in LDS)
__device__ void bt_pointwise32(uint32_t *__restrict__ A, const uint32_t *__restrict__ B, uint32_t n_p, uint8_t *smem,
                               const DevTables *__restrict__ T, int tid, int nth)
{
    static_assert(BF_OFF_TAB == BF_OFF_MUL8 + 32768, "odd rows must follow the even rows");
    static_assert(BT32_OFF_K - BF_OFF_MUL8 >= M8V_BYTES, "m = 32 tables overlap the product tables");
    uint8_t *s_odd = smem + BF_OFF_TAB;
    uint16_t *s_c15 = reinterpret_cast<uint16_t *>(smem + BF_OFF_MUL8 + M8V_OFF_C15);
    const uint4 *src = reinterpret_cast<const uint4 *>(&T->mul8[0][0]);
    uint4 *dst = reinterpret_cast<uint4 *>(s_odd);
    for (int idx = tid; idx < 128 * 16; idx += nth) dst[idx] = src[(2 * (idx >> 4) + 1) * 16 + (idx & 15)];
    for (int idx = tid; idx < 512; idx += nth) s_c15[idx] = (&T->c15[0][0])[idx];
    __syncthreads();
    const Mul8View mv{smem + BF_OFF_MUL8};
    for (uint32_t e = tid; e < n_p; e += nth) A[e] = mv.m32(A[e], B[e]);
    __syncthreads();
}

// grid: persistent workgroups; slab: 4 buffers of slab_words per workgroup.
// Items come from the pools and offset arrays, or from `desc` when it is set.
__global__ __launch_bounds__(BT_THREADS) void k_batch(
    const uint64_t *__restrict__ a_pool, const uint64_t *__restrict__ a_off, const uint64_t *__restrict__ len_a,
    const uint64_t *__restrict__ b_pool, const uint64_t *__restrict__ b_off, const uint64_t *__restrict__ len_b,
    uint64_t *__restrict__ out_pool, const uint64_t *__restrict__ out_off, const BtDesc *__restrict__ desc,
    int32_t *__restrict__ status,
    uint32_t count, uint64_t max_bits, const uint32_t *__restrict__ order, uint32_t *__restrict__ counter,
    uint64_t *__restrict__ slab, uint64_t slab_words, const DevTables *__restrict__ T,
    const BatchSteps *__restrict__ BS, int m32_max_log2n)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_next;
    const int tid = threadIdx.x, nth = blockDim.x;
    uint64_t *TA = slab + (uint64_t)blockIdx.x * 4 * slab_words;
    uint64_t *TB = TA + slab_words, *X = TB + slab_words, *Y = X + slab_words;
    bf_load_mul8_even(smem + BF_OFF_MUL8, T, tid, nth);

    for (;;) {
        if (tid == 0) s_next = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t qpos = s_next;
        __syncthreads();
        if (qpos >= count) break;
        const uint32_t q = order[qpos];
        uint64_t la, lb;
        bt_lengths(desc, len_a, len_b, q, la, lb);
        const int log2n = bt_log2n(la, lb, max_bits);
        if (log2n < 0 || log2n > BT_MAX_LOG2N || (1ull << (log2n - 6)) > slab_words) {
            if (tid == 0 && status) status[q] = log2n < 0 ? 0 : -22;
            continue;
        }
        const int l = log2n - 6;
        const uint64_t n_p = 1ull << l, lc = la + lb - 1;
        // m = 32 for small transforms (GF(2^32) values), else m = 64
        const bool m32 = log2n <= m32_max_log2n && log2n <= BT32_MAX_LOG2N;
        const int l32 = log2n - 5;

        // BasisCvt and Encode of both operands: A -> TA, B -> TB
        for (int side = 0; side < 2; ++side) {
            const uint64_t len = side ? lb : la;
            const uint64_t *src = desc ? (side ? desc[q].b : desc[q].a) : (side ? b_pool + b_off[q] : a_pool + a_off[q]);
            int lgN = bt_ceil_log2(len);
            if (lgN < BT_MIN_LOG2N) lgN = BT_MIN_LOG2N;
            bt_load(src, len, X, n_p, tid, nth);
            __syncthreads();
            uint64_t *cur = bt_basiscvt_lds(X, Y, lgN, false, BS, reinterpret_cast<uint64_t *>(smem), tid, nth);
            for (uint64_t w = (1ull << lgN) / 64 + tid; w < n_p; w += nth) cur[w] = 0;
            __syncthreads();
            if (m32)
                bt_encode32(cur, l32, reinterpret_cast<uint32_t *>(side ? TB : TA), T, tid, nth);
            else
                bt_encode(cur, l, side ? TB : TA, T, tid, nth);
            __syncthreads();
        }

        // BasisCvt used all of LDS: the even rows of the GF(2^8) table back
        bf_load_mul8_even(smem + BF_OFF_MUL8, T, tid, nth);
        __syncthreads();
        if (m32) {
            // Butterfly of A and B, pointwise, iButterfly over GF(2^32); Decode
            uint32_t *A32 = reinterpret_cast<uint32_t *>(TA), *B32 = reinterpret_cast<uint32_t *>(TB);
            bt32_load_tables(smem, T, tid, nth);
            for (int i = l32 - 1; i >= 0; --i) bt_bfly32_layer(A32, B32, l32, i, false, smem, T, tid, nth);
            bt_pointwise32(A32, B32, 1u << l32, smem, T, tid, nth);
            for (int i = 0; i < l32; ++i) bt_bfly32_layer(A32, nullptr, l32, i, true, smem, T, tid, nth);
            bt_decode32(A32, l32, X, B32, T, tid, nth);
        } else {
            // Butterfly of A and B, pointwise, iButterfly: result in TA
            const int R = l < BF_BOTTOM_R ? l : BF_BOTTOM_R;
            for (int i = l - 1; i >= R; --i) bt_upper_layer(TA, TB, l, i, false, smem, T, tid, nth);
            for (uint64_t H = 0; H < (1ull << (l - R)); ++H)
                bf_bottom_tile<BF_PRODUCT>(TA, TB, l, R, H, smem, T, tid, nth);
            for (int i = R; i < l; ++i) bt_upper_layer(TA, nullptr, l, i, true, smem, T, tid, nth);
            bt_decode(TA, l, X, TB, T, tid, nth);
        }
        // iBasisCvt(2^log2n), then the first lc bits to out
        __syncthreads();
        const uint64_t *res = bt_basiscvt_lds(X, Y, log2n, true, BS, reinterpret_cast<uint64_t *>(smem), tid, nth);
        uint64_t *out = desc ? desc[q].out : out_pool + out_off[q];
        const uint64_t ow = (lc + 63) / 64;
        for (uint64_t w = tid; w < ow; w += nth) {
            uint64_t v = res[w];
            if (w == ow - 1 && (lc & 63)) v &= (~0ull) >> (64 - (lc & 63));
            out[w] = v;
        }
        if (tid == 0 && status) status[q] = 0;
        __syncthreads();
    }
}

