// k_steps.h -- one Taylor step of BasisCvt (Alg. 1) on a word array, as
// device functions shared by the per-step kernels and the batch kernel.
//
// A step (S, d) acts on every S-bit segment with halves lo, hi of H = S/2
// bits:  hi[0, d) ^= hi[H-d, H), then lo[d, H) ^= hi[0, H-d) (forward); the
// inverse applies the two updates in the other order.  Out-of-place: the
// new word w is a function of the old array.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

__device__ __forceinline__ uint64_t lowmask(int64_t x)
{
    return x >= 64 ? ~0ull : (x <= 0 ? 0ull : ((1ull << x) - 1ull));
}

__device__ __forceinline__ int64_t floordiv64(int64_t x) { return x >= 0 ? x / 64 : -((-x + 63) / 64); }

// 64 bits of the half-array hp (HW words) from bit offset off; bits outside read 0
__device__ __forceinline__ uint64_t bits_at(const uint64_t *hp, int64_t HW, int64_t off)
{
    int64_t i0 = floordiv64(off);
    int s = (int)(off - i0 * 64);
    uint64_t w0 = (i0 >= 0 && i0 < HW) ? hp[i0] : 0ull;
    uint64_t w1 = (i0 + 1 >= 0 && i0 + 1 < HW) ? hp[i0 + 1] : 0ull;
    return s ? ((w0 >> s) | (w1 << (64 - s))) : w0;
}

// word k of hi' = hi with hi[0, d) ^= hi[H-d, H)
__device__ __forceinline__ uint64_t hi_prime(const uint64_t *hp, int64_t HW, int64_t H, int64_t d, int64_t k)
{
    uint64_t w = hp[k];
    int64_t rem = d - 64 * k;
    if (rem > 0) w ^= bits_at(hp, HW, 64 * k + H - d) & lowmask(rem);
    return w;
}

__device__ __forceinline__ uint64_t bits_at_prime(const uint64_t *hp, int64_t HW, int64_t H, int64_t d, int64_t off)
{
    int64_t i0 = floordiv64(off);
    int s = (int)(off - i0 * 64);
    uint64_t w0 = (i0 >= 0 && i0 < HW) ? hi_prime(hp, HW, H, d, i0) : 0ull;
    uint64_t w1 = (i0 + 1 >= 0 && i0 + 1 < HW) ? hi_prime(hp, HW, H, d, i0 + 1) : 0ull;
    return s ? ((w0 >> s) | (w1 << (64 - s))) : w0;
}

// new word w of a step with S >= 128 bits (segments span whole words)
__device__ __forceinline__ uint64_t bcvt_wide_word(const uint64_t *__restrict__ in, uint64_t w, uint64_t S,
                                                   uint64_t d, int inverse)
{
    const int64_t SW = (int64_t)(S / 64), HW = SW / 2, H = (int64_t)(S / 2);
    const int64_t q = (int64_t)(w % (uint64_t)SW);
    const uint64_t *seg = in + (w - (uint64_t)q);
    const uint64_t *hp = seg + HW;
    if (q >= HW) return hi_prime(hp, HW, H, (int64_t)d, q - HW);
    if (!inverse) return seg[q] ^ bits_at_prime(hp, HW, H, (int64_t)d, 64 * q - (int64_t)d);
    return seg[q] ^ bits_at(hp, HW, 64 * q - (int64_t)d);
}

// new value of word x for a step with S <= 64 (several segments per word);
// L marks the low half of every segment, D its low d bits
__device__ __forceinline__ uint64_t bcvt_in_word(uint64_t x, int H, int d, uint64_t L, uint64_t D, int inverse)
{
    uint64_t lo = x & L, hi = (x >> H) & L;
    if (!inverse) {
        hi ^= (hi >> (H - d)) & D;
        lo ^= (hi << d) & L;
    } else {
        lo ^= (hi << d) & L;
        hi ^= (hi >> (H - d)) & D;
    }
    return lo | (hi << H);
}
