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

// floor(x / 64): the arithmetic shift rounds toward minus infinity
__device__ __forceinline__ int64_t floordiv64(int64_t x) { return x >> 6; }

// 64 bits of the half-array hp (HW words) from bit offset off; bits outside read 0
__device__ __forceinline__ uint64_t bits_at(const uint64_t *hp, int64_t HW, int64_t off)
{
    int64_t i0 = floordiv64(off);
    int s = (int)(off - i0 * 64);
    uint64_t w0 = (i0 >= 0 && i0 < HW) ? hp[i0] : 0ull;
    uint64_t w1 = (i0 + 1 >= 0 && i0 + 1 < HW) ? hp[i0 + 1] : 0ull;
    return s ? ((w0 >> s) | (w1 << (64 - s))) : w0;
}

// Word sources for the out-of-place form: the array itself, or the array
// after one step, read word by word (a step's new word w depends on a few
// words of the old array only, so two steps compose without a pass between).
struct WordArray {
    const uint64_t *p;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return p[i]; }
};

// bits_at on the half-array at words [base, base + HW) of src
template <class Src>
__device__ __forceinline__ uint64_t src_bits_at(const Src &src, uint64_t base, int64_t HW, int64_t off)
{
    int64_t i0 = floordiv64(off);
    int s = (int)(off - i0 * 64);
    uint64_t w0 = (i0 >= 0 && i0 < HW) ? src(base + (uint64_t)i0) : 0ull;
    uint64_t w1 = (i0 + 1 >= 0 && i0 + 1 < HW) ? src(base + (uint64_t)(i0 + 1)) : 0ull;
    return s ? ((w0 >> s) | (w1 << (64 - s))) : w0;
}

// word k of hi' = hi with hi[0, d) ^= hi[H-d, H), hi at words [base, base + HW)
template <class Src>
__device__ __forceinline__ uint64_t src_hi_prime(const Src &src, uint64_t base, int64_t HW, int64_t H, int64_t d,
                                                 int64_t k)
{
    uint64_t w = src(base + (uint64_t)k);
    int64_t rem = d - 64 * k;
    if (rem > 0) w ^= src_bits_at(src, base, HW, 64 * k + H - d) & lowmask(rem);
    return w;
}

template <class Src>
__device__ __forceinline__ uint64_t src_bits_at_prime(const Src &src, uint64_t base, int64_t HW, int64_t H, int64_t d,
                                                      int64_t off)
{
    int64_t i0 = floordiv64(off);
    int s = (int)(off - i0 * 64);
    uint64_t w0 = (i0 >= 0 && i0 < HW) ? src_hi_prime(src, base, HW, H, d, i0) : 0ull;
    uint64_t w1 = (i0 + 1 >= 0 && i0 + 1 < HW) ? src_hi_prime(src, base, HW, H, d, i0 + 1) : 0ull;
    return s ? ((w0 >> s) | (w1 << (64 - s))) : w0;
}

// new word w of a step with S >= 128 bits (segments span whole words)
template <class Src>
__device__ __forceinline__ uint64_t step_word(const Src &src, uint64_t w, uint64_t S, uint64_t d, int inverse)
{
    // S is a power of two, so the segment offset is a mask (no 64-bit division)
    const int64_t SW = (int64_t)(S / 64), HW = SW / 2, H = (int64_t)(S / 2);
    const int64_t q = (int64_t)(w & (uint64_t)(SW - 1));
    const uint64_t seg = w - (uint64_t)q, hb = seg + (uint64_t)HW;
    if (q >= HW) return src_hi_prime(src, hb, HW, H, (int64_t)d, q - HW);
    if (!inverse) return src(w) ^ src_bits_at_prime(src, hb, HW, H, (int64_t)d, 64 * q - (int64_t)d);
    return src(w) ^ src_bits_at(src, hb, HW, 64 * q - (int64_t)d);
}

// the array after one step, as a word source
template <class Src>
struct StepView {
    Src src;
    uint64_t S, d;
    int inverse;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return step_word(src, i, S, d, inverse); }
};

__device__ __forceinline__ uint64_t bcvt_wide_word(const uint64_t *__restrict__ in, uint64_t w, uint64_t S,
                                                   uint64_t d, int inverse)
{
    return step_word(WordArray{in}, w, S, d, inverse);
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
