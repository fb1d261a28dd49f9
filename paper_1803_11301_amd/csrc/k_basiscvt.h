// k_basiscvt.h -- BasisCvt (Alg. 1) and its inverse in a few HBM passes,
// fused with Encode (Alg. 4) and Decode.
//
// Alg. 1 at the top level writes f = sum_q h_q s^q with s = x^tau + x,
// tau = 2^16, deg h_q < tau (Taylor expansion), then converts the sequence
// (h_q) as a polynomial with tau-bit vector coefficients ("outer", BasisCvt of
// length R = N / tau on whole rows) and every tau-bit digit ("inner").  Outer
// and inner act on different index bits and commute.
//
// Taylor expansion without shifted half-segments: with rows c_r (f =
// sum_r c_r x^(tau r)) and x^tau = s + x, the binomial theorem over GF(2)
// gives x^(tau r) = sum_{q subset of r} s^q x^(r-q).  Hence
//     f = sum_q s^q P_q,   P_q = sum_{r superset of q} c_r x^(r-q),
// i.e. after skewing row r left by r bits (Q_r = c_r x^r) P_q is the superset
// sum of the Q_r shifted back by q: plain aligned XORs over the row index.
// P_q has degree < tau + R; writing P_q = L_q + x^tau U_q, the digits are
//     h_q = L_q + x U_q + U_{q-1}.
// The inverse runs the same way: with H_q = h_q x^q, c'_r = (superset sum of
// H)_r / x^r = lo_r + x^tau hi_r and c_r = lo_r + hi_{r-1}.
//
// Layout: rows of tau bits = 1024 words.  The skewed rows live in X with EW
// words per row (tau + R bits rounded up).  Y holds the rows transposed
// (column-major: Y[col][row]) so that the outer conversion sees one column as
// a contiguous vector; the forward path uses 64-bit columns, the inverse
// 32-bit columns.  Encode's input bit j n_p + i with i = r0 tau + c sits in
// row j (n_p / tau) + r0, column c: the outer pass gathers those 64 rows of a
// column, transposes 64 x 64 bits across a wavefront and applies the rows
// r_j by 8-bit windows.  Decode is the mirror image.
#pragma once

#include "gf_device.h"

#define BC_TAU_WORDS 1024            // tau = 2^16 bits
#define BC_THREADS 256                // zeta tiles, final store (divides BC_TAU_WORDS)
#define BC_ZETA_LDS 4096              // words of a zeta tile (2^nb rows x 2^lgWc words)
#define BC_ROW_THREADS 512            // row kernels (two workgroups per CU)
#define BC_COL_THREADS 1024           // column kernels (one workgroup per CU)
#define BC_XCDS 8                     // accelerator complex dies (separate L2 caches)
#define BC_MAX_STEPS 96

struct BcSteps {
    int n;
    uint8_t lgS[BC_MAX_STEPS];       // log2 of the segment length (bits or elements)
    uint8_t lgd[BC_MAX_STEPS];       // log2 of the shift (bits or elements)
    uint64_t L[BC_MAX_STEPS];        // in-word steps (S <= 64): low-half mask of every segment
    uint64_t D[BC_MAX_STEPS];        // in-word steps: low-d mask of every segment
};

// ------------------------------------------------------------ helpers ------

__device__ __forceinline__ uint64_t bc_lowmask(int x)
{
    return x >= 64 ? ~0ull : (x <= 0 ? 0ull : ((1ull << x) - 1ull));
}

// 64 bits starting at bit offset off of a word array w[0, nw); outside reads 0
__device__ __forceinline__ uint64_t bc_bits(const uint64_t *w, int nw, long off)
{
    const long i0 = off >> 6;                     // floor division
    const int s = (int)(off & 63);
    uint64_t a = (i0 >= 0 && i0 < nw) ? w[i0] : 0ull;
    uint64_t b = (i0 + 1 >= 0 && i0 + 1 < nw) ? w[i0 + 1] : 0ull;
    return s ? ((a >> s) | (b << (64 - s))) : a;
}

__device__ __forceinline__ uint64_t bc_word_step(uint64_t x, int H, int d, uint64_t L, uint64_t D, bool inverse)
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

// Alg. 1 steps on rows of bits in LDS (nwords words, in place), all threads.
// A step (S, d): in every S-bit segment with halves lo, hi of H = S/2 bits,
// hi[0, d) ^= hi[H-d, H) then lo[d, H) ^= hi[0, H-d); the inverse applies the
// two updates in the reverse order.  Runs of in-word steps (S <= 64) are
// applied to each word in registers with one barrier.
__device__ void bc_row_steps(uint64_t *row, int nwords, const BcSteps &st, bool inverse, int tid, int nth)
{
    int k = 0;
    while (k < st.n) {
        const int idx = inverse ? st.n - 1 - k : k;
        const int lgS = st.lgS[idx];
        if (lgS <= 6) {
            int k_end = k;
            while (k_end < st.n && st.lgS[inverse ? st.n - 1 - k_end : k_end] <= 6) ++k_end;
            for (int w = tid; w < nwords; w += nth) {
                uint64_t x = row[w];
                for (int kk = k; kk < k_end; ++kk) {
                    const int j = inverse ? st.n - 1 - kk : kk;
                    x = bc_word_step(x, 1 << (st.lgS[j] - 1), 1 << st.lgd[j], st.L[j], st.D[j], inverse);
                }
                row[w] = x;
            }
            __syncthreads();
            k = k_end;
            continue;
        }
        const int lgd = st.lgd[idx], d = 1 << lgd, H = 1 << (lgS - 1);
        const int lgSW = lgS - 6, lgHW = lgSW - 1, HW = 1 << lgHW;
        const int lgdw = lgd > 6 ? lgd - 6 : 0;          // words of hi touched by the first update
        const int lgseg = 0;
        (void)lgseg;
        for (int phase = 0; phase < 2; ++phase) {
            const bool fix_hi = (phase == 0) != inverse;
            if (fix_hi) {
                const int nt = (nwords >> lgSW) << lgdw;
                for (int t = tid; t < nt; t += nth) {
                    const int sg = t >> lgdw, kw = t & ((1 << lgdw) - 1);
                    uint64_t *hp = row + (sg << lgSW) + HW;
                    hp[kw] ^= bc_bits(hp, HW, 64L * kw + H - d) & bc_lowmask(d - 64 * kw);
                }
            } else {
                const int nt = (nwords >> lgSW) << lgHW;
                for (int t = tid; t < nt; t += nth) {
                    const int sg = t >> lgHW, q = t & (HW - 1);
                    uint64_t *lp = row + (sg << lgSW);
                    lp[q] ^= bc_bits(lp + HW, HW, 64L * q - d);
                }
            }
            __syncthreads();
        }
        ++k;
    }
}

// ---------------------------------------- BasisCvt(2^16) on rows, fixed ---
//
// The inner conversion always has 2^16 bits, so its 32 Taylor steps are
// compile-time constants (log2 S, log2 d), in the order the recursion of
// Alg. 1 produces them (the host checks this table against its generator).
#define BC16_NSTEPS 32
static constexpr uint8_t bc16_lgs[BC16_NSTEPS] = {16, 15, 14, 13, 12, 11, 10, 9, 16, 15, 14, 13, 16, 15, 16, 14,
                                                      12, 11, 12, 10, 8,  7,  6,  5, 8,  7,  8,  6,  4,  3,  4,  2};
static constexpr uint8_t bc16_lgd[BC16_NSTEPS] = {7,  6,  5,  4,  3, 2, 1, 0, 11, 10, 9, 8, 13, 12, 14, 12,
                                                      9,  8,  10, 8,  3, 2, 1, 0, 5,  4,  6, 4, 1,  0,  2,  0};

// masks of an in-word step: low half and low d bits of every S-bit segment
__host__ __device__ constexpr uint64_t bc16_mask(int S, int m)
{
    uint64_t r = 0;
    for (int b = 0; b < 64; ++b)
        if (b % S < m) r |= 1ull << b;
    return r;
}

template <int LGS, int LGD, bool INV>
__device__ __forceinline__ uint64_t bc16_inword(uint64_t x)
{
    constexpr int S = 1 << LGS, H = S / 2, d = 1 << LGD;
    constexpr uint64_t L = bc16_mask(S, H), D = bc16_mask(S, d);
    uint64_t lo = x & L, hi = (x >> H) & L;
    if (!INV) {
        hi ^= (hi >> (H - d)) & D;
        lo ^= (hi << d) & L;
    } else {
        lo ^= (hi << d) & L;
        hi ^= (hi >> (H - d)) & D;
    }
    return lo | (hi << H);
}

// one cross-word step (S >= 128 bits) on nrows rows of 1024 words; phase A
// fixes hi[0, d) from hi[H - d, H), phase B adds hi[0, H - d) into lo[d, H)
template <int LGS, int LGD, int PHASE>
__device__ __forceinline__ void bc16_cross_phase(uint64_t *rows, int nrows, int tid, int nth)
{
    constexpr int S = 1 << LGS, d = 1 << LGD;
    constexpr int SW = S / 64, HW = SW / 2, NSEG = 1024 / SW, LGHW = LGS - 7;
    constexpr int dw = d / 64, ds = d % 64;
    static_assert(HW >= 2 && HW % 2 == 0, "cross-word steps have segments of at least 256 bits");
    ulonglong2 *rows2 = reinterpret_cast<ulonglong2 *>(rows);
    if (PHASE == 0) {
        // hi[0, d) ^= hi[H - d, H)
        if constexpr (ds != 0) {
            const int nt = nrows * NSEG;
            for (int t = tid; t < nt; t += nth) {
                uint64_t *hp = rows + t * SW + HW;
                hp[0] ^= hp[HW - 1] >> (64 - d);
            }
        } else if constexpr (dw >= 2) {
            // 16-byte pairs of words
            constexpr int NA2 = dw / 2, LGNA2 = LGD - 7;
            const int nt = nrows * NSEG * NA2;
            for (int t = tid; t < nt; t += nth) {
                ulonglong2 *hp = rows2 + (t >> LGNA2) * (SW / 2) + HW / 2;
                const int k = t & (NA2 - 1);
                ulonglong2 x = hp[k];
                const ulonglong2 y = hp[k + (HW - dw) / 2];
                x.x ^= y.x;
                x.y ^= y.y;
                hp[k] = x;
            }
        } else {
            const int nt = nrows * NSEG;
            for (int t = tid; t < nt; t += nth) {
                uint64_t *hp = rows + t * SW + HW;
                hp[0] ^= hp[HW - 1];
            }
        }
    } else {
        // lo[d, H) ^= hi[0, H - d)
        if constexpr (ds != 0) {
            const int nt = nrows * NSEG * HW;
            for (int t = tid; t < nt; t += nth) {
                const int q = t & (HW - 1);
                uint64_t *lp = rows + (t >> LGHW) * SW, *hp = lp + HW;
                uint64_t v = hp[q] << ds;
                if (q) v |= hp[q - 1] >> (64 - ds);
                lp[q] ^= v;
            }
        } else if constexpr (dw % 2 == 0) {
            constexpr int HW2 = HW / 2, DW2 = dw / 2, LGHW2 = LGHW - 1;
            if constexpr (2 * dw == HW) {
                // H - d = d: DW2 pairs per segment, a power of two
                constexpr int LGDW2 = LGD - 7;
                const int nt = nrows * NSEG * DW2;
                for (int t = tid; t < nt; t += nth) {
                    ulonglong2 *lp = rows2 + (t >> LGDW2) * (SW / 2), *hp = lp + HW2;
                    const int qv = DW2 + (t & (DW2 - 1));
                    ulonglong2 x = lp[qv];
                    const ulonglong2 y = hp[qv - DW2];
                    x.x ^= y.x;
                    x.y ^= y.y;
                    lp[qv] = x;
                }
            } else {
                const int nt = nrows * NSEG * HW2;
                for (int t = tid; t < nt; t += nth) {
                    const int qv = t & (HW2 - 1);
                    if (qv < DW2) continue;
                    ulonglong2 *lp = rows2 + (t >> LGHW2) * (SW / 2), *hp = lp + HW2;
                    ulonglong2 x = lp[qv];
                    const ulonglong2 y = hp[qv - DW2];
                    x.x ^= y.x;
                    x.y ^= y.y;
                    lp[qv] = x;
                }
            }
        } else {
            const int nt = nrows * NSEG * HW;
            for (int t = tid; t < nt; t += nth) {
                const int q = t & (HW - 1);
                if (q < dw) continue;
                uint64_t *lp = rows + (t >> LGHW) * SW, *hp = lp + HW;
                lp[q] ^= hp[q - dw];
            }
        }
    }
}

template <int K, bool INV>
__device__ __forceinline__ void bc16_step(uint64_t *rows, int nrows, int tid, int nth);

// runs of in-word steps [K, KE) are applied to every word at once
template <int K, int KE, bool INV>
__device__ __forceinline__ uint64_t bc16_inword_run(uint64_t x)
{
    if constexpr (K < KE) {
        constexpr int k = INV ? BC16_NSTEPS - 1 - K : K;
        x = bc16_inword<bc16_lgs[k], bc16_lgd[k], INV>(x);
        return bc16_inword_run<K + 1, KE, INV>(x);
    } else {
        return x;
    }
}

__host__ __device__ constexpr int bc16_run_end(int K, bool inv)
{
    int e = K;
    while (e < BC16_NSTEPS && bc16_lgs[inv ? BC16_NSTEPS - 1 - e : e] <= 6) ++e;
    return e;
}

// a cross-word step with S <= 1024 bits on one aligned block of 16 words in
// registers (every segment lies inside the block)
template <int LGS, int LGD, int PHASE>
__device__ __forceinline__ void bc16_block_phase(uint64_t (&w)[16])
{
    constexpr int S = 1 << LGS, H = S / 2, d = 1 << LGD;
    constexpr int SW = S / 64, HW = SW / 2, NSEG = 16 / SW;
#pragma unroll
    for (int sg = 0; sg < NSEG; ++sg) {
        uint64_t *lo = w + sg * SW, *hi = lo + HW;
        if (PHASE == 0) {
            if (d % 64 == 0) {
#pragma unroll
                for (int k = 0; k < d / 64; ++k) hi[k] ^= hi[k + (H - d) / 64];
            } else {
                hi[0] ^= hi[HW - 1] >> (64 - d);
            }
        } else {
            constexpr int dw = d / 64, ds = d % 64;
#pragma unroll
            for (int q = HW - 1; q >= dw; --q) {
                uint64_t v = hi[q - dw];
                if (ds) {
                    v <<= ds;
                    if (q - dw - 1 >= 0) v |= hi[q - dw - 1] >> (64 - ds);
                }
                lo[q] ^= v;
            }
        }
    }
}

__host__ __device__ constexpr int bc16_block_run_end(int K, bool inv)
{
    int e = K;
    while (e < BC16_NSTEPS && bc16_lgs[inv ? BC16_NSTEPS - 1 - e : e] <= 10) ++e;
    return e;
}

template <int K, int KE, bool INV>
__device__ __forceinline__ void bc16_block_run(uint64_t (&w)[16])
{
    if constexpr (K < KE) {
        constexpr int k = INV ? BC16_NSTEPS - 1 - K : K;
        constexpr int LGS = bc16_lgs[k], LGD = bc16_lgd[k];
        if constexpr (LGS <= 6) {
#pragma unroll
            for (int i = 0; i < 16; ++i) w[i] = bc16_inword<LGS, LGD, INV>(w[i]);
        } else {
            bc16_block_phase<LGS, LGD, INV ? 1 : 0>(w);
            bc16_block_phase<LGS, LGD, INV ? 0 : 1>(w);
        }
        bc16_block_run<K + 1, KE, INV>(w);
    }
}

template <int K, bool INV>
__device__ __forceinline__ void bc16_steps_from(uint64_t *rows, int nrows, int tid, int nth)
{
    if constexpr (K < BC16_NSTEPS) {
        constexpr int k = INV ? BC16_NSTEPS - 1 - K : K;
        constexpr int LGS = bc16_lgs[k], LGD = bc16_lgd[k];
        if constexpr (LGS <= 10 && bc16_block_run_end(K, INV) - K >= 2) {
            // a run of steps inside 1024-bit segments: each thread applies it to
            // whole 16-word blocks in registers
            constexpr int KE = bc16_block_run_end(K, INV);
            for (int blk = tid; blk < nrows * 64; blk += nth) {
                uint64_t w[16];
                const ulonglong2 *src = reinterpret_cast<const ulonglong2 *>(rows + blk * 16);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const ulonglong2 v = src[i];
                    w[2 * i] = v.x;
                    w[2 * i + 1] = v.y;
                }
                bc16_block_run<K, KE, INV>(w);
                ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(rows + blk * 16);
#pragma unroll
                for (int i = 0; i < 8; ++i) dst[i] = make_ulonglong2(w[2 * i], w[2 * i + 1]);
            }
            __syncthreads();
            bc16_steps_from<KE, INV>(rows, nrows, tid, nth);
        } else if constexpr (LGS <= 6) {
            constexpr int KE = bc16_run_end(K, INV);
            for (int w = tid; w < nrows * 1024; w += nth) rows[w] = bc16_inword_run<K, KE, INV>(rows[w]);
            __syncthreads();
            bc16_steps_from<KE, INV>(rows, nrows, tid, nth);
        } else {
            bc16_cross_phase<LGS, LGD, INV ? 1 : 0>(rows, nrows, tid, nth);
            __syncthreads();
            bc16_cross_phase<LGS, LGD, INV ? 0 : 1>(rows, nrows, tid, nth);
            __syncthreads();
            bc16_steps_from<K + 1, INV>(rows, nrows, tid, nth);
        }
    }
}

// BasisCvt(2^16) (or its inverse) on nrows rows of 1024 words in LDS
template <bool INV>
__device__ __forceinline__ void bc16_rows(uint64_t *rows, int nrows, int tid, int nth)
{
    bc16_steps_from<0, INV>(rows, nrows, tid, nth);
}

// Alg. 1 steps with whole elements (the outer conversion on a column vector of
// R = 2^lgR elements of type T in LDS), in place.
template <typename T>
__device__ void bc_elem_steps(T *v, int lgR, const BcSteps &st, bool inverse, int tid, int nth)
{
    for (int k = 0; k < st.n; ++k) {
        const int idx = inverse ? st.n - 1 - k : k;
        const int lgS = st.lgS[idx], lgd = st.lgd[idx], lgH = lgS - 1;
        const int S = 1 << lgS, H = 1 << lgH, d = 1 << lgd;
        for (int phase = 0; phase < 2; ++phase) {
            const bool fix_hi = (phase == 0) != inverse;
            if (fix_hi) {
                const int nt = 1 << (lgR - lgS + lgd);
                for (int t = tid; t < nt; t += nth) {
                    const int sg = t >> lgd, p = t & (d - 1);
                    T *hp = v + (sg << lgS) + H;
                    hp[p] ^= hp[p + H - d];
                }
            } else {
                const int nt = 1 << (lgR - 1);           // all lo halves; p < d are left alone
                for (int t = tid; t < nt; t += nth) {
                    const int sg = t >> lgH, p = t & (H - 1);
                    if (p >= d) {
                        T *lp = v + (sg << lgS);
                        lp[p] ^= lp[H + p - d];
                    }
                }
            }
            __syncthreads();
        }
        (void)S;
    }
}

// ------------------------------------------------- zeta over row bits ------
//
// Superset sum over row-index bits [b0, b0 + nb) of X (R rows of EW words),
// tile = 2^nb rows (the other row bits fixed) x W words.  With skew_in set the
// tile is loaded from the unskewed rows of `in` (len bits, row r shifted left
// by r bits) instead of from X.  blockIdx.y picks the operand: (X0, in0,
// len0) or (X1, in1, len1), so that both operands of a product, of the same
// row count, take one launch.
__global__ __launch_bounds__(BC_THREADS) void k_bc_zeta(uint64_t *X0, const uint64_t *in0, uint64_t len0, int lgR,
                                                        int EW, int b0, int nb, int lgWc, int skew_in,
                                                        uint64_t *X1, const uint64_t *in1, uint64_t len1)
{
    uint64_t *__restrict__ X = blockIdx.y ? X1 : X0;
    const uint64_t *__restrict__ in = blockIdx.y ? in1 : in0;
    const uint64_t len = blockIdx.y ? len1 : len0;
    __shared__ uint64_t s[BC_ZETA_LDS];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int Wc = 1 << lgWc, rows = 1 << nb;
    const int ncolt = EW >> lgWc;
    const uint64_t ntiles = (1ull << (lgR - nb)) * (uint64_t)ncolt;
    const uint64_t inwords = (len + 63) / 64;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ct = (int)(tile % ncolt);
        const uint64_t rt = tile / ncolt;                       // row bits outside [b0, b0+nb)
        const uint64_t rlow = rt & ((1ull << b0) - 1), rhigh = rt >> b0;
        const int w0 = ct << lgWc;
        for (int e = tid; e < rows * Wc; e += nth) {
            const int k = e >> lgWc, c = e & (Wc - 1);
            const uint64_t r = (rhigh << (b0 + nb)) | ((uint64_t)k << b0) | rlow;
            const int w = w0 + c;
            uint64_t v;
            if (skew_in) {
                // stored word w of row r = row bits [64 w - r, 64 w - r + 64) of c_r
                const long off = 64L * w - (long)r;
                const uint64_t rb = r * BC_TAU_WORDS;          // first word of row r in `in`
                long i0 = off >= 0 ? off / 64 : -((-off + 63) / 64);
                int sh = (int)(off - i0 * 64);
                uint64_t a = 0, b = 0;
                if (i0 >= 0 && i0 < BC_TAU_WORDS && rb + i0 < inwords) a = in[rb + i0];
                if (i0 + 1 >= 0 && i0 + 1 < BC_TAU_WORDS && rb + i0 + 1 < inwords) b = in[rb + i0 + 1];
                // mask the bits at or above len (last input word)
                if ((len & 63) && i0 >= 0 && rb + i0 == inwords - 1) a &= (~0ull) >> (64 - (len & 63));
                if ((len & 63) && i0 + 1 >= 0 && rb + i0 + 1 == inwords - 1) b &= (~0ull) >> (64 - (len & 63));
                v = sh ? ((a >> sh) | (b << (64 - sh))) : a;
            } else {
                v = X[r * EW + w];
            }
            s[e] = v;
        }
        __syncthreads();
        for (int t = 0; t < nb; ++t) {
            for (int e = tid; e < (rows >> 1) * Wc; e += nth) {
                const int c = e & (Wc - 1), pr = e >> lgWc;
                const int k0 = ((pr >> t) << (t + 1)) | (pr & ((1 << t) - 1));
                s[(k0 << lgWc) | c] ^= s[((k0 | (1 << t)) << lgWc) | c];
            }
            __syncthreads();
        }
        for (int e = tid; e < rows * Wc; e += nth) {
            const int k = e >> lgWc, c = e & (Wc - 1);
            const uint64_t r = (rhigh << (b0 + nb)) | ((uint64_t)k << b0) | rlow;
            X[r * EW + w0 + c] = s[e];
        }
        __syncthreads();
    }
}

// The same superset sums over few row bits (NB = 1 .. 3), for the passes
// left over after a register-tile pass, whose tiles would hold too little
// work per workgroup: each thread takes one word position of the 2^NB rows
// that differ in bits [b0, b0 + NB), sums them in registers and stores all
// but the last (which no sum changes).  Consecutive threads take consecutive
// words of a row.  Operands by blockIdx.y as in k_bc_zeta.
template <int NB>
__global__ __launch_bounds__(256) void k_bc_zeta_s(uint64_t *X0, int lgR, int EW, int b0, uint64_t *X1)
{
    static_assert(NB >= 1 && NB <= 3, "short passes only");
    uint64_t *__restrict__ X = blockIdx.y ? X1 : X0;
    const uint64_t ngroups = (1ull << (lgR - NB)) * (uint64_t)EW;
    for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (uint64_t)gridDim.x * blockDim.x) {
        const int w = (int)(gi % (uint64_t)EW);
        const uint64_t rt = gi / (uint64_t)EW;         // row bits outside [b0, b0 + NB)
        const uint64_t r0 = ((rt >> b0) << (b0 + NB)) | (rt & ((1ull << b0) - 1));
        uint64_t v[1 << NB];
#pragma unroll
        for (int k = 0; k < (1 << NB); ++k) v[k] = X[(r0 | ((uint64_t)k << b0)) * EW + w];
#pragma unroll
        for (int t = 0; t < NB; ++t)
#pragma unroll
            for (int k = 0; k < (1 << NB); ++k)
                if (!((k >> t) & 1)) v[k] ^= v[k | (1 << t)];
#pragma unroll
        for (int k = 0; k < (1 << NB) - 1; ++k) X[(r0 | ((uint64_t)k << b0)) * EW + w] = v[k];
    }
}

// The same superset sums with the values in registers: a tile of 2^12 words
// (2^NB rows by 2^(12-NB) words, NB in 6..8); each of 256 threads holds 16
// values spanning four tile bits.  Pass A sums over the low four row bits
// in registers, the tile is exchanged through LDS, pass B sums over the
// remaining NB - 4 row bits (its other register bits are the top column
// bits).  Tile bits: words 0 .. 11-NB, rows 12-NB .. 11.
template <int NB>
struct BcZetaR {
    static constexpr int LGW = 12 - NB;
    // register tile bits of pass P (ascending)
    static constexpr int reg(int P, int v)
    {
        if (P == 0) return LGW + v;
        const int nrow = NB - 4;                       // row bits of pass B
        const int ncarry = 4 - nrow;                   // top column bits as padding
        return v < ncarry ? LGW - ncarry + v : LGW + 4 + (v - ncarry);
    }
    static constexpr bool is_row(int P, int v) { return reg(P, v) >= LGW; }
};

template <int NB, int P>
__device__ __forceinline__ int bcz_base(int t)
{
    int e = 0, q = 0;
#pragma unroll
    for (int b = 0; b < 12; ++b) {
        bool r = false;
#pragma unroll
        for (int v = 0; v < 4; ++v) r |= BcZetaR<NB>::reg(P, v) == b;
        if (r) continue;
        e |= ((t >> q) & 1) << b;
        ++q;
    }
    return e;
}

template <int NB, int P>
__device__ __forceinline__ int bcz_elem(int base, int v)
{
    int e = base;
#pragma unroll
    for (int m = 0; m < 4; ++m) e |= ((v >> m) & 1) << BcZetaR<NB>::reg(P, m);
    return e;
}

// (operands by blockIdx.y as in k_bc_zeta)
template <int NB>
__global__ __launch_bounds__(256) void k_bc_zeta_r(uint64_t *X0, const uint64_t *in0, uint64_t len0, int lgR, int EW,
                                                   int b0, int skew_in, uint64_t *X1, const uint64_t *in1,
                                                   uint64_t len1)
{
    uint64_t *__restrict__ X = blockIdx.y ? X1 : X0;
    const uint64_t *__restrict__ in = blockIdx.y ? in1 : in0;
    const uint64_t len = blockIdx.y ? len1 : len0;
    using Z = BcZetaR<NB>;
    constexpr int LGW = Z::LGW;
    __shared__ uint64_t s[4096 + 512];
    const int tid = threadIdx.x;
    const int ncolt = EW >> LGW;
    const uint64_t ntiles = (1ull << (lgR - NB)) * (uint64_t)ncolt;
    const uint64_t inwords = (len + 63) / 64;
    const int eA = bcz_base<NB, 0>(tid), eB = bcz_base<NB, 1>(tid);
    uint64_t x[16];
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ct = (int)(tile % ncolt);
        const uint64_t rt = tile / ncolt;
        const uint64_t rlow = rt & ((1ull << b0) - 1), rhigh = rt >> b0;
        const int w0 = ct << LGW;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int e = bcz_elem<NB, 0>(eA, v), k = e >> LGW, w = w0 + (e & ((1 << LGW) - 1));
            const uint64_t r = (rhigh << (b0 + NB)) | ((uint64_t)k << b0) | rlow;
            if (skew_in) {
                // stored word w of row r = bits [64 w - r, 64 w - r + 64) of the input row r
                const long off = 64L * w - (long)r;
                const uint64_t rb = r * BC_TAU_WORDS;
                const long i0 = off >> 6;
                const int sh = (int)(off & 63);
                uint64_t a = 0, b = 0;
                if (i0 >= 0 && i0 < BC_TAU_WORDS && rb + i0 < inwords) a = in[rb + i0];
                if (i0 + 1 >= 0 && i0 + 1 < BC_TAU_WORDS && rb + i0 + 1 < inwords) b = in[rb + i0 + 1];
                if ((len & 63) && i0 >= 0 && rb + i0 == inwords - 1) a &= (~0ull) >> (64 - (len & 63));
                if ((len & 63) && i0 + 1 >= 0 && rb + i0 + 1 == inwords - 1) b &= (~0ull) >> (64 - (len & 63));
                x[v] = sh ? ((a >> sh) | (b << (64 - sh))) : a;
            } else {
                x[v] = X[r * EW + w];
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                if (!((v >> t) & 1)) x[v] ^= x[v | (1 << t)];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int e = bcz_elem<NB, 0>(eA, v);
            s[e + (e >> 3)] = x[v];
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int e = bcz_elem<NB, 1>(eB, v);
            x[v] = s[e + (e >> 3)];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (Z::is_row(1, t))
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    if (!((v >> t) & 1)) x[v] ^= x[v | (1 << t)];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int e = bcz_elem<NB, 1>(eB, v), k = e >> LGW, w = w0 + (e & ((1 << LGW) - 1));
            const uint64_t r = (rhigh << (b0 + NB)) | ((uint64_t)k << b0) | rlow;
            X[r * EW + w] = x[v];
        }
        __syncthreads();   // the exchange area is reused by the next tile
    }
}

// ----------------------------- element steps with compile-time lengths ---
//
// The Taylor steps of BasisCvt(2^LGR) on whole elements, generated at compile
// time by the recursion of Alg. 1 (the host checks them against its own
// generator for every LGR used).
struct BcStepList {
    int n;
    uint8_t lgs[64], lgd[64];
};

__host__ __device__ constexpr void bc_gen(BcStepList &L, int lgN, int lge)
{
    if (lgN <= 1) return;
    int lgtau = 1;
    while (2 * lgtau <= lgN - 1) lgtau *= 2;
    for (int lgS = lgN; lgS >= lgtau + 1; --lgS) {
        L.lgs[L.n] = (uint8_t)(lgS + lge);
        L.lgd[L.n] = (uint8_t)(lgS - lgtau - 1 + lge);
        L.n++;
    }
    bc_gen(L, lgN - lgtau, lgtau + lge);
    bc_gen(L, lgtau, lge);
}

__host__ __device__ constexpr BcStepList bc_steps_of(int lgN)
{
    BcStepList L{};
    L.n = 0;
    bc_gen(L, lgN, 0);
    return L;
}

template <int LGR>
struct BcElemSteps {
    static constexpr BcStepList L = bc_steps_of(LGR);
};

// V consecutive column elements as one LDS access (up to 16 bytes)
template <typename T, int V>
struct BcVec;
template <> struct BcVec<uint32_t, 1> { using type = uint32_t; };
template <> struct BcVec<uint32_t, 2> { using type = uint2; };
template <> struct BcVec<uint32_t, 4> { using type = uint4; };
template <> struct BcVec<uint64_t, 1> { using type = uint64_t; };
template <> struct BcVec<uint64_t, 2> { using type = ulonglong2; };

__device__ __forceinline__ void bc_xorv(uint32_t &a, uint32_t b) { a ^= b; }
__device__ __forceinline__ void bc_xorv(uint64_t &a, uint64_t b) { a ^= b; }
__device__ __forceinline__ void bc_xorv(uint2 &a, uint2 b) { a.x ^= b.x; a.y ^= b.y; }
__device__ __forceinline__ void bc_xorv(uint4 &a, uint4 b) { a.x ^= b.x; a.y ^= b.y; a.z ^= b.z; a.w ^= b.w; }
__device__ __forceinline__ void bc_xorv(ulonglong2 &a, ulonglong2 b) { a.x ^= b.x; a.y ^= b.y; }

// A column of 2^lgR elements sits in LDS with element r at bc_swz(r): bits
// [G, G + 5) of r (G = log2 of the elements in one 16-byte access) take the
// XOR of bits [sws, sws + 5).  With sws >= G + 5 the map is an involution
// that keeps every aligned 16-byte group in place, so vector accesses and the
// per-wave shares of the steps stay valid; it spreads the 64 rows j rpj + r0
// (rpj = 2^sws) that Encode and Decode gather over distinct banks.  sws >=
// lgR leaves the column unpermuted.
template <typename T>
__device__ __forceinline__ int bc_swz(int r, int sws)
{
    constexpr int G = sizeof(T) == 8 ? 1 : 2;
    return r ^ (((r >> sws) & 31) << G);
}

// one phase of step (2^LGS, 2^LGD) on the 2^LGN elements of a column that
// start at element off, by 2^LGT threads (tid < 2^LGT), V consecutive
// elements per access (V divides d, so both operands of every access are
// V-aligned).  A phase writes elements it does not read, so every thread
// issues all its reads before its writes.
// items of a phase whose reads a thread issues together: four 16-byte
// accesses for 32-bit columns; two for 64-bit ones, whose kernel also holds
// the next column's 16 words in registers and would spill with four
template <typename T>
constexpr int bc_phase_batch() { return sizeof(T) == 8 ? 2 : 4; }
template <int LGS, int LGD, int PHASE, int LGN, int LGT, typename T>
__device__ __forceinline__ void bc_elem_phase(T *col, int off, int tid, int sws)
{
    constexpr int LGH = LGS - 1, H = 1 << LGH, d = 1 << LGD;
    constexpr int VMAX = 16 / (int)sizeof(T), V = d < VMAX ? d : VMAX, LGV = V == 4 ? 2 : V == 2 ? 1 : 0;
    constexpr int G = sizeof(T) == 8 ? 1 : 2;
    using VT = typename BcVec<T, V>::type;
    VT *vv = reinterpret_cast<VT *>(col);
    // phase 0 (hi[0, d) ^= hi[H - d, H)) and phase 1 with H - d = d have
    // d / V items per segment; phase 1 otherwise runs over all of lo and
    // leaves its first d elements alone
    constexpr bool ALL_LO = PHASE != 0 && 2 * d != H;
    constexpr int LGI = ALL_LO ? LGN - 1 - LGV : LGN - LGS + LGD - LGV;
    constexpr int PER = LGI > LGT ? 1 << (LGI - LGT) : 1;
    const int offv = off >> LGV;
    auto phys = [&](int a) -> int {   // vector index a of the region -> LDS vector index
        const int e = (offv + a) << LGV;
        return (offv + a) ^ ((((e >> sws) & 31) << G) >> LGV);
    };
    // item t -> vector index of its destination (region-relative) and whether it is written
    auto item = [&](int t, bool &w) -> int {
        int a;
        if constexpr (!ALL_LO) {
            const int sg = t >> (LGD - LGV), q = t & ((d >> LGV) - 1);
            a = (sg << (LGS - LGV)) + (PHASE == 0 ? (H >> LGV) : (d >> LGV)) + q;
            w = true;
        } else {
            const int sg = t >> (LGH - LGV), q = t & ((H >> LGV) - 1);
            a = (sg << (LGS - LGV)) + q;
            w = q >= (d >> LGV);
        }
        if (LGI < LGT && !(t < (1 << LGI))) {
            w = false;
            a = 0;   // keeps the read in range
        }
        return a;
    };
    constexpr int CH = PER < bc_phase_batch<T>() ? PER : bc_phase_batch<T>();
#pragma unroll
    for (int p0 = 0; p0 < PER; p0 += CH) {
        VT x[CH], y[CH];
#pragma unroll
        for (int p = 0; p < CH; ++p) {
            bool w;
            const int a = item(tid + ((p0 + p) << LGT), w);
            x[p] = vv[phys(a)];
            y[p] = vv[phys(a + ((H - d) >> LGV))];
        }
#pragma unroll
        for (int p = 0; p < CH; ++p) {
            bool w;
            const int a = item(tid + ((p0 + p) << LGT), w);
            if (w) {
                bc_xorv(x[p], y[p]);
                vv[phys(a)] = x[p];
            }
        }
    }
}

// LDS accesses of the lanes of one wave are made visible to the wave's other
// lanes (DS instructions of a wave complete in order; the fences keep the
// compiler from moving accesses across)
__device__ __forceinline__ void bc_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Steps [K, L.n) of BasisCvt(2^LGR) on a column of a workgroup of 2^LGW
// waves.  A step whose segments (2^LGS elements) fit in one wave's share of
// 2^(LGR - LGW) consecutive elements runs on that share alone, ordered by
// wave-level syncs instead of workgroup barriers.
template <int LGR, int K, bool INV, typename T, int LGW = 4>
__device__ __forceinline__ void bc_elem_steps_from(T *v, int tid, int sws)
{
    constexpr BcStepList L = BcElemSteps<LGR>::L;
    constexpr int LGL = LGR - LGW;   // log2 elements per wave
    if constexpr (K < L.n) {
        constexpr int k = INV ? L.n - 1 - K : K;
        constexpr int LGS = L.lgs[k], LGD = L.lgd[k];
        constexpr bool LOCAL = LGS <= LGL;
        if constexpr (LOCAL) {
            constexpr int kn = INV ? L.n - 2 - K : K + 1;   // the next step, if any
            constexpr bool NEXT_LOCAL = K + 1 < L.n && L.lgs[kn < 0 ? 0 : kn] <= LGL;
            const int off = (tid >> 6) << LGL;
            bc_elem_phase<LGS, LGD, INV ? 1 : 0, LGL, 6>(v, off, tid & 63, sws);
            bc_wave_sync();
            bc_elem_phase<LGS, LGD, INV ? 0 : 1, LGL, 6>(v, off, tid & 63, sws);
            if constexpr (NEXT_LOCAL)
                bc_wave_sync();
            else
                __syncthreads();
        } else {
            bc_elem_phase<LGS, LGD, INV ? 1 : 0, LGR, 6 + LGW>(v, 0, tid, sws);
            __syncthreads();
            bc_elem_phase<LGS, LGD, INV ? 0 : 1, LGR, 6 + LGW>(v, 0, tid, sws);
            __syncthreads();
        }
        bc_elem_steps_from<LGR, K + 1, INV, T, LGW>(v, tid, sws);
    }
}

// BasisCvt(2^lgR) on the elements of a column in LDS (swizzled by sws);
// compile-time steps for lgR in 6 .. 15, the run-time list otherwise (the
// column is then unpermuted: bc_col_sws gives sws >= lgR)
// (a workgroup of 2^LGW waves; compile-time lists up to 2^MAXLG elements)
template <typename T, int LGW = 4, int MAXLG = 15>
__device__ __forceinline__ void bc_elem_steps_any(T *v, int lgR, const BcSteps &st, bool inverse, int tid, int nth,
                                                  int sws)
{
#define BC_ELEM_CASE(R)                                                         \
    case R:                                                                     \
        if constexpr (R <= MAXLG) {                                             \
            if (inverse)                                                        \
                bc_elem_steps_from<R, 0, true, T, LGW>(v, tid, sws);            \
            else                                                                \
                bc_elem_steps_from<R, 0, false, T, LGW>(v, tid, sws);           \
            return;                                                             \
        }                                                                       \
        break;
    switch (lgR) {
        BC_ELEM_CASE(6)
        BC_ELEM_CASE(7)
        BC_ELEM_CASE(8)
        BC_ELEM_CASE(9)
        BC_ELEM_CASE(10)
        BC_ELEM_CASE(11)
        BC_ELEM_CASE(12)
        BC_ELEM_CASE(13)
        BC_ELEM_CASE(14)
        BC_ELEM_CASE(15)
    default:
        break;
    }
    bc_elem_steps<T>(v, lgR, st, inverse, tid, nth);
#undef BC_ELEM_CASE
}

// swizzle shift of a column of 2^lgR elements whose gathered rows are
// 2^lgrpj apart (only the compile-time step lists handle a swizzled column)
template <typename T>
__device__ __forceinline__ int bc_col_sws(int lgR, int lgrpj)
{
    constexpr int G = sizeof(T) == 8 ? 1 : 2;
    if (lgR < 6 || lgR > 15) return 31;
    return lgrpj > G + 5 ? lgrpj : G + 5;
}

// ------------------------------------ forward: unskew, carry, inner --------
//
// Rows q of X (skewed, superset-summed) -> digits h_q -> inner BasisCvt(2^16)
// -> Y[col][q] (64-bit columns).  BC_ROWS consecutive rows per iteration so
// the transposed store writes 64-byte runs.  With R == 1 (a single row, no
// Taylor step) the row is read from `in` directly.
#define BC_ROWS 8
#define BC_ROW_PER (BC_ROWS * BC_TAU_WORDS / BC_ROW_THREADS)   // row words per thread

// word i of w[0, nw), 0 outside; the load itself is unconditional (clamped
// index), so that a thread's loads go out together
__device__ __forceinline__ uint64_t bc_ld0(const uint64_t *w, long i, int nw)
{
    const uint64_t v = w[i < 0 ? 0 : (i >= nw ? nw - 1 : i)];
    return (i >= 0 && i < nw) ? v : 0ull;
}

// bc_bits with unconditional loads
__device__ __forceinline__ uint64_t bc_bits_u(const uint64_t *w, int nw, long off)
{
    const long i0 = off >> 6;
    const int s = (int)(off & 63);
    const uint64_t a = bc_ld0(w, i0, nw), b = bc_ld0(w, i0 + 1, nw);
    return s ? ((a >> s) | (b << (64 - s))) : a;
}

// rpw: rows per workgroup iteration, a power of two up to BC_ROWS (fewer
// spread a short operand's few rows over more CUs).  blockIdx.y picks the
// operand: (X0, in0, len0, Y0) or (X1, in1, len1, Y1).
__global__ __launch_bounds__(BC_ROW_THREADS) void k_bc_fwd_rows(const uint64_t *X0, const uint64_t *in0,
                                                            uint64_t len0, int lgR, int EW, uint64_t *Y0,
                                                            BcSteps inner, int rpw, const uint64_t *X1,
                                                            const uint64_t *in1, uint64_t len1, uint64_t *Y1)
{
    const uint64_t *__restrict__ X = blockIdx.y ? X1 : X0;
    const uint64_t *__restrict__ in = blockIdx.y ? in1 : in0;
    const uint64_t len = blockIdx.y ? len1 : len0;
    uint64_t *__restrict__ Y = blockIdx.y ? Y1 : Y0;
    __shared__ __align__(16) uint64_t rows[BC_ROWS * BC_TAU_WORDS];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int R = 1 << lgR, T = R < rpw ? R : rpw;
    const uint64_t inwords = (len + 63) / 64;
    for (int q0 = blockIdx.x * T; q0 < R; q0 += gridDim.x * T) {
        if (T == BC_ROWS && nth == BC_ROW_THREADS) {
            // L_q: bits [64 w + q, 64 w + q + 64) of row q, words w + q/64 and
            // the next (both below EW); all loads of the thread in flight together
            uint64_t a[BC_ROW_PER], b[BC_ROW_PER];
#pragma unroll
            for (int i = 0; i < BC_ROW_PER; ++i) {
                const int e = tid + i * BC_ROW_THREADS, k = e / BC_TAU_WORDS, w = e % BC_TAU_WORDS, q = q0 + k;
                const uint64_t *p = X + (uint64_t)q * EW + w + (q >> 6);
                a[i] = p[0];
                b[i] = p[1];
            }
#pragma unroll
            for (int i = 0; i < BC_ROW_PER; ++i) {
                const int e = tid + i * BC_ROW_THREADS, k = e / BC_TAU_WORDS, s = (q0 + k) & 63;
                rows[e] = s ? ((a[i] >> s) | (b[i] << (64 - s))) : a[i];
            }
            __syncthreads();
            // x U_q + U_{q-1} on the first R/64 + 1 words of every row
            const int nu = R / 64 + 1;
            for (int e = tid; e < BC_ROWS * nu; e += BC_ROW_THREADS) {
                const int k = e / nu, w = e % nu, q = q0 + k;
                const uint64_t *pq = X + (uint64_t)q * EW;
                uint64_t u = bc_bits_u(pq, EW, 64L * (BC_TAU_WORDS + w) + q - 1);   // U bit b -> bit b + 1
                uint64_t m = ~0ull;
                if (w == 0) m &= ~1ull;
                if ((long)R + 1 - 64L * w < 64) m &= bc_lowmask(R + 1 - 64 * w);
                uint64_t v = u & m;
                const uint64_t *pp = X + (uint64_t)(q > 0 ? q - 1 : 0) * EW;
                uint64_t up = bc_bits_u(pp, EW, 64L * (BC_TAU_WORDS + w) + (q - 1));
                if (64 * (w + 1) > R) up &= bc_lowmask(R - 64 * w);
                if (q > 0 && 64 * w < R) v ^= up;
                rows[k * BC_TAU_WORDS + w] ^= v;
            }
        } else {
            for (int e = tid; e < T * BC_TAU_WORDS; e += nth) {
                const int k = e / BC_TAU_WORDS, w = e % BC_TAU_WORDS, q = q0 + k;
                uint64_t v;
                if (R == 1) {
                    v = (uint64_t)w < inwords ? in[w] : 0ull;
                    if ((uint64_t)w == inwords - 1 && (len & 63)) v &= (~0ull) >> (64 - (len & 63));
                } else {
                    const uint64_t *pq = X + (uint64_t)q * EW;
                    v = bc_bits(pq, EW, 64L * w + q);                                   // L_q
                    if (64 * w <= R) {                                                 // x U_q: U bit b -> bit b + 1
                        uint64_t u = bc_bits(pq, EW, 64L * (BC_TAU_WORDS + w) + q - 1);
                        uint64_t m = ~0ull;
                        if (w == 0) m &= ~1ull;
                        if ((long)R + 1 - 64L * w < 64) m &= bc_lowmask(R + 1 - 64 * w);
                        v ^= u & m;
                    }
                    if (q > 0 && 64 * w < R) {                                         // U_{q-1}
                        const uint64_t *pp = X + (uint64_t)(q - 1) * EW;
                        uint64_t u = bc_bits(pp, EW, 64L * (BC_TAU_WORDS + w) + (q - 1));
                        if (64 * (w + 1) > R) u &= bc_lowmask(R - 64 * w);
                        v ^= u;
                    }
                }
                rows[e] = v;
            }
        }
        __syncthreads();
        bc16_rows<false>(rows, T, tid, nth);
        if (T == BC_ROWS) {
            // eight consecutive threads write one 64-byte run of a column
            for (int e = tid; e < BC_ROWS * BC_TAU_WORDS; e += nth) {
                const int k = e & (BC_ROWS - 1), w = e >> 3;
                Y[(uint64_t)w * R + q0 + k] = rows[k * BC_TAU_WORDS + w];
            }
        } else {
            for (int e = tid; e < T * BC_TAU_WORDS; e += nth) {
                const int k = e % T, w = e / T;
                Y[(uint64_t)w * R + q0 + k] = rows[k * BC_TAU_WORDS + w];
            }
        }
        __syncthreads();
    }
}

// Lane exchanges without the LDS: the value of lane (lane ^ J) for J < 64,
// through DPP row operations (J <= 8; row_ror:N delivers lane (i - N) mod 16
// of each 16-lane row) and the gfx950 half-row / half-wave swaps (J = 16, 32).
// Every lane has a source lane in these DPP patterns, so bound_ctrl (zero for
// a lane without one) never applies; it lets the move drop its old operand.
template <int J>
__device__ __forceinline__ uint32_t bc_xor_lane(uint32_t v, int lane)
{
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, true);   // quad_perm [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, true);   // quad_perm [2,3,0,1]
    } else if constexpr (J == 4) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x12C, 0xf, 0xf, true);   // i + 4
        const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, true);   // i - 4
        return (lane & 4) ? dn : up;
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, true);   // row_ror:8
    } else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
}

// one stage of the transpose on a 32-bit word: lanes with bit J clear keep
// the bits of mask m and take the partner's bits of m shifted up by J; the
// others keep ~m and take the partner's bits of ~m shifted down by J
//
// Both cases are one rotation and one bit-field insert: the partner's word
// rotated right by J (upper lanes) or by 32 - J (lower lanes) has the wanted
// bits in place, and the bits that wrap around fall outside the taken mask.
// The rotation amount and the kept mask depend on the lane only.
template <int J>
__device__ __forceinline__ uint32_t bc_tstage(uint32_t x, uint32_t m, int lane)
{
    const uint32_t y = bc_xor_lane<J>(x, lane);
    const bool up = (lane & J) != 0;
    const uint32_t keep = up ? ~m : m, rot = up ? (uint32_t)J : (uint32_t)(32 - J);
    const uint32_t t = __builtin_amdgcn_alignbit(y, y, rot);   // y rotated right by rot
    return ((x ^ t) & keep) ^ t;   // x on keep, t elsewhere: one bit-field insert
}

// The J = 16 stage on both words of a lane at once: the low 16-bit halves
// of lo and hi packed in one register, the high halves in another.  One
// half-row swap (odd rows of the first with even rows of the second) leaves
// a lane of an even row its own low halves and its partner's, a lane of an
// odd row its partner's high halves and its own, in the same two registers;
// two byte permutes put them back as lo and hi.
__device__ __forceinline__ void bc_tstage16_pair(uint32_t &lo, uint32_t &hi)
{
    const uint32_t a = __builtin_amdgcn_perm(hi, lo, 0x05040100u);   // lo[15:0], hi[15:0]
    const uint32_t b = __builtin_amdgcn_perm(hi, lo, 0x07060302u);   // lo[31:16], hi[31:16]
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    lo = __builtin_amdgcn_perm(r[1], r[0], 0x05040100u);
    hi = __builtin_amdgcn_perm(r[1], r[0], 0x07060302u);
}

// 64 x 64 bit transpose across a wavefront: lane i holds row i; afterwards
// lane t holds column t (bit i = bit t of row i)
__device__ __forceinline__ uint64_t bc_wave_transpose64(uint64_t x, int lane)
{
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {
        // J = 32: lanes below 32 take the partner's low word as their high word,
        // lanes from 32 up take the partner's high word as their low word: one
        // swap of the upper half-wave of lo with the lower half-wave of hi
        const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        lo = r[0];
        hi = r[1];
    }
    bc_tstage16_pair(lo, hi);
    lo = bc_tstage<8>(lo, 0x00FF00FFu, lane);
    hi = bc_tstage<8>(hi, 0x00FF00FFu, lane);
    lo = bc_tstage<4>(lo, 0x0F0F0F0Fu, lane);
    hi = bc_tstage<4>(hi, 0x0F0F0F0Fu, lane);
    lo = bc_tstage<2>(lo, 0x33333333u, lane);
    hi = bc_tstage<2>(hi, 0x33333333u, lane);
    lo = bc_tstage<1>(lo, 0x55555555u, lane);
    hi = bc_tstage<1>(hi, 0x55555555u, lane);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// the 8-bit window product sum_k tab[k][byte k of x] (Encode's R, Decode's
// R^-1), the eight lookups issued together
__device__ __forceinline__ uint64_t bc_win8(const uint64_t (*tab)[256], uint64_t x)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint64_t t0 = tab[0][lo & 255u], t1 = tab[1][(lo >> 8) & 255u], t2 = tab[2][(lo >> 16) & 255u],
                   t3 = tab[3][lo >> 24], t4 = tab[4][hi & 255u], t5 = tab[5][(hi >> 8) & 255u],
                   t6 = tab[6][(hi >> 16) & 255u], t7 = tab[7][hi >> 24];
    auto x3 = [](uint64_t a, uint64_t b, uint64_t c, int h) -> uint32_t {   // three-input XOR of half h
        return (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(a >> (32 * h)), (uint32_t)(b >> (32 * h)),
                                           (uint32_t)(c >> (32 * h)), 0x96);
    };
    auto half = [&](int h) -> uint32_t {   // unsigned: the halves are joined below without sign extension
        return (uint32_t)__builtin_amdgcn_bitop3_b32(x3(t0, t1, t2, h), x3(t3, t4, t5, h),
                                                     (uint32_t)(t6 >> (32 * h)) ^ (uint32_t)(t7 >> (32 * h)), 0x96);
    };
    return (uint64_t)half(0) | ((uint64_t)half(1) << 32);
}

// Outer BasisCvt(R) on one 64-bit column of Y, then Encode: element
// i = r0 tau + 64 col + t takes bits j n_p + i, found in rows j (n_p/tau) + r0.
// One column per workgroup iteration; R <= 2^14 (the column fits LDS).  The
// next column is loaded into registers while this one is converted and
// encoded.
#define BC_ENC_PRE 16   // column words per thread: R <= 2^14 = BC_ENC_PRE x BC_COL_THREADS
// Column kernels come in two sizes: the full one (16 waves, columns of up to
// 2^14 (Encode) or 2^15 (Decode) rows in LDS, one workgroup per CU) and a
// compact one for short columns (4 waves, up to 2^10 or 2^11 rows, four
// workgroups per CU), so that the columns of a short operand are converted
// side by side on a CU rather than one after another.  2^LGW waves, columns
// of up to 2^LGCAP elements (the host launches only lgR <= LGCAP), PRE column
// words per thread in flight, at least MINW waves per SIMD.  The Encode
// kernel takes the operand by blockIdx.y: (Y0, vals0) or (Y1, vals1).
#define BC_ENC_SMALL_LG 10   // compact Encode kernel for lgR up to this
template <int LGW, int LGCAP, int PRE, int MINW>
__global__ __launch_bounds__(64 << LGW, MINW) void k_bc_outer_encode(const uint64_t *Y0, int lgR, int l,
                                                                   uint64_t *vals0, BcSteps outer,
                                                                   const DevTables *__restrict__ T,
                                                                   const uint64_t *Y1, uint64_t *vals1)
{
    const uint64_t *__restrict__ Y = blockIdx.y ? Y1 : Y0;
    uint64_t *__restrict__ vals = blockIdx.y ? vals1 : vals0;
    constexpr int NT = 64 << LGW, NW = NT / 64;
    static_assert((1 << LGCAP) <= PRE * NT, "a thread's share of the column is in flight at once");
    __shared__ __align__(16) uint64_t col[1 << LGCAP];
    __shared__ uint64_t enc[8][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int R = 1 << lgR;
    const int lgrpj = l - 16, rpj = 1 << lgrpj;           // n_p / tau
    const int sws = bc_col_sws<uint64_t>(lgR, lgrpj);
    const int per = R >= NT ? R / NT : 1;
    for (int i = tid; i < 8 * 256; i += NT) (&enc[0][0])[i] = (&T->enc_win[0][0])[i];
    uint64_t pre[PRE];
    auto load = [&](int c, int tid_c) {
        const uint64_t *src = Y + (uint64_t)c * R;
#pragma unroll
        for (int k = 0; k < PRE; ++k) {
            const int r = tid_c + k * NT;
            if (k < per) pre[k] = src[r < R ? r : R - 1];
        }
    };
    int c = blockIdx.x;
    if (c < BC_TAU_WORDS) load(c, tid);
    for (; c < BC_TAU_WORDS; c += gridDim.x) {
        // every address below depends on tid only; recomputing them per
        // column keeps the compiler from holding hundreds of them live (and
        // spilled) across the loop
        int tid_c = tid;
        asm volatile("" : "+v"(tid_c));
#pragma unroll
        for (int k = 0; k < PRE; ++k) {
            const int r = tid_c + k * NT;
            if (k < per && r < R) col[bc_swz<uint64_t>(r, sws)] = pre[k];
        }
        __syncthreads();
        if (c + (int)gridDim.x < BC_TAU_WORDS) load(c + gridDim.x, tid_c);   // in flight during this column
        bc_elem_steps_any<uint64_t, LGW, LGCAP>(col, lgR, outer, false, tid_c, NT, sws);
#pragma unroll 1
        for (int r0 = wave; r0 < rpj; r0 += NW) {
            const int rr = lane * rpj + r0;              // row of Encode input row j = lane
            uint64_t x = rr < R ? col[bc_swz<uint64_t>(rr, sws)] : 0ull;
            x = bc_wave_transpose64(x, lane);
            vals[((uint64_t)r0 << 16) + 64u * c + lane] = bc_win8(enc, x);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ inverse ------

// Decode and the inverse outer conversion: for a 32-bit column c (bits
// [32 c, 32 c + 32) of every row), element i = r0 tau + 32 c + t decodes to 64
// bits; bit j goes to row j (n_p/tau) + r0.  Then iOuter on the column.  A
// half-wave decodes the 32 elements of one r0; the values of the next column
// are loaded into registers while this one is converted and stored.
#define BC_DEC_PRE 16   // r0 pairs per wave and column: n_p / tau <= 2 x 16 waves x BC_DEC_PRE
#define BC_DEC_SMALL_LG 11   // compact Decode kernel for lgR up to this
// (sizes as for k_bc_outer_encode; PRE r0 passes per wave in flight)
template <int LGW, int LGCAP, int PRE, int MINW>
__global__ __launch_bounds__(64 << LGW, MINW) void k_bc_decode_outer(const uint64_t *__restrict__ vals, int lgR, int l,
                                                                   uint32_t *__restrict__ Y32, BcSteps outer,
                                                                   const DevTables *__restrict__ T)
{
    constexpr int NT = 64 << LGW, NW = NT / 64;
    static_assert((1 << (LGCAP - 6)) <= 2 * NW * PRE, "a wave's r0 passes are in flight at once");
    __shared__ __align__(16) uint32_t col[1 << LGCAP];
    __shared__ uint64_t dec[8][256];
    const int R = 1 << lgR;
    const int lgrpj = l - 16, rpj = 1 << lgrpj;
    const int sws = bc_col_sws<uint32_t>(lgR, lgrpj);
    const int kmax = (rpj + 2 * NW - 1) / (2 * NW);       // r0 passes per wave
    constexpr int NCOL = 2 * BC_TAU_WORDS;
    for (int i = threadIdx.x; i < 8 * 256; i += NT) (&dec[0][0])[i] = (&T->dec_win[0][0])[i];
    uint64_t pre[PRE];
    // lane (half, t) of wave w decodes element 32 c + t of r0 = 2 w + 2 NW k + half
    auto load = [&](int c, int tid_c) {
        const int wave = tid_c >> 6, half = (tid_c >> 5) & 1, t = tid_c & 31;
#pragma unroll
        for (int k = 0; k < PRE; ++k) {
            const int r0 = 2 * wave + 2 * NW * k + half;
            if (k < kmax) pre[k] = vals[((uint64_t)(r0 < rpj ? r0 : rpj - 1) << 16) + 32u * c + t];
        }
    };
    int c = blockIdx.x;
    if (c < NCOL) load(c, threadIdx.x);
    __syncthreads();   // dec
    for (; c < NCOL; c += gridDim.x) {
        // every address below depends on the thread index only; recomputing
        // them per column keeps the compiler from holding them live (and
        // spilled) across the loop
        int tid_c = threadIdx.x;
        asm volatile("" : "+v"(tid_c));
        const int lane = tid_c & 63, wave = tid_c >> 6, half = lane >> 5, t = lane & 31;
#pragma unroll
        for (int k = 0; k < PRE; ++k) {
            if (k >= kmax) continue;   // uniform
            const int r0 = 2 * wave + 2 * NW * k + half;
            const uint64_t a = bc_win8(dec, pre[k]);
            // transpose the two 32 x 64 blocks (one per half-wave): afterwards lane
            // (half, j) holds bits j and j + 32 of the 32 decoded vectors
            uint32_t lo = (uint32_t)a, hi = (uint32_t)(a >> 32);
            bc_tstage16_pair(lo, hi);
            lo = bc_tstage<8>(lo, 0x00FF00FFu, lane);
            hi = bc_tstage<8>(hi, 0x00FF00FFu, lane);
            lo = bc_tstage<4>(lo, 0x0F0F0F0Fu, lane);
            hi = bc_tstage<4>(hi, 0x0F0F0F0Fu, lane);
            lo = bc_tstage<2>(lo, 0x33333333u, lane);
            hi = bc_tstage<2>(hi, 0x33333333u, lane);
            lo = bc_tstage<1>(lo, 0x55555555u, lane);
            hi = bc_tstage<1>(hi, 0x55555555u, lane);
            if (r0 < rpj) {
                // lane t now holds bit t of vector s at bit s: that is row j = t (lo) and j = t + 32 (hi)
                const int rlo = t * rpj + r0, rhi = (t + 32) * rpj + r0;
                if (rlo < R) col[bc_swz<uint32_t>(rlo, sws)] = lo;
                if (rhi < R) col[bc_swz<uint32_t>(rhi, sws)] = hi;
            }
        }
        __syncthreads();
        if (c + (int)gridDim.x < NCOL) load(c + gridDim.x, tid_c);   // in flight during this column
        bc_elem_steps_any<uint32_t, LGW, LGCAP>(col, lgR, outer, true, tid_c, NT, sws);
        uint32_t *dst = Y32 + (uint64_t)c * R;
        if (R >= 4 * NT) {
            // 16-byte groups stay whole under the swizzle
            const uint4 *c4 = reinterpret_cast<const uint4 *>(col);
            uint4 *d4 = reinterpret_cast<uint4 *>(dst);
            for (int g = tid_c; g < R / 4; g += NT) d4[g] = c4[bc_swz<uint32_t>(4 * g, sws) >> 2];
        } else {
            for (int r = tid_c; r < R; r += NT) dst[r] = col[bc_swz<uint32_t>(r, sws)];
        }
        __syncthreads();
    }
}

// Inverse inner conversion of rows (read from the 32-bit columns of Y32,
// BC_ROWS per iteration), then skew: X row q = h_q << q (EW words).
__global__ __launch_bounds__(BC_ROW_THREADS) void k_bc_inv_rows(const uint32_t *__restrict__ Y32, int lgR, int EW,
                                                            uint64_t *__restrict__ X, BcSteps inner, int rpw)
{
    __shared__ __align__(16) uint64_t rows[BC_ROWS * BC_TAU_WORDS];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int R = 1 << lgR, T = R < rpw ? R : rpw;
    // workgroups go to the 8 XCDs round robin; those of one XCD take
    // consecutive row groups, so that each 128-byte line of a column (32
    // rows) is fetched once into that XCD's L2 rather than into four
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned w = G % BC_XCDS == 0 ? (b % BC_XCDS) * (G / BC_XCDS) + b / BC_XCDS : b;
    for (int q0 = (int)w * T; q0 < R; q0 += (int)G * T) {
        uint32_t *rows32 = reinterpret_cast<uint32_t *>(rows);
        if (T == BC_ROWS && nth == BC_ROW_THREADS) {
            // 32-bit columns c = tid + j BC_ROW_THREADS: a 32-byte run of Y32
            // each, all loads in flight together; LDS writes of consecutive
            // words per wave (no bank conflicts)
            constexpr int NC = 2 * BC_TAU_WORDS / BC_ROW_THREADS;
            uint4 v0[NC], v1[NC];
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const uint4 *src = reinterpret_cast<const uint4 *>(Y32 + (uint64_t)(tid + j * BC_ROW_THREADS) * R + q0);
                v0[j] = src[0];
                v1[j] = src[1];
            }
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int c = tid + j * BC_ROW_THREADS;
                rows32[0 * 2 * BC_TAU_WORDS + c] = v0[j].x;
                rows32[1 * 2 * BC_TAU_WORDS + c] = v0[j].y;
                rows32[2 * 2 * BC_TAU_WORDS + c] = v0[j].z;
                rows32[3 * 2 * BC_TAU_WORDS + c] = v0[j].w;
                rows32[4 * 2 * BC_TAU_WORDS + c] = v1[j].x;
                rows32[5 * 2 * BC_TAU_WORDS + c] = v1[j].y;
                rows32[6 * 2 * BC_TAU_WORDS + c] = v1[j].z;
                rows32[7 * 2 * BC_TAU_WORDS + c] = v1[j].w;
            }
        } else {
            for (int e = tid; e < T * 2 * BC_TAU_WORDS; e += nth) {
                const int k = e % T, c = e / T;                 // 32-bit column c of row q0 + k
                rows32[k * 2 * BC_TAU_WORDS + c] = Y32[(uint64_t)c * R + q0 + k];
            }
        }
        __syncthreads();
        bc16_rows<true>(rows, T, tid, nth);
        // row by row: no division by the run-time row length
        for (int k = 0; k < T; ++k) {
            const int q = q0 + k;
            const uint64_t *rk = rows + k * BC_TAU_WORDS;
            uint64_t *xq = X + (uint64_t)q * EW;
            for (int w = tid; w < EW; w += nth) xq[w] = bc_bits(rk, BC_TAU_WORDS, 64L * w - q);
        }
        __syncthreads();
    }
}

// Last inverse pass: unskew (c'_r = Z_r >> r), carry (c_r = lo_r + hi_{r-1})
// and the masked store of the first len bits.  One row per iteration.
__global__ __launch_bounds__(BC_THREADS) void k_bc_inv_store(const uint64_t *__restrict__ X, int lgR, int EW,
                                                             uint64_t len, uint64_t *__restrict__ out)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int R = 1 << lgR;
    const uint64_t outw = (len + 63) / 64;
    // the loads of the row's words a thread handles go out together
    constexpr int PER = BC_TAU_WORDS / BC_THREADS;
    for (int r = blockIdx.x; r < R; r += gridDim.x) {
        const uint64_t *xr = X + (uint64_t)r * EW;
        const uint64_t *xp = r ? X + (uint64_t)(r - 1) * EW : nullptr;
        const int sh = r & 63, wr = r >> 6;   // output word w = bits [64 (w + wr) + sh, + 64) of row r
        uint64_t a[PER], b[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * nth + wr;
            a[k] = i < EW ? xr[i] : 0ull;
            b[k] = i + 1 < EW ? xr[i + 1] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int w = tid + k * nth;
            const uint64_t ow = (uint64_t)r * BC_TAU_WORDS + w;
            if (ow >= outw) continue;
            uint64_t v = sh ? ((a[k] >> sh) | (b[k] << (64 - sh))) : a[k];
            if (xp && 64 * w < R) {
                uint64_t h = bc_bits(xp, EW, 64L * (BC_TAU_WORDS + w) + (r - 1));
                if (64 * (w + 1) > R) h &= bc_lowmask(R - 64 * w);
                v ^= h;
            }
            if (ow == outw - 1 && (len & 63)) v &= (~0ull) >> (64 - (len & 63));
            out[ow] = v;
        }
    }
}
