// fpmul.hip -- gfx950 kernels and the C ABI (include/fpmul.h) for the product
// of bit polynomials with Frobenius partitions in the additive FFT.
//
// Pipeline of one product (Alg. 5, FP_Polymul), n = transform length in bits,
// l = log2(n) - 6, n_p = 2^l points of Sigma = v_{l+32} + V_l (Eq. 6):
//   BasisCvt(A), Encode, Butterfly      (Alg. 1, Alg. 4, Alg. 2 at v_{l+32})
//   BasisCvt(B), Encode, Butterfly
//   pointwise products in GF(2^64)      (Alg. 5, the pointwise step)
//   iButterfly, Decode, iBasisCvt       (Alg. 5, the inverse steps)
//
// Field elements are uint64_t in the tower representation over V_8 (see
// consts_host.h and gf_device.h).  Layer i of block b multiplies by
// s_i(v_{l+32} + b 2^(i+1)) whose Cantor vector is 2^(32+d) XOR 2b, d = l - i
// (Eq. 4 and the recursion of Alg. 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fpmul.h"
#include "consts_host.h"
#include "plan.h"

#define FPMUL_VERSION "fpmul 0.1 (gfx950)"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(POLYMUL_EIO, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

#define LAUNCH_CHECK(name)                                                               \
    do {                                                                                 \
        hipError_t _e = hipGetLastError();                                               \
        if (_e != hipSuccess)                                                            \
            return fail(POLYMUL_EIO, std::string("launch " name ": ") + hipGetErrorString(_e)); \
    } while (0)

#include "gf_device.h"
#include "k_butterfly.h"
#include "k_basiscvt.h"
#include "k_steps.h"
#include "k_batch.h"
#include "k_bf2.h"
#include "k_bf3.h"
#include "k_m128.h"

// ---------------------------------------------------------------------------
// elementary kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t gid() { return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return (uint64_t)gridDim.x * blockDim.x; }

// The elementary kernels below loop over their index range with the grid's
// stride, so one launch of a capped grid covers any length (a launch of more
// than 2^32 work items does not exist).

// dst[0 .. dst_words) = src bits [0, len) zero-padded
__global__ void k_load_mask(const uint64_t *__restrict__ src, uint64_t len, uint64_t *__restrict__ dst,
                            uint64_t dst_words)
{
    const uint64_t nw = (len + 63) / 64;
    for (uint64_t w = gid(); w < dst_words; w += gstride()) {
        uint64_t v = 0;
        if (w < nw) {
            v = src[w];
            if (w == nw - 1 && (len & 63)) v &= (~0ull) >> (64 - (len & 63));
        }
        dst[w] = v;
    }
}

// out[0 .. ceil(len/64)) = src bits [0, len), tail zeroed
__global__ void k_store_mask(const uint64_t *__restrict__ src, uint64_t len, uint64_t *__restrict__ out)
{
    const uint64_t nw = (len + 63) / 64;
    for (uint64_t w = gid(); w < nw; w += gstride()) {
        uint64_t v = src[w];
        if (w == nw - 1 && (len & 63)) v &= (~0ull) >> (64 - (len & 63));
        out[w] = v;
    }
}

// ---------------------------------------------------------------------------
// BasisCvt (Alg. 1) as a list of Taylor steps
//
// Alg. 1 writes f(x) = sum_j h_j(x) s^j with s = s_{2^k}(x) = x^tau + x
// (tau = 2^(2^k) the largest with tau <= deg f), converts the sequence (h_j)
// as a polynomial in y (block-vector coefficients, because X_j(s(x)) =
// X_{j 2^(2^k)}(x)), and converts each tau-bit block.  The Taylor expansion
// splits a segment of S coefficients in halves lo, hi of H = S/2 and uses
// x^H = s^(H/tau) + x^(H/tau) (Frobenius in GF(2)[x]):
//     hi[0, d) ^= hi[H-d, H);   lo[d, H) ^= hi[0, H-d);   d = H / tau,
// then recurses on both halves.  Every step is such a pair on all S-aligned
// segments; outer (block-vector) steps are the same with element size tau.
// The inverse undoes the two updates in reverse order.
// ---------------------------------------------------------------------------

struct BStep {
    uint64_t S, d;   // segment length and shift, in bits
};

static void bcvt_steps(uint64_t N, uint64_t e, std::vector<BStep> &out)
{
    if (N <= 2) return;
    uint64_t tau = 2;
    while (tau * tau > tau && tau * tau <= N / 2) tau = tau * tau;
    for (uint64_t S = N; S >= 2 * tau; S /= 2) out.push_back({S * e, (S / (2 * tau)) * e});
    bcvt_steps(N / tau, tau * e, out);   // outer conversion on tau-element blocks
    bcvt_steps(tau, e, out);             // inner conversion of each block
}

// One step with S >= 128 bits in place, as its two updates (forward: the hi
// fix first; inverse: the lo update first).  d = S / (2 tau) <= H / 2, so
// the fix writes hi[0, d) from hi[H-d, H), bits it does not write, and the
// lo update reads hi only: every word is written by one thread from words
// no thread writes in the same launch.
// hi[0, d) ^= hi[H-d, H) on every segment of words [0, nw)
__global__ void k_bcvt_wide_hi(uint64_t *__restrict__ X, uint64_t nw, uint64_t S, uint64_t d)
{
    const uint64_t SW = S / 64, HW = SW / 2, H = S / 2, dw = (d + 63) / 64, n = (nw / SW) * dw;
    for (uint64_t t = gid(); t < n; t += gstride()) {
        const uint64_t seg = t / dw, k = t - seg * dw;
        uint64_t *hp = X + seg * SW + HW;
        const int64_t rem = (int64_t)d - 64 * (int64_t)k;
        hp[k] ^= bits_at(hp, (int64_t)HW, 64 * (int64_t)k + (int64_t)(H - d)) & lowmask(rem);
    }
}

// lo[d, H) ^= hi[0, H-d) on every segment of words [0, nw)
__global__ void k_bcvt_wide_lo(uint64_t *__restrict__ X, uint64_t nw, uint64_t S, uint64_t d)
{
    const uint64_t SW = S / 64, HW = SW / 2, n = (nw / SW) * HW;
    for (uint64_t t = gid(); t < n; t += gstride()) {
        const uint64_t seg = t / HW, q = t - seg * HW;
        uint64_t *lp = X + seg * SW;
        lp[q] ^= bits_at(lp + HW, (int64_t)HW, 64 * (int64_t)q - (int64_t)d);
    }
}

// Two consecutive steps with S >= 128 bits out of place: Y = step b of
// (step a of X), word by word.  The array between the steps is read lazily
// from X (a new word depends on at most seven old ones, nearly all of them
// read by a neighbouring thread as well), so the pair costs one read and one
// write of the array where the in-place updates cost two passes of 1.5.
// nw is a multiple of both segment lengths, so every read stays in [0, nw).
__global__ void k_bcvt_wide2(const uint64_t *__restrict__ X, uint64_t *__restrict__ Y, uint64_t nw, uint64_t Sa,
                             uint64_t da, uint64_t Sb, uint64_t db, int inverse)
{
    const StepView<WordArray> va{WordArray{X}, Sa, da, inverse};
    for (uint64_t w = gid(); w < nw; w += gstride()) Y[w] = step_word(va, w, Sb, db, inverse);
}

// ---------------------------------------------------------------------------
// Encode (Alg. 4): f_i = sum_j a_{j n_p + i} r_j, the 64-bit column of bits
// (a_{j n_p + i})_j multiplied into the rows r_j by 8-bit windows
// ---------------------------------------------------------------------------

__global__ void k_encode(const uint64_t *__restrict__ bits, int l, const DevTables *__restrict__ T,
                         uint64_t *__restrict__ vals)
{
    const uint64_t n_p = 1ull << l;
    for (uint64_t i = gid(); i < n_p; i += gstride()) {
        uint64_t col = 0;
        for (int j = 0; j < 64; ++j) {
            uint64_t p = ((uint64_t)j << l) + i;
            col |= ((bits[p >> 6] >> (p & 63)) & 1ull) << j;
        }
        uint64_t f = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) f ^= T->enc_win[k][(col >> (8 * k)) & 255u];
        vals[i] = f;
    }
}

// Encode with 64 x 64 bit transposes across the wave (l >= 9): one wave per
// 8 blocks of 64 consecutive values; lane t loads the words of row t over
// their columns (one 64-byte run), and the transpose gives lane k the column
// of value k.  Rows at or above nzrows are zero and are not read.
#define ENC_NB 8
__global__ __launch_bounds__(256) void k_encode_w8(const uint64_t *__restrict__ bits, int l, int nzrows,
                                                   const DevTables *__restrict__ T, uint64_t *__restrict__ vals)
{
    __shared__ uint64_t s_win[8][256];
    for (int q = threadIdx.x; q < 8 * 256; q += blockDim.x) (&s_win[0][0])[q] = (&T->enc_win[0][0])[q];
    __syncthreads();
    const uint64_t rw = 1ull << (l - 6), ngrp = rw / ENC_NB;
    const int lane = threadIdx.x & 63;
    const uint64_t nwaves = gstride() >> 6;
    const bool live = lane < nzrows;
    for (uint64_t grp = gid() >> 6; grp < ngrp; grp += nwaves) {
        const uint64_t b0 = grp * ENC_NB;
        ulonglong2 w[ENC_NB / 2];
        const ulonglong2 *r = reinterpret_cast<const ulonglong2 *>(bits + (uint64_t)lane * rw + b0);
#pragma unroll
        for (int h = 0; h < ENC_NB / 2; ++h) w[h] = live ? r[h] : make_ulonglong2(0, 0);
#pragma unroll
        for (int bb = 0; bb < ENC_NB; ++bb) {
            const uint64_t x = (bb & 1) ? w[bb / 2].y : w[bb / 2].x;
            const uint64_t col = bc_wave_transpose64(x, lane);
            uint64_t f = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) f ^= s_win[k][(col >> (8 * k)) & 255u];
            vals[(b0 + bb) * 64 + lane] = f;
        }
    }
}

// Decode part 1: each value -> its 64 bits, in place
__global__ void k_decode_vec(uint64_t *__restrict__ vals, int l, const DevTables *__restrict__ T)
{
    for (uint64_t i = gid(); i < (1ull << l); i += gstride()) {
        uint64_t h = vals[i], a = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) a ^= T->dec_win[k][(h >> (8 * k)) & 255u];
        vals[i] = a;
    }
}

// Decode part 2: bit j of vector i goes to bit j n_p + i
__global__ void k_decode_scatter(const uint64_t *__restrict__ vecs, int l, uint64_t *__restrict__ bits)
{
    const uint64_t nw = 1ull << l;   // n / 64 words
    const uint64_t mask = (1ull << l) - 1;
    for (uint64_t W = gid(); W < nw; W += gstride()) {
        uint64_t r = 0;
        for (int t = 0; t < 64; ++t) {
            uint64_t p = 64 * W + t;
            uint64_t j = p >> l, i = p & mask;
            r |= ((vecs[i] >> j) & 1ull) << t;
        }
        bits[W] = r;
    }
}

// Decode, both parts, with wave transposes (l >= 9): R^-1 on every value,
// then the transpose gives lane t the word of row t over a block's 64
// columns; 8 blocks per wave, so every row is written as one 64-byte run
__global__ __launch_bounds__(256) void k_decode_w8(const uint64_t *__restrict__ vecs, int l,
                                                   const DevTables *__restrict__ T, uint64_t *__restrict__ bits)
{
    __shared__ uint64_t s_win[8][256];
    for (int q = threadIdx.x; q < 8 * 256; q += blockDim.x) (&s_win[0][0])[q] = (&T->dec_win[0][0])[q];
    __syncthreads();
    const uint64_t rw = 1ull << (l - 6), ngrp = rw / ENC_NB;
    const int lane = threadIdx.x & 63;
    const uint64_t nwaves = gstride() >> 6;
    for (uint64_t grp = gid() >> 6; grp < ngrp; grp += nwaves) {
        const uint64_t b0 = grp * ENC_NB;
        uint64_t r[ENC_NB];
#pragma unroll
        for (int bb = 0; bb < ENC_NB; ++bb) {
            const uint64_t v = vecs[(b0 + bb) * 64 + lane];
            uint64_t h = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) h ^= s_win[k][(v >> (8 * k)) & 255u];
            r[bb] = bc_wave_transpose64(h, lane);
        }
        ulonglong2 *w = reinterpret_cast<ulonglong2 *>(bits + (uint64_t)lane * rw + b0);
#pragma unroll
        for (int h = 0; h < ENC_NB / 2; ++h) w[h] = make_ulonglong2(r[2 * h], r[2 * h + 1]);
    }
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

struct ProfRec {
    std::string name;
    hipEvent_t start, stop;
};

#define SMALL_FIELD_DEFAULT_LOG2N 20   // m = 32 batch items: transforms up to 2^20 bits
using fpmul_plan::M64_MAX_LOG2N;               // m = 64 field bound: n <= (m/2) 2^(m/2) = 2^37
#define LARGE_FIELD_DEFAULT_LOG2N 38   // m = 128 from the first transform m = 64 cannot take

struct PStepTable;

struct polymul_ctx {
    int device = 0;
    size_t cap = 0;
    uint64_t *ws[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t ws_words = 0;   // words per workspace buffer
    DevTables *tables = nullptr;
    int num_cu = 256;
    // batch: per-size BasisCvt steps, and one allocation holding the
    // per-workgroup slabs, the queue order and the queue counter
    BatchSteps *bsteps = nullptr;
    void *bws = nullptr;
    size_t bws_bytes = 0;
    // batch items with transforms of at most 2^small_field_log2n bits run over
    // GF(2^32) (m = 32); 0 keeps every item on m = 64
    int small_field_log2n = SMALL_FIELD_DEFAULT_LOG2N;
    // workspaces lent by a server's arena: never freed or grown here
    bool borrowed = false;
    // products whose transform has at least 2^large_field_log2n bits run over
    // GF(2^128) (m = 128); above 2^37 bits m = 64 cannot take them
    int large_field_log2n = LARGE_FIELD_DEFAULT_LOG2N;
    DevTables128 *tables128 = nullptr;   // built on the first m = 128 product
    PStepTable *psteps = nullptr;        // BasisCvt step lists of the per-step path
    uint64_t *scratch = nullptr;         // device address of this GPU's `scratch` (polymul_ex_noalloc)
    // schedules of the fused path chosen by polymul_tune (or loaded from its
    // cache), by log2 of the transform length; views point at their parent's
    std::map<int, fpmul_plan::Schedule> tuned_own;
    const std::map<int, fpmul_plan::Schedule> *tuned = &tuned_own;
    // per-kernel timing with HIP events on the launch stream (off by default)
    bool prof = false;
    std::vector<ProfRec> prof_live;       // recorded, not yet read
    std::vector<hipEvent_t> prof_pool;    // free events
    std::map<std::string, std::pair<uint64_t, double>> prof_acc;   // name -> (launches, ms)
};

static hipEvent_t prof_event(polymul_ctx *c)
{
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void prof_begin(polymul_ctx *c, hipStream_t s, const char *name)
{
    if (!c || !c->prof) return;
    ProfRec r{name, prof_event(c), prof_event(c)};
    if (r.start) (void)hipEventRecord(r.start, s);
    c->prof_live.push_back(r);
}

static void prof_end(polymul_ctx *c, hipStream_t s)
{
    if (!c || !c->prof || c->prof_live.empty()) return;
    if (c->prof_live.back().stop) (void)hipEventRecord(c->prof_live.back().stop, s);
}

static void prof_collect(polymul_ctx *c)
{
    for (ProfRec &r : c->prof_live) {
        if (r.start && r.stop && hipEventSynchronize(r.stop) == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
                auto &a = c->prof_acc[r.name];
                a.first += 1;
                a.second += ms;
            }
        }
        if (r.start) c->prof_pool.push_back(r.start);
        if (r.stop) c->prof_pool.push_back(r.stop);
    }
    c->prof_live.clear();
}

// launch a kernel on stream s, timed when profiling is on; returns on error
#define KLAUNCH(ctx, s, name, kernel, grid, block, ...)        \
    do {                                                       \
        prof_begin((ctx), (s), (name));                        \
        kernel<<<(grid), (block), 0, (s)>>>(__VA_ARGS__);      \
        hipError_t _le = hipGetLastError();                    \
        prof_end((ctx), (s));                                  \
        if (_le != hipSuccess)                                 \
            return fail(POLYMUL_EIO, std::string("launch ") + (name) + ": " + hipGetErrorString(_le)); \
    } while (0)

// grid of the grid-stride elementary kernels: one item per thread up to
// 2^16 workgroups, at least one workgroup
#define GRID_CAP (1u << 16)
static unsigned grid_for(uint64_t n, unsigned bs)
{
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + bs - 1) / bs, GRID_CAP));
}

static int ensure_ws(polymul_ctx *ctx, uint64_t words)
{
    if (words <= ctx->ws_words) return 0;
    if (ctx->borrowed) return fail(POLYMUL_EIO, "borrowed workspace smaller than the launch needs");
    size_t bytes = (size_t)words * 8;
    if (ctx->cap && 4 * bytes > ctx->cap)
        return fail(POLYMUL_ENOMEM, "workspace of " + std::to_string(4 * bytes) + " bytes exceeds the cap of " +
                                        std::to_string(ctx->cap));
    for (int k = 0; k < 4; ++k) {
        if (ctx->ws[k]) { (void)hipFree(ctx->ws[k]); ctx->ws[k] = nullptr; }
    }
    ctx->ws_words = 0;
    for (int k = 0; k < 4; ++k) {
        hipError_t e = hipMalloc(&ctx->ws[k], bytes);
        if (e != hipSuccess) {
            for (int j = 0; j < 4; ++j)
                if (ctx->ws[j]) { (void)hipFree(ctx->ws[j]); ctx->ws[j] = nullptr; }
            return fail(POLYMUL_ENOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
        }
    }
    ctx->ws_words = words;
    return 0;
}

static int check_dev_ptr(const void *p, const char *name)
{
    if (!p) return fail(POLYMUL_EINVAL, std::string(name) + " is null");
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(POLYMUL_EINVAL, std::string(name) + " is not a device pointer");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(POLYMUL_EINVAL, std::string(name) + " is not device memory");
    return 0;
}

using fpmul_plan::ilog2;
using fpmul_plan::next_pow2;

// Step lists of BasisCvt(2^k) for every k <= PSTEP_MAX_LOG2N, in one device
// table built once per context: entries first[k] .. first[k] + count[k] - 1,
// with the in-word masks of the steps of at most 64 bits (BatchStep)
#define PSTEP_MAX_LOG2N 62
#define PSTEP_MAX 5120
struct PStepTable {
    BatchStep st[PSTEP_MAX];
};

struct PStepIndex {
    int first[PSTEP_MAX_LOG2N + 1];
    int count[PSTEP_MAX_LOG2N + 1];
};

static const PStepIndex &pstep_index()
{
    static const PStepIndex idx = [] {
        PStepIndex r{};
        int at = 0;
        for (int k = 0; k <= PSTEP_MAX_LOG2N; ++k) {
            std::vector<BStep> v;
            bcvt_steps(1ull << k, 1, v);
            r.first[k] = at;
            r.count[k] = (int)v.size();
            at += (int)v.size();
        }
        return r;
    }();
    return idx;
}

static int build_psteps(PStepTable &P)
{
    const PStepIndex &ix = pstep_index();
    if (ix.first[PSTEP_MAX_LOG2N] + ix.count[PSTEP_MAX_LOG2N] > PSTEP_MAX)
        return fail(POLYMUL_EIO, "BasisCvt step table overflow");
    for (int k = 0; k <= PSTEP_MAX_LOG2N; ++k) {
        std::vector<BStep> v;
        bcvt_steps(1ull << k, 1, v);
        for (size_t j = 0; j < v.size(); ++j) {
            BatchStep b{v[j].S, v[j].d, 0, 0};
            if (v[j].S <= 64) {
                const int S = (int)v[j].S, H = S / 2, d = (int)v[j].d;
                for (int t = 0; t < 64; ++t) {
                    if (t % S < H) b.L |= 1ull << t;
                    if (t % S < d) b.D |= 1ull << t;
                }
            }
            P.st[ix.first[k] + j] = b;
        }
    }
    return 0;
}

// Runs of consecutive steps whose segments fit BT_LDS_WORDS words, applied
// chunk by chunk in LDS in place (each chunk holds whole segments).  When
// the run holds BasisCvt(2^16) of every 2^16-bit block (bc16 = 1: its last
// BC16_NSTEPS steps, forward; bc16 = 2: its first BC16_NSTEPS, inverse),
// that part runs as the compile-time row conversion, whose steps within
// 1024-bit segments stay in registers.
__global__ __launch_bounds__(1024) void k_bcvt_lds_run(uint64_t *__restrict__ X, uint64_t nw, int chw,
                                                       const BatchStep *__restrict__ st0, int cnt, int inverse, int k0,
                                                       int k1, int bc16)
{
    __shared__ __align__(16) uint64_t lds[BT_LDS_WORDS];
    const int tid = threadIdx.x, nth = blockDim.x;
    for (uint64_t c0 = (uint64_t)blockIdx.x * chw; c0 < nw; c0 += (uint64_t)gridDim.x * chw) {
        for (int w = tid; w < chw; w += nth) lds[w] = X[c0 + w];
        __syncthreads();
        if (bc16 == 1) {
            bt_lds_steps(lds, chw, st0, cnt, false, k0, k1 - BC16_NSTEPS, tid, nth);
            bc16_rows<false>(lds, chw / BC_TAU_WORDS, tid, nth);
            __syncthreads();
        } else if (bc16 == 2) {
            bc16_rows<true>(lds, chw / BC_TAU_WORDS, tid, nth);
            __syncthreads();
            bt_lds_steps(lds, chw, st0, cnt, true, k0 + BC16_NSTEPS, k1, tid, nth);
        } else {
            bt_lds_steps(lds, chw, st0, cnt, inverse != 0, k0, k1, tid, nth);
        }
        for (int w = tid; w < chw; w += nth) X[c0 + w] = lds[w];
        __syncthreads();
    }
}

// run the BasisCvt steps for N bits (or their inverse) on the nw words of cur
// (nw >= N / 64), the result in cur: every run of steps with segments of at
// most 2^20 bits in one LDS pass; larger steps two at a time out of place
// between cur and spare (nw words, contents not kept) when spare is given,
// an even number of such passes so that the result ends in cur, the others
// in place as their two updates.  The callers give a spare to the inverse
// only: there a pair takes 0.9 of the time of two in-place steps, while the
// forward pair, whose lo words read the fixed hi, takes 1.02.
static int run_bcvt(polymul_ctx *ctx, uint64_t N, bool inverse, uint64_t *cur, uint64_t *spare, uint64_t nw,
                    hipStream_t s)
{
    std::vector<BStep> steps;
    bcvt_steps(N, 1, steps);
    const int cnt = (int)steps.size(), lg = ilog2(N);
    if (!cnt) return 0;
    if (lg > PSTEP_MAX_LOG2N || pstep_index().count[lg] != cnt || !ctx->psteps)
        return fail(POLYMUL_EIO, "BasisCvt step table");
    const BatchStep *st0 = ctx->psteps->st + pstep_index().first[lg];
    const uint64_t lds_bits = 64ull * BT_LDS_WORDS, chw = std::min<uint64_t>(nw, BT_LDS_WORDS);
    auto S_of = [&](int k) { return steps[inverse ? cnt - 1 - k : k].S; };
    // for N >= 2^17 the list ends with BasisCvt(2^16) of every 2^16-bit block
    bool tail16 = N >= (1ull << 17) && chw >= BC_TAU_WORDS && cnt >= BC16_NSTEPS;
    if (tail16) {
        std::vector<BStep> b16;
        bcvt_steps(1ull << 16, 1, b16);
        for (int j = 0; j < BC16_NSTEPS && tail16; ++j)
            tail16 = steps[cnt - BC16_NSTEPS + j].S == b16[j].S && steps[cnt - BC16_NSTEPS + j].d == b16[j].d;
    }
    for (int k = 0; k < cnt; ++k)
        if (S_of(k) > lds_bits && ((S_of(k) & (S_of(k) - 1)) || nw % (S_of(k) / 64)))
            return fail(POLYMUL_EIO, "BasisCvt segment beyond the array");
    // paired[k]: steps k and k + 1 run as one out-of-place pass
    std::vector<char> paired(cnt, 0);
    int npairs = 0, last = -1;
    if (spare)
        for (int k = 0; k + 1 < cnt; ++k)
            if (S_of(k) > lds_bits && S_of(k + 1) > lds_bits) { paired[k] = 1; last = k; ++npairs; ++k; }
    if (npairs & 1) paired[last] = 0;
    uint64_t *X = cur, *Y = spare;
    for (int k = 0; k < cnt;) {
        if (paired[k]) {
            const BStep &a = steps[inverse ? cnt - 1 - k : k], &b = steps[inverse ? cnt - 2 - k : k + 1];
            KLAUNCH(ctx, s, inverse ? "ibasiscvt_wide2" : "basiscvt_wide2", k_bcvt_wide2, grid_for(nw, 256), 256, X,
                    Y, nw, a.S, a.d, b.S, b.d, inverse ? 1 : 0);
            std::swap(X, Y);
            k += 2;
        } else if (S_of(k) <= lds_bits) {
            int e = k + 1;
            while (e < cnt && S_of(e) <= lds_bits) ++e;
            // forward: the run ends the list; inverse: it starts it
            int bc16 = 0;
            if (tail16 && e - k >= BC16_NSTEPS) bc16 = !inverse && e == cnt ? 1 : (inverse && k == 0 ? 2 : 0);
            const unsigned grid = (unsigned)std::min<uint64_t>(nw / chw, GRID_CAP);
            KLAUNCH(ctx, s, inverse ? "ibasiscvt_lds" : "basiscvt_lds", k_bcvt_lds_run, grid, 1024, X, nw,
                    (int)chw, st0, cnt, inverse ? 1 : 0, k, e, bc16);
            k = e;
        } else {
            const BStep &st = steps[inverse ? cnt - 1 - k : k];
            const uint64_t nhi = (nw / (st.S / 64)) * ((st.d + 63) / 64), nlo = nw / 2;
            if (!inverse)
                KLAUNCH(ctx, s, "basiscvt_wide_hi", k_bcvt_wide_hi, grid_for(nhi, 256), 256, X, nw, st.S, st.d);
            KLAUNCH(ctx, s, inverse ? "ibasiscvt_wide" : "basiscvt_wide", k_bcvt_wide_lo, grid_for(nlo, 256), 256,
                    X, nw, st.S, st.d);
            if (inverse)
                KLAUNCH(ctx, s, "ibasiscvt_wide_hi", k_bcvt_wide_hi, grid_for(nhi, 256), 256, X, nw, st.S, st.d);
            ++k;
        }
    }
    if (X != cur) return fail(POLYMUL_EIO, "BasisCvt ended in the spare buffer");
    return 0;
}

// The forward steps of an operand of N = 2^k >= len bits touch its first N
// bits only (every segment of a step lies inside them), so they run on those
// words; the rest of both buffers is zero.
static uint64_t bcvt_active_words(uint64_t N, uint64_t nw) { return std::max<uint64_t>(1, std::min(nw, N / 64)); }

// A (len bits) -> BasisCvt -> Encode: n_p values in *cur (cur/spare swapped as needed)
static int run_encode_in(polymul_ctx *ctx, const uint64_t *a, uint64_t len, int log2n, uint64_t *&cur,
                         uint64_t *&spare, hipStream_t s)
{
    const int l = log2n - 6;
    const uint64_t nw = 1ull << l, n_p = 1ull << l, N = next_pow2(std::max<uint64_t>(len, 1));
    const uint64_t nwa = bcvt_active_words(N, nw);
    const unsigned bs = 256;
    KLAUNCH(ctx, s, "load", k_load_mask, grid_for(nw, bs), bs, a, len, cur, nw);
    int rc = run_bcvt(ctx, N, false, cur, nullptr, nwa, s);
    if (rc) return rc;
    if (l >= 9) {
        // rows at or above ceil(N / n_p) hold no bit of the operand
        const int nz = (int)std::min<uint64_t>(64, (N + n_p - 1) / n_p);
        KLAUNCH(ctx, s, "encode", k_encode_w8, grid_for(n_p / ENC_NB, bs), bs, cur, l, nz, ctx->tables, spare);
    } else
        KLAUNCH(ctx, s, "encode", k_encode, grid_for(n_p, bs), bs, cur, l, ctx->tables, spare);
    std::swap(cur, spare);
    return 0;
}

// values in *cur (destroyed) -> Decode -> iBasisCvt: n bits in *cur
static int run_decode_out(polymul_ctx *ctx, int log2n, uint64_t *&cur, uint64_t *&spare, hipStream_t s)
{
    const int l = log2n - 6;
    const uint64_t nw = 1ull << l, n_p = 1ull << l;
    const unsigned bs = 256;
    if (l >= 9) {
        KLAUNCH(ctx, s, "decode", k_decode_w8, grid_for(nw / ENC_NB, bs), bs, cur, l, ctx->tables, spare);
    } else {
        KLAUNCH(ctx, s, "decode_vec", k_decode_vec, grid_for(n_p, bs), bs, cur, l, ctx->tables);
        KLAUNCH(ctx, s, "decode_scatter", k_decode_scatter, grid_for(nw, bs), bs, cur, l, spare);
    }
    std::swap(cur, spare);
    return run_bcvt(ctx, 1ull << log2n, true, cur, spare, nw, s);
}

// the layers above the bottom tile, as (i_lo, k) groups of at most BF_UPPER_MAXK, lowest first
static std::vector<std::pair<int, int>> upper_groups(int l, int R)
{
    std::vector<std::pair<int, int>> g;
    int U = l - R;
    if (U <= 0) return g;
    int ng = (U + BF_UPPER_MAXK - 1) / BF_UPPER_MAXK, base = U / ng, extra = U % ng, lo = R;
    for (int q = 0; q < ng; ++q) {
        int k = base + (q < extra ? 1 : 0);
        g.push_back({lo, k});
        lo += k;
    }
    return g;
}

// the schedule of transforms of 2^log2n bits: the tuned one, else the default
static fpmul_plan::Schedule sched_of(const polymul_ctx *ctx, int log2n)
{
    if (ctx->tuned) {
        auto it = ctx->tuned->find(log2n);
        if (it != ctx->tuned->end()) return it->second;
    }
    return fpmul_plan::Schedule();
}

// the resident-table upper passes of a 2^l-value transform as (i_lo, k), lowest first
static std::vector<std::pair<int, int>> upper_groups_of(const polymul_ctx *ctx, int l)
{
    const fpmul_plan::Schedule sc = sched_of(ctx, l + 6);
    if (sc.upper.empty() || !fpmul_plan::upper_valid(l, sc.upper)) return upper_groups(l, B3_BOT_LAYERS);
    std::vector<std::pair<int, int>> g;
    int lo = fpmul_plan::bottom_layers(l, sc.upper);   // the lowest upper pass starts above the bottom pass
    for (int k : sc.upper) {
        g.push_back({lo, k});
        lo += k;
    }
    return g;
}

static int set_lds_limits()
{
    static std::mutex mu;
    static int done = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (done) return 0;
    const int big = 160 * 1024;
    HIP_TRY(hipFuncSetAttribute((const void *)k_bfly_bottom<BF_FWD>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
    HIP_TRY(hipFuncSetAttribute((const void *)k_bfly_bottom<BF_INV>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
    HIP_TRY(hipFuncSetAttribute((const void *)k_bfly_bottom<BF_PRODUCT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                big));
    // k_batch also has static LDS, so its dynamic limit is exactly what it uses
    HIP_TRY(hipFuncSetAttribute((const void *)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bf_bottom_lds(BF_BOTTOM_R, true)));
    done = 1;
    return 0;
}

#define KLAUNCH_LDS(ctx, s, name, kernel, grid, block, lds, ...)                                   \
    do {                                                                                           \
        prof_begin((ctx), (s), (name));                                                            \
        kernel<<<(grid), (block), (lds), (s)>>>(__VA_ARGS__);                                      \
        hipError_t _le = hipGetLastError();                                                        \
        prof_end((ctx), (s));                                                                      \
        if (_le != hipSuccess)                                                                     \
            return fail(POLYMUL_EIO, std::string("launch ") + (name) + ": " + hipGetErrorString(_le)); \
    } while (0)

// upper layer group [i_lo, i_lo + k) with the register-resident passes

// upper pass of K = k layers with resident tables: one workgroup per CU, the
// grid split between the operands when B is given
template <bool INV>
static int launch_bf3_upper(polymul_ctx *ctx, hipStream_t s, const char *name, uint64_t *A, uint64_t *B, int l,
                            int i_lo, int k)
{
    const uint64_t nops = B ? 2 : 1, ntiles = 1ull << (l - B3_TILE_LG);
    const uint64_t per_op = std::max<uint64_t>(1, std::min<uint64_t>(ntiles, (uint64_t)ctx->num_cu / nops));
    const unsigned grid = (unsigned)(per_op * nops);
    void (*kern)(uint64_t *, uint64_t *, int, int, const DevTables *) = nullptr;
    switch (k) {
    case 1: kern = k_bf3_upper<INV, 1>; break;
    case 2: kern = k_bf3_upper<INV, 2>; break;
    case 3: kern = k_bf3_upper<INV, 3>; break;
    case 4: kern = k_bf3_upper<INV, 4>; break;
    case 5: kern = k_bf3_upper<INV, 5>; break;
    case 6: kern = k_bf3_upper<INV, 6>; break;
    case 7: kern = k_bf3_upper<INV, 7>; break;
    default: return fail(POLYMUL_EINVAL, "upper layer group of more than 7 layers");
    }
    if (l < B3_TILE_LG || i_lo + k > l || i_lo < B3_TILE_LG - k)
        return fail(POLYMUL_EINVAL, "upper pass does not fit the tile geometry");
    KLAUNCH(ctx, s, name, kern, grid, B3_THREADS, A, B, l, i_lo, ctx->tables);
    return 0;
}

#define BF3_MIN_L 20    // resident-table bottom pass from 2^20 transform values
using fpmul_plan::SINGLE_VIA_BATCH_LOG2N;   // polymul_ex of products up to 2^16 bits runs as a one-item batch

// the bottom pass of layers 0 .. nl - 1 (nl = 6 or 7)
template <bool INV>
static int launch_bf3_bottom(polymul_ctx *ctx, hipStream_t s, const char *name, uint64_t *A, uint64_t *B, int l,
                             int nl)
{
    const uint64_t nops = B ? 2 : 1, ntiles = 1ull << (l - B3_TILE_LG);
    const uint64_t per_op = std::max<uint64_t>(1, std::min<uint64_t>(ntiles, (uint64_t)ctx->num_cu / nops));
    if (l < B3_TILE_LG) return fail(POLYMUL_EINVAL, "bottom pass needs at least one tile");
    if (nl == 7)
        KLAUNCH(ctx, s, name, (k_bf3_bottom<INV, 7>), (unsigned)(per_op * nops), B3_THREADS, A, B, l, ctx->tables);
    else if (nl == 6)
        KLAUNCH(ctx, s, name, (k_bf3_bottom<INV, 6>), (unsigned)(per_op * nops), B3_THREADS, A, B, l, ctx->tables);
    else
        return fail(POLYMUL_EINVAL, "bottom pass of 6 or 7 layers");
    return 0;
}

// Butterflies of one transform (mode BF_FWD or BF_INV) or of a product
// (BF_PRODUCT: forward A and B, pointwise, inverse; result in A).  Large
// transforms: upper passes down to layer 7, then the bottom pass of layers
// 0 .. 6, all with resident K tables.  Smaller ones: upper passes down to
// layer 11 and the 2^11-value bottom pass (more tiles to spread).
static int run_butterflies(polymul_ctx *ctx, int mode, uint64_t *A, uint64_t *B, int l, hipStream_t s)
{
    const uint64_t n = 1ull << l;
    if (l >= BF3_MIN_L) {
        // the layers above the bottom pass split into passes of at most 7
        // (evenly by default, or the tuned split); the bottom pass has 7
        // layers, or 6 under a split that gives layer 6 to the lowest upper
        // pass, which needs K >= 12 - i_lo (every split for l >= 20 allows one)
        const auto groups = upper_groups_of(ctx, l);
        const int nl = groups.empty() ? B3_BOT_LAYERS : groups.front().first;   // layers of the bottom pass
        int rc;
        if (mode != BF_INV) {
            for (auto it = groups.rbegin(); it != groups.rend(); ++it)
                if ((rc = launch_bf3_upper<false>(ctx, s, "butterfly_upper", A, mode == BF_PRODUCT ? B : nullptr, l,
                                                  it->first, it->second)))
                    return rc;
            if ((rc = launch_bf3_bottom<false>(ctx, s, "butterfly_bottom", A, mode == BF_PRODUCT ? B : nullptr, l,
                                               nl)))
                return rc;
        }
        if (mode == BF_PRODUCT)
            KLAUNCH(ctx, s, "pointwise", k_pointwise,
                    (unsigned)std::min<uint64_t>((n + 1023) / 1024, (uint64_t)ctx->num_cu), 1024, A, B, n,
                    ctx->tables);
        if (mode != BF_FWD) {
            if ((rc = launch_bf3_bottom<true>(ctx, s, "ibutterfly_bottom", A, nullptr, l, nl))) return rc;
            for (auto it = groups.begin(); it != groups.end(); ++it)
                if ((rc = launch_bf3_upper<true>(ctx, s, "ibutterfly_upper", A, nullptr, l, it->first, it->second)))
                    return rc;
        }
        return 0;
    }
    const int R = std::min(l, BF_BOTTOM_R);
    const auto groups = upper_groups(l, R);
    const dim3 blk(BF_THREADS);
    const uint64_t persist_bot = (uint64_t)ctx->num_cu;
    if (mode != BF_INV) {
        for (auto it = groups.rbegin(); it != groups.rend(); ++it) {
            const int i_lo = it->first, k = it->second;
            const int rc = launch_bf3_upper<false>(ctx, s, "butterfly_upper", A, mode == BF_PRODUCT ? B : nullptr,
                                                   l, i_lo, k);
            if (rc) return rc;
        }
    }
    if (l >= B2_TILE_LG) {
        // register-resident bottom passes; the pointwise step in between
        const unsigned bt = (unsigned)std::min<uint64_t>(1ull << (l - B2_TILE_LG), (uint64_t)ctx->num_cu * 2);
        if (mode == BF_PRODUCT) {
            KLAUNCH(ctx, s, "butterfly_bottom", k_bf2_bottom<BF_FWD>, dim3(bt, 2), B2_THREADS, A, B, l, ctx->tables);
            KLAUNCH(ctx, s, "pointwise", k_pointwise, (unsigned)std::min<uint64_t>((n + 1023) / 1024,
                                                                                   (uint64_t)ctx->num_cu),
                    1024, A, B, n, ctx->tables);
            KLAUNCH(ctx, s, "ibutterfly_bottom", k_bf2_bottom<BF_INV>, bt, B2_THREADS, A, B, l, ctx->tables);
        } else if (mode == BF_FWD) {
            KLAUNCH(ctx, s, "butterfly_bottom", k_bf2_bottom<BF_FWD>, bt, B2_THREADS, A, B, l, ctx->tables);
        } else {
            KLAUNCH(ctx, s, "ibutterfly_bottom", k_bf2_bottom<BF_INV>, bt, B2_THREADS, A, B, l, ctx->tables);
        }
    } else {
        const unsigned bt = (unsigned)std::min<uint64_t>(1ull << (l - R), persist_bot);
        if (mode == BF_PRODUCT)
            KLAUNCH_LDS(ctx, s, "butterfly_bottom_product", k_bfly_bottom<BF_PRODUCT>, bt, blk, bf_bottom_lds(R, true),
                        A, B, l, R, ctx->tables);
        else if (mode == BF_FWD)
            KLAUNCH_LDS(ctx, s, "butterfly_bottom", k_bfly_bottom<BF_FWD>, bt, blk, bf_bottom_lds(R, false), A, B, l,
                        R, ctx->tables);
        else
            KLAUNCH_LDS(ctx, s, "ibutterfly_bottom", k_bfly_bottom<BF_INV>, bt, blk, bf_bottom_lds(R, false), A, B, l,
                        R, ctx->tables);
    }
    if (mode != BF_FWD) {
        for (auto it = groups.begin(); it != groups.end(); ++it) {
            const int rc = launch_bf3_upper<true>(ctx, s, "ibutterfly_upper", A, nullptr, l, it->first, it->second);
            if (rc) return rc;
        }
    }
    return 0;
}

using fpmul_plan::product_log2n;

static int transform_log2(uint64_t len_a, uint64_t len_b) { return product_log2n(len_a + len_b - 1); }

static int ranges_overlap(const void *a, size_t an, const void *b, size_t bn)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

// makes ctx's device current for a scope and restores the caller's device
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// ---------------------------------------------------------------------------
// fast BasisCvt + Encode / Decode + iBasisCvt (k_basiscvt.h), 2^22 <= n <= 2^31
// ---------------------------------------------------------------------------

using fpmul_plan::fast_path;

static BcSteps make_steps(uint64_t N)
{
    std::vector<BStep> v;
    bcvt_steps(N, 1, v);
    BcSteps st;
    std::memset(&st, 0, sizeof st);
    st.n = (int)v.size();
    for (size_t k = 0; k < v.size() && k < BC_MAX_STEPS; ++k) {
        const int S = (int)v[k].S, d = (int)v[k].d, H = S / 2;
        st.lgS[k] = (uint8_t)ilog2(v[k].S);
        st.lgd[k] = (uint8_t)ilog2(v[k].d);
        uint64_t L = 0, D = 0;
        if (S <= 64)
            for (int b = 0; b < 64; ++b) {
                int r = b % S;
                if (r < H) L |= 1ull << b;
                if (r < d) D |= 1ull << b;
            }
        st.L[k] = L;
        st.D[k] = D;
    }
    return st;
}

// the step lists of BasisCvt(2^lg) for the fused path's inner (2^16) and
// outer (up to 2^15 rows) conversions, built once: a list takes a few
// microseconds of host time, and a product needs four
static const BcSteps &steps_of(int lg)
{
    static const std::vector<BcSteps> all = [] {
        std::vector<BcSteps> v(17);
        for (int k = 0; k <= 16; ++k) v[k] = make_steps(1ull << k);
        return v;
    }();
    return all[lg];
}

using fpmul_plan::bc_ew;
using fpmul_plan::ws_words_for;
static_assert(fpmul_plan::TAU_WORDS == BC_TAU_WORDS, "row length of the fused BasisCvt");

// rows per workgroup iteration of the row kernels: BC_ROWS (the fast path)
// while that still gives every CU a workgroup, fewer for shorter operands
static int rows_per_wg(const polymul_ctx *ctx, int lgR)
{
    int rpw = BC_ROWS;
    while (rpw > 1 && ((1ull << lgR) / rpw) < (uint64_t)ctx->num_cu) rpw /= 2;
    return rpw;
}

// the superset sums of one operand (X, in, len), or of two of the same row
// count in the same launches (the second as X1, in1, len1; grid y = operand)
static int run_zeta(polymul_ctx *ctx, hipStream_t s, uint64_t *X, const uint64_t *in, uint64_t len, int lgR, int EW,
                    bool skew_first, int zeta_mult, uint64_t *X1 = nullptr, const uint64_t *in1 = nullptr,
                    uint64_t len1 = 0)
{
    const unsigned ny = X1 ? 2 : 1;
    // two passes of 6 .. 8 row bits where they cover lgR (12 .. 16), both on
    // the register-tile kernel; else up to 8 bits and the rest
    const int nb1 = lgR >= 12 ? std::min(8, lgR - 6) : std::min(lgR, 8), nb2 = lgR - nb1;
    for (int pass = 0; pass < 2; ++pass) {
        const int b0 = pass ? nb1 : 0, nb = pass ? nb2 : nb1;
        if (nb <= 0) continue;
        // 2^nb rows x 2^lgWc words fill the tile; with nb <= 8 a row segment is
        // at least 16 words (128 bytes, one full line)
        const int lgWc = std::min(6, 12 - nb);
        if ((1 << (nb + lgWc)) > BC_ZETA_LDS) return fail(POLYMUL_EINVAL, "zeta tile exceeds LDS");
        const uint64_t tiles = (1ull << (lgR - nb)) * (uint64_t)(EW >> lgWc);
        const unsigned grid = (unsigned)std::min<uint64_t>(tiles, (uint64_t)ctx->num_cu * zeta_mult);
        const char *name = skew_first ? "basiscvt_zeta" : "ibasiscvt_zeta";
        const int skew = (pass == 0 && skew_first && in) ? 1 : 0;
        if (nb >= 6 && nb <= 8 && (EW % (1 << (12 - nb))) == 0) {
            // register-resident tiles of 2^12 words
            const uint64_t rt = (1ull << (lgR - nb)) * (uint64_t)(EW >> (12 - nb));
            const unsigned g = (unsigned)std::min<uint64_t>(rt, (uint64_t)ctx->num_cu * zeta_mult);
            if (nb == 8)
                KLAUNCH(ctx, s, name, k_bc_zeta_r<8>, dim3(g, ny), 256, X, in, len, lgR, EW, b0, skew, X1, in1, len1);
            else if (nb == 7)
                KLAUNCH(ctx, s, name, k_bc_zeta_r<7>, dim3(g, ny), 256, X, in, len, lgR, EW, b0, skew, X1, in1, len1);
            else
                KLAUNCH(ctx, s, name, k_bc_zeta_r<6>, dim3(g, ny), 256, X, in, len, lgR, EW, b0, skew, X1, in1, len1);
            continue;
        }
        if (nb <= 3 && !skew) {
            // one word position of 2^nb rows per thread, no tile (for the
            // skewed first pass of short operands the LDS tiles are faster:
            // 2^21 x 2^21 bits 0.129 ms against 0.133)
            const uint64_t groups = (1ull << (lgR - nb)) * (uint64_t)EW;
            const unsigned gs = (unsigned)std::min<uint64_t>((groups + 255) / 256, (uint64_t)ctx->num_cu * zeta_mult);
            if (nb == 1)
                KLAUNCH(ctx, s, name, k_bc_zeta_s<1>, dim3(gs, ny), 256, X, lgR, EW, b0, X1);
            else if (nb == 2)
                KLAUNCH(ctx, s, name, k_bc_zeta_s<2>, dim3(gs, ny), 256, X, lgR, EW, b0, X1);
            else
                KLAUNCH(ctx, s, name, k_bc_zeta_s<3>, dim3(gs, ny), 256, X, lgR, EW, b0, X1);
            continue;
        }
        KLAUNCH(ctx, s, name, k_bc_zeta, dim3(grid, ny), BC_THREADS, X, in, len, lgR, EW, b0, nb, lgWc, skew, X1, in1,
                len1);
    }
    return 0;
}

// workgroups of k_square for n values: eight per CU (16 KiB of LDS each),
// fewer for short transforms
static unsigned square_grid(const polymul_ctx *ctx, uint64_t n)
{
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + SQ_THREADS - 1) / SQ_THREADS,
                                                              (uint64_t)ctx->num_cu * 8));
}

// rows of 2^16 bits in the fused BasisCvt of a len-bit operand: 2^lgR
static int bc_lgR(uint64_t len)
{
    const uint64_t N = next_pow2(std::max<uint64_t>(len, 1));
    return N <= (1ull << 16) ? 0 : ilog2(N) - 16;
}

// one operand of the fused forward steps: its bits, the transform values
// out (2^(log2n-6) words) and the scratch X (skewed rows), Y (columns)
struct EncOp {
    const uint64_t *a;
    uint64_t len;
    uint64_t *vals, *X, *Y;
};

// operand (len bits) -> BasisCvt -> Encode -> vals; with B as well (same row
// count), both operands go through the same launches, one per grid row y
static int run_encode_fast(polymul_ctx *ctx, const EncOp &A, const EncOp *B, int log2n, hipStream_t s)
{
    const int l = log2n - 6;
    const int lgR = bc_lgR(A.len);
    if (B && bc_lgR(B->len) != lgR) return fail(POLYMUL_EIO, "operands of one launch differ in row count");
    const unsigned ny = B ? 2 : 1;
    const EncOp &B1 = B ? *B : A;   // a valid second set of arguments, unused when ny = 1
    const int EW = bc_ew(lgR);
    const fpmul_plan::Schedule sc = sched_of(ctx, log2n);
    if (lgR >= 1) {
        int rc = run_zeta(ctx, s, A.X, A.a, A.len, lgR, EW, true, sc.zeta_mult, B ? B->X : nullptr,
                          B ? B->a : nullptr, B ? B->len : 0);
        if (rc) return rc;
    }
    const BcSteps &inner = steps_of(16), &outer = steps_of(lgR);
    const int rpw = rows_per_wg(ctx, lgR);
    const unsigned grows = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((1ull << lgR) / rpw,
                                                                              (uint64_t)ctx->num_cu * sc.rows_mult));
    KLAUNCH(ctx, s, "basiscvt_rows", k_bc_fwd_rows, dim3(grows, ny), BC_ROW_THREADS, A.X, A.a, A.len, lgR, EW, A.Y,
            inner, rpw, B1.X, B1.a, B1.len, B1.Y);
    // short columns: the compact kernel, four workgroups per CU
    if (lgR <= BC_ENC_SMALL_LG)
        KLAUNCH(ctx, s, "basiscvt_outer_encode", (k_bc_outer_encode<2, BC_ENC_SMALL_LG, 4, 4>),
                dim3((unsigned)std::min(BC_TAU_WORDS, 4 * ctx->num_cu), ny), 256, A.Y, lgR, l, A.vals, outer,
                ctx->tables, B1.Y, B1.vals);
    else
        KLAUNCH(ctx, s, "basiscvt_outer_encode", (k_bc_outer_encode<4, 14, BC_ENC_PRE, 1>),
                dim3((unsigned)std::min(BC_TAU_WORDS, ctx->num_cu), ny), BC_COL_THREADS, A.Y, lgR, l, A.vals, outer,
                ctx->tables, B1.Y, B1.vals);
    return 0;
}

static int run_encode_fast(polymul_ctx *ctx, const uint64_t *a, uint64_t len, int log2n, uint64_t *vals,
                           uint64_t *X, uint64_t *Y, hipStream_t s)
{
    const EncOp A{a, len, vals, X, Y};
    return run_encode_fast(ctx, A, nullptr, log2n, s);
}

// vals (destroyed? no: read only) -> Decode -> iBasisCvt -> out (len bits)
static int run_decode_fast(polymul_ctx *ctx, const uint64_t *vals, int log2n, uint64_t *out, uint64_t len,
                           uint64_t *X, uint64_t *Y, hipStream_t s)
{
    const int l = log2n - 6, lgR = log2n - 16, EW = bc_ew(lgR);
    const fpmul_plan::Schedule sc = sched_of(ctx, log2n);
    const BcSteps &inner = steps_of(16), &outer = steps_of(lgR);
    if (lgR <= BC_DEC_SMALL_LG)
        KLAUNCH(ctx, s, "decode_outer", (k_bc_decode_outer<2, BC_DEC_SMALL_LG, 4, 4>),
                (unsigned)std::min(2 * BC_TAU_WORDS, 4 * ctx->num_cu), 256, vals, lgR, l,
                reinterpret_cast<uint32_t *>(Y), outer, ctx->tables);
    else
        KLAUNCH(ctx, s, "decode_outer", (k_bc_decode_outer<4, 15, BC_DEC_PRE, 1>),
                (unsigned)std::min(2 * BC_TAU_WORDS, ctx->num_cu), BC_COL_THREADS, vals, lgR, l,
                reinterpret_cast<uint32_t *>(Y), outer, ctx->tables);
    // four times the forward grid (capped at one row group per workgroup):
    // for the 2^31-bit product 383 us with the forward grid, 366 with twice
    // it, 345 with four times
    const int rpw = rows_per_wg(ctx, lgR);
    const unsigned grows = (unsigned)std::min<uint64_t>((1ull << lgR) / rpw, (uint64_t)ctx->num_cu * sc.rows_mult * 4);
    KLAUNCH(ctx, s, "ibasiscvt_rows", k_bc_inv_rows, grows, BC_ROW_THREADS, reinterpret_cast<const uint32_t *>(Y), lgR,
            EW, X, inner, rpw);
    int rc = run_zeta(ctx, s, X, nullptr, 0, lgR, EW, false, sc.zeta_mult);
    if (rc) return rc;
    // a row per workgroup iteration; 16 workgroups per CU keep enough rows in
    // flight to stream (4 per CU: 156 us, 16: 137 us for the 2^31-bit product)
    KLAUNCH(ctx, s, "ibasiscvt_store", k_bc_inv_store, (unsigned)std::min<uint64_t>(1ull << lgR,
                                                                                    (uint64_t)ctx->num_cu * 16),
            BC_THREADS, X, lgR, EW, len, out);
    return 0;
}

static int batch_steps_upload(polymul_ctx *ctx);

// ---------------------------------------------------------------------------
// m = 128 products (k_m128.h): per-step BasisCvt, Encode over GF(2^128), one
// launch per butterfly layer (both operands together), pointwise, the inverse
// layers, Decode, per-step iBasisCvt
// ---------------------------------------------------------------------------

static int ensure_tables128(polymul_ctx *ctx)
{
    if (ctx->tables128) return 0;
    std::unique_ptr<fpmul_host::Tables> H(new fpmul_host::Tables());
    std::unique_ptr<fpmul_host::Tables128> H2(new fpmul_host::Tables128());
    std::unique_ptr<DevTables128> D(new DevTables128());
    try {
        fpmul_host::build_tables(*H);
        fpmul_host::build_tables128(*H, *H2);
    } catch (const std::exception &ex) {
        return fail(POLYMUL_EIO, std::string("m = 128 constant tables: ") + ex.what());
    }
    for (int k = 0; k < 8; ++k)
        for (int e = 0; e < 256; ++e) {
            uint64_t f = 0, a = 0;
            for (int t = 0; t < 8; ++t)
                if ((e >> t) & 1) {
                    f ^= H2->enc[8 * k + t];
                    a ^= H2->dec[8 * k + t];
                }
            D->enc_win[k][e] = f;
            D->dec_win[k][e] = a;
        }
    for (int d = 0; d < M128_MAXD; ++d) D->lo[d] = H2->v[64 + d].lo;
    for (int d = 0; d <= 32; ++d)
        for (int t = 0; t < 64; ++t) D->gbase[d][t] = H->tw.m64(H2->v[64 + d].lo, 1ull << t);
    static_assert(sizeof(D->ktab) == sizeof(H2->ktab), "window table layout");
    std::memcpy(D->ktab, H2->ktab, sizeof(D->ktab));
    DevTables128 *dev = nullptr;
    hipError_t e = hipMalloc(&dev, sizeof(DevTables128));
    if (e == hipSuccess) e = hipMemcpy(dev, D.get(), sizeof(DevTables128), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (dev) (void)hipFree(dev);
        return fail(POLYMUL_EIO, std::string("upload m = 128 tables: ") + hipGetErrorString(e));
    }
    ctx->tables128 = dev;
    return 0;
}

// A (len bits) -> BasisCvt -> Encode over GF(2^128): 2^(log2n-7) values in dst
static int run_encode128(polymul_ctx *ctx, const uint64_t *src, uint64_t len, int log2n, uint64_t *dst,
                         uint64_t *spare, hipStream_t s)
{
    const int l = log2n - 7;
    const uint64_t nw = 1ull << (log2n - 6), n_p = 1ull << l, N = next_pow2(std::max<uint64_t>(len, 1));
    uint64_t *cur = spare;
    KLAUNCH(ctx, s, "load", k_load_mask, grid_for(nw, 256), 256, src, len, cur, nw);
    int rc = run_bcvt(ctx, N, false, cur, nullptr, bcvt_active_words(N, nw), s);
    if (rc) return rc;
    if (l >= 9) {
        // rows at or above ceil(N / n_p) hold no bit of the operand
        const int nz = (int)std::min<uint64_t>(128, (N + n_p - 1) / n_p);
        KLAUNCH(ctx, s, "encode128", k_encode128_w8, grid_for(n_p / M128_NB, 256), 256, cur, l, nz,
                ctx->tables128, dst);
    } else
        KLAUNCH(ctx, s, "encode128", k_encode128, grid_for(n_p, 256), 256, cur, l, ctx->tables128, dst);
    return 0;
}

// forward layers of A and B, pointwise, inverse layers: the product's values in A
static int run_product128(polymul_ctx *ctx, uint64_t *A, uint64_t *B, int l, hipStream_t s)
{
    const uint64_t n_p = 1ull << l;
    const uint64_t wgs = std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->num_cu, (n_p + 1023) / 1024));
    // layer groups: for 12 <= l <= 32 triples (i + 2, i + 1, i) from the top
    // (the three-layer kernel needs i >= 4), pairs down to layer 3, then layers
    // 2, 1, 0 in one pass; otherwise from the top greedily pairs (i >= 3,
    // l >= 11, l - i <= 32) and single layers
    std::vector<std::pair<int, int>> plan;   // (lowest layer, layers)
    if (l >= 12 && l <= 32) {
        // layers 3 .. l - 1: triples from the top, then 1 to 3 pairs (a
        // triple's lowest layer must be >= 4), no single layer; then 2, 1, 0
        const int U = l - 3;
        const int np = (2 * U) % 3 == 0 ? 3 : (2 * U) % 3;
        int i = l - 1;
        for (int t = 0; t < (U - 2 * np) / 3; ++t, i -= 3) plan.push_back({i - 2, 3});
        for (int t = 0; t < np; ++t, i -= 2) plan.push_back({i - 1, 2});
        if (i != 2) return fail(POLYMUL_EIO, "m = 128 layer grouping");
        plan.push_back({0, 3});
    }
    for (int i = plan.empty() ? l - 1 : -1; i >= 0;) {
        if (i - 2 >= 4 && l >= 12 && l - (i - 2) <= 32) {
            plan.push_back({i - 2, 3});
            i -= 3;
        } else if (i - 1 >= 3 && l >= 11 && l - (i - 1) <= 32) {
            plan.push_back({i - 1, 2});
            i -= 2;
        } else {
            plan.push_back({i, 1});
            i -= 1;
        }
    }
    const unsigned low_grid = (unsigned)ctx->num_cu;
    for (const auto &p : plan) {
        if (p.second == 3 && p.first == 0)
            KLAUNCH(ctx, s, "butterfly128", k_bfly128_low3<false>, low_grid, M128_LOW_THREADS, A, B, l,
                    ctx->tables, ctx->tables128);
        else if (p.second == 3)
            KLAUNCH(ctx, s, "butterfly128", k_bfly128_3layer<false>, (unsigned)ctx->num_cu, M128_TILE2, A, B, l,
                    p.first, ctx->tables, ctx->tables128);
        else if (p.second == 2)
            KLAUNCH(ctx, s, "butterfly128", k_bfly128_2layer<false>, (unsigned)ctx->num_cu, M128_TILE2, A, B, l,
                    p.first, ctx->tables, ctx->tables128);
        else
            KLAUNCH(ctx, s, "butterfly128", k_bfly128_layer<false>, (unsigned)wgs, 1024, A, B, l, p.first,
                    ctx->tables, ctx->tables128);
    }
    KLAUNCH(ctx, s, "pointwise128", k_pointwise128, (unsigned)wgs, 1024, A, B, n_p, ctx->tables, ctx->tables128);
    for (auto it = plan.rbegin(); it != plan.rend(); ++it) {
        if (it->second == 3 && it->first == 0)
            KLAUNCH(ctx, s, "ibutterfly128", k_bfly128_low3<true>, low_grid, M128_LOW_THREADS, A, nullptr, l,
                    ctx->tables, ctx->tables128);
        else if (it->second == 3)
            KLAUNCH(ctx, s, "ibutterfly128", k_bfly128_3layer<true>, (unsigned)ctx->num_cu, M128_TILE2, A, nullptr,
                    l, it->first, ctx->tables, ctx->tables128);
        else if (it->second == 2)
            KLAUNCH(ctx, s, "ibutterfly128", k_bfly128_2layer<true>, (unsigned)ctx->num_cu, M128_TILE2, A, nullptr,
                    l, it->first, ctx->tables, ctx->tables128);
        else
            KLAUNCH(ctx, s, "ibutterfly128", k_bfly128_layer<true>, (unsigned)wgs, 1024, A, nullptr, l, it->first,
                    ctx->tables, ctx->tables128);
    }
    return 0;
}

static int product128_body(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                           uint64_t *out, hipStream_t s)
{
    const uint64_t lc = len_a + len_b - 1;
    const int log2n = fpmul_plan::product128_log2n(lc), l = log2n - 7;
    const uint64_t nw = 1ull << (log2n - 6);
    if (ctx->ws_words < nw) return fail(POLYMUL_EIO, "m = 128 product: workspace smaller than its transform");
    int rc;
    if ((rc = ensure_tables128(ctx))) return rc;
    uint64_t *W0 = ctx->ws[0], *W1 = ctx->ws[1], *W2 = ctx->ws[2];
    if ((rc = run_encode128(ctx, a, len_a, log2n, W0, W2, s))) return rc;
    if ((rc = run_encode128(ctx, b, len_b, log2n, W1, W2, s))) return rc;
    if ((rc = run_product128(ctx, W0, W1, l, s))) return rc;
    if (l >= 9) {
        KLAUNCH(ctx, s, "decode128", k_decode128_w8, grid_for(nw / 2 / M128_NB, 256), 256, W0, l, ctx->tables128, W1);
    } else {
        KLAUNCH(ctx, s, "decode128_vec", k_decode128_vec, grid_for(nw, 256), 256, W0, nw, ctx->tables128);
        KLAUNCH(ctx, s, "decode128_scatter", k_decode128_scatter, grid_for(nw, 256), 256, W0, l, W1);
    }
    if ((rc = run_bcvt(ctx, 1ull << log2n, true, W1, W0, nw, s))) return rc;
    KLAUNCH(ctx, s, "store", k_store_mask, grid_for((lc + 63) / 64, 256), 256, W1, lc, out);
    return 0;
}

static int product_body(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                        uint64_t *out, hipStream_t s)
{
    const uint64_t lc = len_a + len_b - 1;
    const int log2n = transform_log2(len_a, len_b);
    // the workspace of either route, sized by the rule the server's admission uses too
    int rc = ensure_ws(ctx, fpmul_plan::product_ws_words(len_a, len_b, ctx->large_field_log2n));
    if (rc) return rc;
    if (fpmul_plan::routes_m128(lc, ctx->large_field_log2n)) return product128_body(ctx, a, len_a, b, len_b, out, s);
    if ((rc = set_lds_limits())) return rc;
    uint64_t *W0 = ctx->ws[0], *W1 = ctx->ws[1], *W2 = ctx->ws[2], *W3 = ctx->ws[3];
    uint64_t *pa, *pb;
    // a square (the same operand twice): one forward transform, squared
    // pointwise (Alg. 5 with both transforms equal)
    const bool square = a == b && len_a == len_b;
    // forward transforms of A into W0, of B into W1.  Operands of one row
    // count share each launch, their skewed rows in W0 and W1 (free until
    // Encode writes the values there) and their columns in W2 and W3; else
    // one after the other with W2, W3 as scratch.
    const bool paired = !square && fast_path(log2n) && std::max(len_a, len_b) <= (1ull << 30) &&
                        bc_lgR(len_a) == bc_lgR(len_b);
    if (paired) {
        const EncOp A{a, len_a, W0, W0, W2}, B{b, len_b, W1, W1, W3};
        if ((rc = run_encode_fast(ctx, A, &B, log2n, s))) return rc;
    }
    for (int side = 0; side < (square ? 1 : 2) && !paired; ++side) {
        const uint64_t *src = side ? b : a;
        const uint64_t len = side ? len_b : len_a;
        uint64_t *dst = side ? W1 : W0;
        const uint64_t N = next_pow2(std::max<uint64_t>(len, 1));
        if (fast_path(log2n) && N <= (1ull << 30)) {
            if ((rc = run_encode_fast(ctx, src, len, log2n, dst, W2, W3, s))) return rc;
        } else {
            uint64_t *cur = dst, *spare = W2;
            if ((rc = run_encode_in(ctx, src, len, log2n, cur, spare, s))) return rc;
            if (cur != dst) HIP_TRY(hipMemcpyAsync(dst, cur, (1ull << (log2n - 6)) * 8, hipMemcpyDeviceToDevice, s));
        }
    }
    pa = W0;
    pb = W1;
    if (square) {
        const uint64_t nw = 1ull << (log2n - 6);
        if ((rc = run_butterflies(ctx, BF_FWD, pa, nullptr, log2n - 6, s))) return rc;
        KLAUNCH(ctx, s, "pointwise", k_square, square_grid(ctx, nw), SQ_THREADS, pa, nw, ctx->tables);
        if ((rc = run_butterflies(ctx, BF_INV, pa, nullptr, log2n - 6, s))) return rc;
    } else if ((rc = run_butterflies(ctx, BF_PRODUCT, pa, pb, log2n - 6, s))) {
        return rc;
    }
    if (fast_path(log2n)) return run_decode_fast(ctx, pa, log2n, out, lc, W2, W3, s);
    uint64_t *cur = pa, *spare = pb;
    if ((rc = run_decode_out(ctx, log2n, cur, spare, s))) return rc;
    KLAUNCH(ctx, s, "store", k_store_mask, grid_for((lc + 63) / 64, 256), 256, cur, lc, out);
    return 0;
}

static int addfft_body(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, int log2n, uint64_t *values,
                       hipStream_t s)
{
    const uint64_t nw = 1ull << (log2n - 6);
    int rc = ensure_ws(ctx, ws_words_for(log2n));
    if (rc) return rc;
    if ((rc = set_lds_limits())) return rc;
    uint64_t *cur = ctx->ws[0], *spare = ctx->ws[1];
    const uint64_t N = next_pow2(std::max<uint64_t>(len_a, 1));
    if (fast_path(log2n) && N <= (1ull << 30) && len_a) {
        if ((rc = run_encode_fast(ctx, a, len_a, log2n, cur, ctx->ws[2], ctx->ws[3], s))) return rc;
    } else {
        if ((rc = run_encode_in(ctx, len_a ? a : ctx->ws[2], len_a, log2n, cur, spare, s))) return rc;
    }
    if ((rc = run_butterflies(ctx, BF_FWD, cur, nullptr, log2n - 6, s))) return rc;
    HIP_TRY(hipMemcpyAsync(values, cur, nw * 8, hipMemcpyDeviceToDevice, s));
    return 0;
}

static int iaddfft_body(polymul_ctx *ctx, const uint64_t *values, int log2n, uint64_t *out, uint64_t out_bits,
                        hipStream_t s)
{
    const uint64_t nw = 1ull << (log2n - 6);
    int rc = ensure_ws(ctx, ws_words_for(log2n));
    if (rc) return rc;
    if ((rc = set_lds_limits())) return rc;
    uint64_t *cur = ctx->ws[0], *spare = ctx->ws[1];
    HIP_TRY(hipMemcpyAsync(cur, values, nw * 8, hipMemcpyDeviceToDevice, s));
    if ((rc = run_butterflies(ctx, BF_INV, cur, nullptr, log2n - 6, s))) return rc;
    if (fast_path(log2n)) return run_decode_fast(ctx, cur, log2n, out, out_bits, ctx->ws[2], ctx->ws[3], s);
    if ((rc = run_decode_out(ctx, log2n, cur, spare, s))) return rc;
    KLAUNCH(ctx, s, "store", k_store_mask, grid_for((out_bits + 63) / 64, 256), 256, cur, out_bits, out);
    return 0;
}

// C = A B (lc bits) from A's forward transform fa of 2^log2n bits (f2:
// transform reuse): B's BasisCvt, Encode and Butterfly, the pointwise
// products with fa, then the inverse steps (Alg. 5 with A's forward steps
// already done; any n >= lc gives the same product)
static int resident_body(polymul_ctx *ctx, const uint64_t *fa, int log2n, const uint64_t *b, uint64_t len_b,
                         uint64_t *out, uint64_t lc, hipStream_t s)
{
    const uint64_t nw = 1ull << (log2n - 6);
    int rc = ensure_ws(ctx, ws_words_for(log2n));
    if (rc) return rc;
    if ((rc = set_lds_limits())) return rc;
    uint64_t *cur = ctx->ws[0], *spare = ctx->ws[1];
    const uint64_t N = next_pow2(std::max<uint64_t>(len_b, 1));
    if (fast_path(log2n) && N <= (1ull << 30)) {
        if ((rc = run_encode_fast(ctx, b, len_b, log2n, cur, ctx->ws[2], ctx->ws[3], s))) return rc;
    } else {
        if ((rc = run_encode_in(ctx, b, len_b, log2n, cur, spare, s))) return rc;
    }
    if ((rc = run_butterflies(ctx, BF_FWD, cur, nullptr, log2n - 6, s))) return rc;
    KLAUNCH(ctx, s, "pointwise", k_pointwise,
            (unsigned)std::min<uint64_t>((nw + 1023) / 1024, (uint64_t)ctx->num_cu), 1024, cur, fa, nw, ctx->tables);
    if ((rc = run_butterflies(ctx, BF_INV, cur, nullptr, log2n - 6, s))) return rc;
    if (fast_path(log2n)) return run_decode_fast(ctx, cur, log2n, out, lc, ctx->ws[2], ctx->ws[3], s);
    if ((rc = run_decode_out(ctx, log2n, cur, spare, s))) return rc;
    KLAUNCH(ctx, s, "store", k_store_mask, grid_for((lc + 63) / 64, 256), 256, cur, lc, out);
    return 0;
}

// an operand kept on the device as its forward transform (polymul_resident_*)
struct polymul_resident {
    int device = 0;
    int log2n = 0;
    uint64_t len_a = 0;
    uint64_t *vals = nullptr;   // 2^(log2n - 6) transform values
};

static int basiscvt_body(polymul_ctx *ctx, const uint64_t *in, uint64_t len, int log2n, int inverse, uint64_t *out,
                         hipStream_t s)
{
    const uint64_t nbits = 1ull << log2n, nw = (nbits + 63) / 64;
    int rc = ensure_ws(ctx, nw);
    if (rc) return rc;
    uint64_t *cur = ctx->ws[0];
    KLAUNCH(ctx, s, "load", k_load_mask, grid_for(nw, 256), 256, in, inverse ? nbits : len, cur, nw);
    if ((rc = run_bcvt(ctx, inverse ? nbits : next_pow2(std::max<uint64_t>(len, 1)), inverse != 0, cur,
                       inverse ? ctx->ws[1] : nullptr, nw, s)))
        return rc;
    KLAUNCH(ctx, s, "store", k_store_mask, grid_for(nw, 256), 256, cur, nbits, out);
    return 0;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------

// the compile-time step table of the inner conversion must be the recursion's
static int check_bc16_table()
{
    std::vector<BStep> v;
    bcvt_steps(1ull << 16, 1, v);
    if ((int)v.size() != BC16_NSTEPS) return fail(POLYMUL_EIO, "inner BasisCvt step table has the wrong length");
    for (int k = 0; k < BC16_NSTEPS; ++k)
        if (v[k].S != (1ull << bc16_lgs[k]) || v[k].d != (1ull << bc16_lgd[k]))
            return fail(POLYMUL_EIO, "inner BasisCvt step table differs from the recursion at step " + std::to_string(k));
    for (int lg = 6; lg <= 15; ++lg) {
        std::vector<BStep> w;
        bcvt_steps(1ull << lg, 1, w);
        const BcStepList L = bc_steps_of(lg);
        if ((int)w.size() != L.n) return fail(POLYMUL_EIO, "element step list has the wrong length");
        for (int k = 0; k < L.n; ++k)
            if (w[k].S != (1ull << L.lgs[k]) || w[k].d != (1ull << L.lgd[k]))
                return fail(POLYMUL_EIO, "element step list differs from the recursion");
    }
    return 0;
}

static int batch_steps_upload(polymul_ctx *ctx)
{
    if (ctx->bsteps) return 0;
    std::unique_ptr<BatchSteps> H(new BatchSteps());
    std::memset(H.get(), 0, sizeof(BatchSteps));
    int pos = 0;
    for (int k = BT_MIN_LOG2N; k <= BT_MAX_LOG2N; ++k) {
        std::vector<BStep> v;
        bcvt_steps(1ull << k, 1, v);
        if (pos + (int)v.size() > BT_MAX_STEPS) return fail(POLYMUL_EIO, "batch step table too small");
        H->first[k] = pos;
        H->count[k] = (int)v.size();
        for (const BStep &st : v) {
            BatchStep &o = H->st[pos++];
            o.S = st.S;
            o.d = st.d;
            o.L = o.D = 0;
            if (st.S < 128) {
                const int Hh = (int)(st.S / 2), d = (int)st.d;
                for (int b = 0; b < 64; ++b) {
                    const int r = b % (int)st.S;
                    if (r < Hh) o.L |= 1ull << b;
                    if (r < d) o.D |= 1ull << b;
                }
            }
        }
    }
    HIP_TRY(hipMalloc(&ctx->bsteps, sizeof(BatchSteps)));
    hipError_t e = hipMemcpy(ctx->bsteps, H.get(), sizeof(BatchSteps), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ctx->bsteps);
        ctx->bsteps = nullptr;
        return fail(POLYMUL_EIO, std::string("upload batch steps: ") + hipGetErrorString(e));
    }
    return 0;
}

// layout of a batch workspace: per-workgroup slabs (4 buffers each), the
// queue order, the queue counter
struct BatchLayout {
    unsigned grid;
    uint64_t slab_words;
    size_t slab_bytes, order_bytes, total;
};

static BatchLayout batch_layout(const polymul_ctx *ctx, uint32_t count, uint64_t max_bits)
{
    BatchLayout L;
    const int maxlog = std::max(BT_MIN_LOG2N, ilog2(max_bits));
    L.slab_words = 1ull << (maxlog - 6);
    L.grid = (unsigned)std::min<uint64_t>(count, (uint64_t)ctx->num_cu);
    L.slab_bytes = (size_t)L.grid * 4 * L.slab_words * 8;
    L.order_bytes = ((size_t)count * 4 + 255) / 256 * 256;
    L.total = L.slab_bytes + L.order_bytes + 256;
    return L;
}

static size_t batch_ws_bytes(const polymul_ctx *ctx, uint32_t count, uint64_t max_bits)
{
    return batch_layout(ctx, count, max_bits).total;
}

// one_host: a single product given on the host; its descriptor goes into
// the workspace (the 256-byte tail beside the queue counter)
static int batch_body(polymul_ctx *ctx, uint32_t count, const uint64_t *a_pool, const uint64_t *a_off,
                      const uint64_t *len_a, const uint64_t *b_pool, const uint64_t *b_off, const uint64_t *len_b,
                      uint64_t *out_pool, const uint64_t *out_off, const BtDesc *desc, uint64_t max_bits,
                      int32_t *status, hipStream_t s, const BtDesc *one_host = nullptr)
{
    int rc;
    if ((rc = batch_steps_upload(ctx)) || (rc = set_lds_limits())) return rc;
    const BatchLayout BL = batch_layout(ctx, count, max_bits);
    const unsigned grid = BL.grid;
    const uint64_t slab_words = BL.slab_words;
    const size_t slab_bytes = BL.slab_bytes, order_bytes = BL.order_bytes, need = BL.total;
    if (need > ctx->bws_bytes) {
        if (ctx->borrowed) return fail(POLYMUL_EIO, "borrowed batch workspace smaller than the launch needs");
        if (ctx->cap && need > ctx->cap)
            return fail(POLYMUL_ENOMEM, "batch workspace of " + std::to_string(need) + " bytes exceeds the cap of " +
                                            std::to_string(ctx->cap));
        if (ctx->bws) {
            HIP_TRY(hipStreamSynchronize(s));
            (void)hipFree(ctx->bws);
            ctx->bws = nullptr;
            ctx->bws_bytes = 0;
        }
        hipError_t e = hipMalloc(&ctx->bws, need);
        if (e != hipSuccess) {
            ctx->bws = nullptr;
            return fail(POLYMUL_ENOMEM, std::string("hipMalloc batch workspace: ") + hipGetErrorString(e));
        }
        ctx->bws_bytes = need;
    }
    uint64_t *slab = static_cast<uint64_t *>(ctx->bws);
    uint32_t *order = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->bws) + slab_bytes);
    uint32_t *counter = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->bws) + slab_bytes + order_bytes);
    if (one_host) {
        BtDesc *d1 = reinterpret_cast<BtDesc *>(static_cast<char *>(ctx->bws) + slab_bytes + order_bytes + 64);
        KLAUNCH(ctx, s, "batch_desc", k_bt_put_desc, 1, 64, *one_host, d1);
        desc = d1;
    }
    KLAUNCH(ctx, s, "batch_plan", k_batch_plan, 1, 1024, count, len_a, len_b, desc, max_bits, order, counter);
    KLAUNCH_LDS(ctx, s, "batch", k_batch, grid, BT_THREADS, bf_bottom_lds(BF_BOTTOM_R, true), a_pool, a_off, len_a,
                b_pool, b_off, len_b, out_pool, out_off, desc, status, count, max_bits, order, counter, slab,
                slab_words, ctx->tables, ctx->bsteps, ctx->small_field_log2n);
    return 0;
}

static void fill_dev_tables(const fpmul_host::Tables &H, DevTables &D)
{
    const fpmul_host::Tower &tw = H.tw;
    std::memcpy(D.iota, H.iota, sizeof(D.iota));
    for (int k = 0; k < 8; ++k)
        for (int e = 0; e < 256; ++e) {
            uint64_t f = 0, a = 0;
            for (int u = 0; u < 8; ++u)
                if ((e >> u) & 1) {
                    f ^= H.enc[8 * k + u];
                    a ^= H.dec[8 * k + u];
                }
            D.enc_win[k][e] = f;
            D.dec_win[k][e] = a;
        }
    for (int d = 0; d < 32; ++d)
        for (int t = 0; t < 64; ++t) D.gbasis[d][t] = tw.m64(H.cantor[32 + d], 1ull << t);
    // squaring is GF(2)-linear (characteristic 2): x^2 is the XOR of the
    // squares of x's byte windows
    for (int k = 0; k < 8; ++k)
        for (int e = 0; e < 256; ++e) {
            const uint64_t x = (uint64_t)e << (8 * k);
            D.sq_win[k][e] = tw.m64(x, x);
        }
    for (int v = 0; v < 24; ++v)
        for (int t = 0; t < 64; ++t) D.pbasis[v][t] = tw.m64(H.cantor[8 + v], 1ull << t);
    std::memcpy(D.mul8, tw.mul8, sizeof(D.mul8));
    for (int p = 0; p < 2; ++p)
        for (int e = 0; e < 256; ++e) D.c15[p][e] = tw.m16(tw.v15, (uint16_t)(e << (8 * p)));
    for (int p = 0; p < 4; ++p)
        for (int e = 0; e < 256; ++e) D.c31[p][e] = tw.m32(tw.v31, (uint32_t)e << (8 * p));
    auto permtab = [&](uint8_t beta, uint32_t *pt) {
        uint8_t g0[8], g1[8], g2[4];
        for (int e = 0; e < 8; ++e) {
            g0[e] = tw.mul8[beta][e];
            g1[e] = tw.mul8[beta][e << 3];
        }
        for (int e = 0; e < 4; ++e) g2[e] = tw.mul8[beta][e << 6];
        auto pack = [](const uint8_t *b) {
            return (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
        };
        pt[0] = pack(g0);
        pt[1] = pack(g0 + 4);
        pt[2] = pack(g1);
        pt[3] = pack(g1 + 4);
        pt[4] = pack(g2);
        pt[5] = pt[6] = pt[7] = 0;
    };
    for (int bl = 0; bl < 128; ++bl) permtab((uint8_t)H.iota[0][2 * bl], D.pt_beta8[bl]);   // iota(2 bl) is in V_8
    for (int e = 0; e < 256; ++e) permtab((uint8_t)e, D.pt8[e]);
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) {
            const uint8_t p = tw.mul8[a][b];
            D.mulp[a][b] = (uint16_t)(p | (tw.mul8[0x80][p] << 8));   // v_7 = Cantor byte 0x80
        }
    for (int k = 0; k < 4; ++k)
        for (int e = 0; e < 256; ++e) {
            uint32_t f = 0, a = 0;
            for (int u = 0; u < 8; ++u)
                if ((e >> u) & 1) {
                    f ^= H.enc32[8 * k + u];
                    a ^= H.dec32[8 * k + u];
                }
            D.enc32_win[k][e] = f;
            D.dec32_win[k][e] = a;
        }
    for (int d = 0; d < 16; ++d)
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 256; ++e)
                D.kt32[d][256 * k + e] = tw.m32((uint32_t)H.cantor[16 + d], (uint32_t)e << (8 * k));
}

// ---------------------------------------------------------------------------
// The workspace of polymul_ex_noalloc: a file-scope device array, one copy
// per GPU that the library runs on, held until the process ends.  Host code
// never names it except to look up its device address, once per device with
// that device current; kernels get that address.
// ---------------------------------------------------------------------------

static __device__ __align__(256) uint64_t scratch[fpmul_plan::NOALLOC_SCRATCH_WORDS];

static int scratch_address(int device, uint64_t **out)
{
    static std::mutex mu;
    static std::map<int, uint64_t *> addr;   // device -> address of its copy
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the caller made `device` current
        if (e != hipSuccess || !p)
            return fail(POLYMUL_EIO, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = addr.emplace(device, static_cast<uint64_t *>(p)).first;
    }
    *out = it->second;
    return 0;
}

// ---------------------------------------------------------------------------
// captured launch chains (polymul_graph_*): the kernels of one product (or of
// one batch) recorded once into a HIP graph on a private stream and replayed
// on the caller's stream.  A graph owns the workspaces its kernels were
// recorded with, so nothing the context later grows or frees can move them.
// ---------------------------------------------------------------------------

struct polymul_graph {
    polymul_ctx view;        // the parent's tables, this graph's workspaces (borrowed)
    void *mem = nullptr;     // 4 product workspaces, then the batch workspace
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

static void graph_free(polymul_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->mem) (void)hipFree(g->mem);
    delete g;
}

// a graph whose view shares ctx's tables and owns ws_words x 4 + bws_bytes of workspace
static int graph_new(polymul_ctx *ctx, uint64_t ws_words, size_t bws_bytes, polymul_graph **out)
{
    std::unique_ptr<polymul_graph> g(new polymul_graph());
    g->device = ctx->device;
    polymul_ctx &v = g->view;
    v.device = ctx->device;
    v.tables = ctx->tables;
    v.psteps = ctx->psteps;
    v.bsteps = ctx->bsteps;
    v.num_cu = ctx->num_cu;
    v.tuned = ctx->tuned;
    v.small_field_log2n = ctx->small_field_log2n;
    v.large_field_log2n = M64_MAX_LOG2N + 1;   // graphs run over GF(2^64)
    v.borrowed = true;
    const size_t ws_bytes = (size_t)ws_words * 8, bws_al = (bws_bytes + 255) / 256 * 256;
    hipError_t e = hipMalloc(&g->mem, 4 * ws_bytes + bws_al);
    if (e != hipSuccess) {
        g->mem = nullptr;
        return fail(POLYMUL_ENOMEM, std::string("hipMalloc graph workspace: ") + hipGetErrorString(e));
    }
    for (int k = 0; k < 4; ++k) v.ws[k] = reinterpret_cast<uint64_t *>(static_cast<char *>(g->mem) + k * ws_bytes);
    v.ws_words = ws_words;
    v.bws = bws_al ? static_cast<char *>(g->mem) + 4 * ws_bytes : nullptr;
    v.bws_bytes = bws_al;
    *out = g.release();
    return 0;
}

// record body(view, stream) into g->graph on a private stream and instantiate it
template <typename Body>
static int graph_capture(polymul_graph *g, Body body)
{
    int rc;
    if ((rc = set_lds_limits())) return rc;   // function attributes are set outside the capture
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(POLYMUL_EIO, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    rc = body(&g->view, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess || !graph) return fail(POLYMUL_EIO, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g->exec = nullptr;
        return fail(POLYMUL_EIO, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return 0;
}

// ---------------------------------------------------------------------------
// schedule tuner (polymul_tune): times the fused path's schedule choices on
// the device -- the split of the upper butterfly layers into passes, the
// row-kernel and zeta-kernel grids -- by coordinate descent from the default,
// keeps the fastest, checks that it gives the default's product word for
// word, and can append it to a text cache keyed by device architecture, CU
// count and transform length.  Every choice is a valid schedule of the same
// computation (any split of the layers, any grid of the grid-stride loops).
// ---------------------------------------------------------------------------

// operand words from SplitMix64 (the product path is data-oblivious: any
// operands time the same)
__global__ void k_tune_fill(uint64_t *__restrict__ p, uint64_t n, uint64_t seed)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        p[i] = z ^ (z >> 31);
    }
}

static std::string device_arch(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static int write_report(char *buf, size_t len, const std::string &text)
{
    if (!buf || len == 0) return 0;
    std::snprintf(buf, len, "%s", text.c_str());
    return 0;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *polymul_last_error(void) { return g_err.c_str(); }

const char *polymul_version(void) { return FPMUL_VERSION; }

int polymul_ctx_create(polymul_ctx **out, int device, size_t workspace_cap)
{
    if (!out) return fail(POLYMUL_EINVAL, "ctx out pointer is null");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(POLYMUL_EINVAL, "no such device");
    DeviceGuard g(device);
    HIP_TRY(g.err);
    if (int rc = check_bc16_table()) return rc;
    std::unique_ptr<fpmul_host::Tables> H(new fpmul_host::Tables());
    std::unique_ptr<DevTables> D(new DevTables());
    try {
        fpmul_host::build_tables(*H);
        fill_dev_tables(*H, *D);
    } catch (const std::exception &ex) {
        return fail(POLYMUL_EIO, std::string("constant tables: ") + ex.what());
    }
    polymul_ctx *ctx = new polymul_ctx();
    ctx->device = device;
    ctx->cap = workspace_cap;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            ctx->num_cu = cus;
    }
    std::unique_ptr<PStepTable> P(new PStepTable());
    if (int rc = build_psteps(*P)) {
        delete ctx;
        return rc;
    }
    hipError_t e = hipMalloc(&ctx->tables, sizeof(DevTables));
    if (e == hipSuccess) e = hipMemcpy(ctx->tables, D.get(), sizeof(DevTables), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&ctx->psteps, sizeof(PStepTable));
    if (e == hipSuccess) e = hipMemcpy(ctx->psteps, P.get(), sizeof(PStepTable), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (ctx->tables) (void)hipFree(ctx->tables);
        if (ctx->psteps) (void)hipFree(ctx->psteps);
        delete ctx;
        return fail(POLYMUL_EIO, std::string("upload tables: ") + hipGetErrorString(e));
    }
    // everything polymul_ex_noalloc needs is in place before its first call:
    // the batch step lists and the address of this device's scratch
    int rc = batch_steps_upload(ctx);
    if (!rc) rc = scratch_address(device, &ctx->scratch);
    if (rc) {
        (void)polymul_ctx_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return 0;
}

int polymul_ctx_destroy(polymul_ctx *ctx)
{
    if (!ctx) return 0;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    for (int k = 0; k < 4; ++k)
        if (ctx->ws[k]) (void)hipFree(ctx->ws[k]);
    if (ctx->tables) (void)hipFree(ctx->tables);
    if (ctx->tables128) (void)hipFree(ctx->tables128);
    if (ctx->psteps) (void)hipFree(ctx->psteps);
    if (ctx->bsteps) (void)hipFree(ctx->bsteps);
    if (ctx->bws) (void)hipFree(ctx->bws);
    for (ProfRec &r : ctx->prof_live) {
        if (r.start) (void)hipEventDestroy(r.start);
        if (r.stop) (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    delete ctx;
    return 0;
}

int polymul_ex(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
               uint64_t *out, void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (len_a == 0 || len_b == 0) return 0;
    if (len_a > POLYMUL_MAX_PRODUCT_BITS || len_b > POLYMUL_MAX_PRODUCT_BITS ||
        len_a + len_b - 1 > POLYMUL_MAX_PRODUCT_BITS)
        return fail(POLYMUL_EINVAL, "product length exceeds 2^62 bits");
    const uint64_t lc = len_a + len_b - 1;
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(a, "a_bits")) || (rc = check_dev_ptr(b, "b_bits")) || (rc = check_dev_ptr(out, "out")))
        return rc;
    size_t ob = (size_t)((lc + 63) / 64) * 8;
    if (ranges_overlap(out, ob, a, (size_t)((len_a + 63) / 64) * 8) ||
        ranges_overlap(out, ob, b, (size_t)((len_b + 63) / 64) * 8))
        return fail(POLYMUL_EINVAL, "out overlaps an input");
    const int log2n = transform_log2(len_a, len_b);
    if (log2n <= SINGLE_VIA_BATCH_LOG2N && log2n < ctx->large_field_log2n) {
        // a small product is one workgroup's work: the batch kernel takes it in
        // three launches instead of one launch per BasisCvt step
        const BtDesc one{a, b, out, len_a, len_b};
        return batch_body(ctx, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          1ull << log2n, nullptr, (hipStream_t)stream, &one);
    }
    return product_body(ctx, a, len_a, b, len_b, out, (hipStream_t)stream);
}

int polymul_ex_noalloc(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                       uint64_t *out, void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (len_a == 0 || len_b == 0) return 0;
    if (len_a > (1ull << fpmul_plan::NOALLOC_MAX_LOG2N) || len_b > (1ull << fpmul_plan::NOALLOC_MAX_LOG2N) ||
        len_a + len_b - 1 > (1ull << fpmul_plan::NOALLOC_MAX_LOG2N))
        return fail(POLYMUL_EINVAL, "polymul_ex_noalloc takes products of at most 2^" +
                                        std::to_string(fpmul_plan::NOALLOC_MAX_LOG2N) +
                                        " bits (its device scratch holds one such product's workspace); "
                                        "polymul_ex takes longer ones");
    if (!ctx->scratch) return fail(POLYMUL_EIO, "ctx has no device scratch address");
    const uint64_t lc = len_a + len_b - 1;
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(a, "a_bits")) || (rc = check_dev_ptr(b, "b_bits")) || (rc = check_dev_ptr(out, "out")))
        return rc;
    size_t ob = (size_t)((lc + 63) / 64) * 8;
    if (ranges_overlap(out, ob, a, (size_t)((len_a + 63) / 64) * 8) ||
        ranges_overlap(out, ob, b, (size_t)((len_b + 63) / 64) * 8))
        return fail(POLYMUL_EINVAL, "out overlaps an input");
    // a view of ctx whose workspaces are slices of the scratch: borrowed, so
    // nothing on the path below grows or frees them
    polymul_ctx view;
    view.device = ctx->device;
    view.tables = ctx->tables;
    view.psteps = ctx->psteps;
    view.bsteps = ctx->bsteps;
    view.num_cu = ctx->num_cu;
    view.tuned = ctx->tuned;
    view.small_field_log2n = ctx->small_field_log2n;
    view.large_field_log2n = M64_MAX_LOG2N + 1;   // every product it takes is m = 64
    view.borrowed = true;
    for (int k = 0; k < 4; ++k) view.ws[k] = ctx->scratch + (uint64_t)k * fpmul_plan::NOALLOC_WS_WORDS;
    view.ws_words = fpmul_plan::NOALLOC_WS_WORDS;
    view.bws = ctx->scratch + 4 * fpmul_plan::NOALLOC_WS_WORDS;
    view.bws_bytes = fpmul_plan::NOALLOC_BWS_BYTES;
    if (!view.bsteps) return fail(POLYMUL_EIO, "ctx has no batch step lists");
    const int log2n = transform_log2(len_a, len_b);
    if (log2n <= SINGLE_VIA_BATCH_LOG2N) {
        const BtDesc one{a, b, out, len_a, len_b};
        return batch_body(&view, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          1ull << log2n, nullptr, (hipStream_t)stream, &one);
    }
    return product_body(&view, a, len_a, b, len_b, out, (hipStream_t)stream);
}

int polymul_graph_create(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                         uint64_t *out, polymul_graph **graph)
{
    if (!graph) return fail(POLYMUL_EINVAL, "graph out pointer is null");
    *graph = nullptr;
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (len_a == 0 || len_b == 0) return fail(POLYMUL_EINVAL, "a graph needs two non-empty operands");
    if (len_a > POLYMUL_M64_MAX_PRODUCT_BITS || len_b > POLYMUL_M64_MAX_PRODUCT_BITS ||
        len_a + len_b - 1 > POLYMUL_M64_MAX_PRODUCT_BITS)
        return fail(POLYMUL_EINVAL, "graphs take products of at most 2^37 bits (GF(2^64))");
    const uint64_t lc = len_a + len_b - 1;
    DeviceGuard dg(ctx->device);
    HIP_TRY(dg.err);
    int rc;
    if ((rc = check_dev_ptr(a, "a_bits")) || (rc = check_dev_ptr(b, "b_bits")) || (rc = check_dev_ptr(out, "out")))
        return rc;
    size_t ob = (size_t)((lc + 63) / 64) * 8;
    if (ranges_overlap(out, ob, a, (size_t)((len_a + 63) / 64) * 8) ||
        ranges_overlap(out, ob, b, (size_t)((len_b + 63) / 64) * 8))
        return fail(POLYMUL_EINVAL, "out overlaps an input");
    if ((rc = batch_steps_upload(ctx))) return rc;
    const int log2n = transform_log2(len_a, len_b);
    const bool one_item = log2n <= SINGLE_VIA_BATCH_LOG2N;
    const uint64_t ws_words = one_item ? 1 : fpmul_plan::ws_words_for(log2n);
    const size_t bws = one_item ? batch_ws_bytes(ctx, 1, 1ull << log2n) : 0;
    polymul_graph *g = nullptr;
    if ((rc = graph_new(ctx, ws_words, bws, &g))) return rc;
    rc = graph_capture(g, [&](polymul_ctx *v, hipStream_t cs) {
        if (one_item) {
            const BtDesc one{a, b, out, len_a, len_b};
            return batch_body(v, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                              1ull << log2n, nullptr, cs, &one);
        }
        return product_body(v, a, len_a, b, len_b, out, cs);
    });
    if (rc) {
        graph_free(g);
        return rc;
    }
    *graph = g;
    return 0;
}

int polymul_batch_graph_create(polymul_ctx *ctx, uint32_t count, const uint64_t *a_pool, const uint64_t *a_word_off,
                               const uint64_t *len_a, const uint64_t *b_pool, const uint64_t *b_word_off,
                               const uint64_t *len_b, uint64_t *out_pool, const uint64_t *out_word_off,
                               uint64_t max_product_bits, int32_t *status, polymul_graph **graph)
{
    if (!graph) return fail(POLYMUL_EINVAL, "graph out pointer is null");
    *graph = nullptr;
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (count == 0) return fail(POLYMUL_EINVAL, "a batch graph needs at least one item");
    if (max_product_bits == 0 || max_product_bits > POLYMUL_BATCH_MAX_PRODUCT_BITS)
        return fail(POLYMUL_EINVAL, "max_product_bits must be in [1, 2^22]");
    DeviceGuard dg(ctx->device);
    HIP_TRY(dg.err);
    int rc;
    if ((rc = check_dev_ptr(a_pool, "a_pool")) || (rc = check_dev_ptr(a_word_off, "a_word_off")) ||
        (rc = check_dev_ptr(len_a, "len_a")) || (rc = check_dev_ptr(b_pool, "b_pool")) ||
        (rc = check_dev_ptr(b_word_off, "b_word_off")) || (rc = check_dev_ptr(len_b, "len_b")) ||
        (rc = check_dev_ptr(out_pool, "out_pool")) || (rc = check_dev_ptr(out_word_off, "out_word_off")))
        return rc;
    if (status && (rc = check_dev_ptr(status, "status"))) return rc;
    if ((rc = batch_steps_upload(ctx))) return rc;
    polymul_graph *g = nullptr;
    if ((rc = graph_new(ctx, 1, batch_ws_bytes(ctx, count, max_product_bits), &g))) return rc;
    rc = graph_capture(g, [&](polymul_ctx *v, hipStream_t cs) {
        return batch_body(v, count, a_pool, a_word_off, len_a, b_pool, b_word_off, len_b, out_pool, out_word_off,
                          nullptr, max_product_bits, status, cs);
    });
    if (rc) {
        graph_free(g);
        return rc;
    }
    *graph = g;
    return 0;
}

int polymul_graph_launch(polymul_graph *graph, void *stream)
{
    if (!graph || !graph->exec) return fail(POLYMUL_EINVAL, "graph is null");
    DeviceGuard dg(graph->device);
    HIP_TRY(dg.err);
    HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return 0;
}

int polymul_graph_destroy(polymul_graph *graph)
{
    if (!graph) return 0;
    DeviceGuard dg(graph->device);
    (void)hipDeviceSynchronize();   // no replay may still use the workspace
    graph_free(graph);
    return 0;
}

int polymul_tune(polymul_ctx *ctx, int log2n, int reps, const char *cache_path, char *report, size_t report_len)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (!fpmul_plan::fast_path(log2n))
        return fail(POLYMUL_EINVAL, "polymul_tune takes transforms of 2^22 .. 2^31 bits (the fused path)");
    if (reps < 1 || reps > 100) return fail(POLYMUL_EINVAL, "reps must be in [1, 100]");
    DeviceGuard dg(ctx->device);
    HIP_TRY(dg.err);
    const uint64_t L = 1ull << (log2n - 1), aw = L / 64, ow = (2 * L + 63) / 64;
    uint64_t *a = nullptr, *b = nullptr, *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<uint64_t> ref(ow), got(ow);
    const bool prof = ctx->prof;
    const bool had = ctx->tuned_own.count(log2n) != 0;
    const fpmul_plan::Schedule before = had ? ctx->tuned_own[log2n] : fpmul_plan::Schedule();
    auto cleanup = [&]() {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (out) (void)hipFree(out);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
        ctx->prof = prof;
    };
    auto restore = [&]() {
        if (had)
            ctx->tuned_own[log2n] = before;
        else
            ctx->tuned_own.erase(log2n);
    };
    hipError_t e = hipMalloc(&a, aw * 8);
    if (e == hipSuccess) e = hipMalloc(&b, aw * 8);
    if (e == hipSuccess) e = hipMalloc(&out, ow * 8);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return fail(POLYMUL_ENOMEM, std::string("tuner buffers: ") + hipGetErrorString(e));
    }
    ctx->prof = false;
    k_tune_fill<<<grid_for(aw, 256), 256, 0, st>>>(a, aw, 0x5EED7E57ull);
    k_tune_fill<<<grid_for(aw, 256), 256, 0, st>>>(b, aw, 0x5EED7E58ull);
    int rc = 0;
    // mean time of reps products under schedule sc (one untimed product first)
    auto time_of = [&](const fpmul_plan::Schedule &sc, double &ms) -> int {
        ctx->tuned_own[log2n] = sc;
        int r = product_body(ctx, a, L, b, L, out, st);
        if (r) return r;
        HIP_TRY(hipEventRecord(e0, st));
        for (int k = 0; k < reps && !r; ++k) r = product_body(ctx, a, L, b, L, out, st);
        if (r) return r;
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        ms = t / reps;
        return 0;
    };
    const int l = log2n - 6;
    fpmul_plan::Schedule best;
    best.upper = fpmul_plan::default_upper(l);
    double t_def = 0, t_best = 0;
    // the first products after idle time run slower (clocks, caches): warm
    // up before the default is timed, so that it is not beaten by that alone
    ctx->tuned_own[log2n] = best;
    for (int k = 0; k < 3 && !rc; ++k) rc = product_body(ctx, a, L, b, L, out, st);
    if (!rc) rc = time_of(best, t_def);
    if (rc) {
        restore();
        cleanup();
        return rc;
    }
    if ((e = hipMemcpy(ref.data(), out, ow * 8, hipMemcpyDeviceToHost)) != hipSuccess) {
        restore();
        cleanup();
        return fail(POLYMUL_EIO, std::string("tuner copy: ") + hipGetErrorString(e));
    }
    t_best = t_def;
    int tried = 1;
    auto consider = [&](const fpmul_plan::Schedule &sc) -> int {
        double t = 0;
        int r = time_of(sc, t);
        ++tried;
        if (!r && t < t_best * 0.995) {
            t_best = t;
            best = sc;
        }
        return r;
    };
    // below BF3_MIN_L transform values the short-transform passes take their
    // own fixed split: only the grids are searched
    for (const auto &u : l >= BF3_MIN_L ? fpmul_plan::upper_candidates(l) : std::vector<std::vector<int>>()) {
        if (u == best.upper) continue;
        fpmul_plan::Schedule sc = best;
        sc.upper = u;
        if ((rc = consider(sc))) break;
    }
    for (int m : {1, 2, 4, 8}) {
        if (rc || m == best.rows_mult) continue;
        fpmul_plan::Schedule sc = best;
        sc.rows_mult = m;
        rc = consider(sc);
    }
    for (int m : {4, 8, 16, 32}) {
        if (rc || m == best.zeta_mult) continue;
        fpmul_plan::Schedule sc = best;
        sc.zeta_mult = m;
        rc = consider(sc);
    }
    if (!rc && !(best.upper == fpmul_plan::default_upper(l) && best.rows_mult == fpmul_plan::Schedule().rows_mult &&
                 best.zeta_mult == fpmul_plan::Schedule().zeta_mult)) {
        // confirm against the default: the fastest of some 200 noisy timings
        // reads low by chance, so both are timed again, alternately, three
        // times each, and the choice stands only if its median still beats
        // the default's by 0.5%
        fpmul_plan::Schedule def;
        def.upper = fpmul_plan::default_upper(l);
        double tb[3] = {0, 0, 0}, td[3] = {0, 0, 0};
        for (int k = 0; k < 3 && !rc; ++k) {
            rc = time_of(best, tb[k]);
            if (!rc) rc = time_of(def, td[k]);
        }
        if (!rc) {
            std::sort(tb, tb + 3);
            std::sort(td, td + 3);
            t_def = td[1];
            if (tb[1] < td[1] * 0.995) {
                t_best = tb[1];
            } else {
                best = def;
                t_best = td[1];
            }
        }
    }
    if (rc) {
        restore();
        cleanup();
        return rc;
    }
    // the chosen schedule gives the default's product, word for word
    ctx->tuned_own[log2n] = best;
    rc = product_body(ctx, a, L, b, L, out, st);
    if (!rc && (e = hipStreamSynchronize(st)) != hipSuccess) rc = fail(POLYMUL_EIO, hipGetErrorString(e));
    if (!rc && (e = hipMemcpy(got.data(), out, ow * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        rc = fail(POLYMUL_EIO, hipGetErrorString(e));
    if (!rc && std::memcmp(got.data(), ref.data(), ow * 8) != 0)
        rc = fail(POLYMUL_EIO, "tuned schedule changed the product (kept the previous one)");
    if (rc) {
        restore();
        cleanup();
        return rc;
    }
    const std::string arch = device_arch(ctx->device);
    const std::string line = fpmul_plan::schedule_line(arch.c_str(), ctx->num_cu, log2n, best, t_best);
    if (cache_path && *cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (!f) {
            cleanup();
            return fail(POLYMUL_EIO, std::string("cannot append to ") + cache_path);
        }
        std::fprintf(f, "%s\n", line.c_str());
        std::fclose(f);
    }
    char head[160];
    std::snprintf(head, sizeof head, "default_ms=%.4f tuned_ms=%.4f tried=%d | ", t_def, t_best, tried);
    write_report(report, report_len, head + line);
    cleanup();
    return 0;
}

int polymul_tune_load(polymul_ctx *ctx, const char *cache_path, int *applied)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (!cache_path) return fail(POLYMUL_EINVAL, "cache path is null");
    if (applied) *applied = 0;
    FILE *f = std::fopen(cache_path, "r");
    if (!f) return fail(POLYMUL_EINVAL, std::string("cannot read ") + cache_path);
    const std::string arch = device_arch(ctx->device);
    char line[512];
    int n = 0;
    while (std::fgets(line, sizeof line, f)) {
        int lg = 0;
        fpmul_plan::Schedule sc;
        if (fpmul_plan::schedule_parse(line, arch.c_str(), ctx->num_cu, lg, sc)) {
            ctx->tuned_own[lg] = sc;   // a later line for the same length wins
            ++n;
        }
    }
    std::fclose(f);
    if (applied) *applied = n;
    return 0;
}

int polymul_tune_get(polymul_ctx *ctx, int log2n, char *buf, size_t buflen)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (!fpmul_plan::fast_path(log2n)) return fail(POLYMUL_EINVAL, "log2n must be in [22, 31]");
    fpmul_plan::Schedule sc = sched_of(ctx, log2n);
    if (sc.upper.empty()) sc.upper = fpmul_plan::default_upper(log2n - 6);
    const std::string arch = device_arch(ctx->device);
    return write_report(buf, buflen, fpmul_plan::schedule_line(arch.c_str(), ctx->num_cu, log2n, sc, 0.0));
}

int polymul_resident_create(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, uint64_t max_product_bits,
                            polymul_resident **res)
{
    if (!res) return fail(POLYMUL_EINVAL, "resident out pointer is null");
    *res = nullptr;
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (len_a == 0) return fail(POLYMUL_EINVAL, "a resident operand needs at least one bit");
    if (max_product_bits < len_a || max_product_bits > POLYMUL_M64_MAX_PRODUCT_BITS)
        return fail(POLYMUL_EINVAL, "max_product_bits must be in [len_a, 2^37]");
    DeviceGuard dg(ctx->device);
    HIP_TRY(dg.err);
    int rc;
    if ((rc = check_dev_ptr(a, "a_bits"))) return rc;
    std::unique_ptr<polymul_resident> r(new polymul_resident());
    r->device = ctx->device;
    r->log2n = fpmul_plan::product_log2n(max_product_bits);
    r->len_a = len_a;
    hipError_t e = hipMalloc(&r->vals, (1ull << (r->log2n - 6)) * 8);
    if (e != hipSuccess) {
        r->vals = nullptr;
        return fail(POLYMUL_ENOMEM, std::string("hipMalloc resident transform: ") + hipGetErrorString(e));
    }
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(r->vals);
        return fail(POLYMUL_EIO, std::string("resident stream: ") + hipGetErrorString(e));
    }
    rc = addfft_body(ctx, a, len_a, r->log2n, r->vals, st);
    e = hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (!rc && e != hipSuccess) rc = fail(POLYMUL_EIO, std::string("resident transform: ") + hipGetErrorString(e));
    if (rc) {
        (void)hipFree(r->vals);
        return rc;
    }
    *res = r.release();
    return 0;
}

int polymul_resident_destroy(polymul_resident *res)
{
    if (!res) return 0;
    DeviceGuard dg(res->device);
    (void)hipDeviceSynchronize();   // no launch may still read the transform
    if (res->vals) (void)hipFree(res->vals);
    delete res;
    return 0;
}

int polymul_resident_mul(polymul_ctx *ctx, const polymul_resident *res, const uint64_t *b, uint64_t len_b,
                         uint64_t *out, void *stream)
{
    if (!ctx || !res) return fail(POLYMUL_EINVAL, "ctx or resident operand is null");
    if (res->device != ctx->device) return fail(POLYMUL_EINVAL, "resident operand is on another device");
    if (len_b == 0) return 0;
    const uint64_t lc = res->len_a + len_b - 1;
    if (lc > (1ull << res->log2n)) return fail(POLYMUL_EINVAL, "product longer than the resident operand's transform");
    DeviceGuard dg(ctx->device);
    HIP_TRY(dg.err);
    int rc;
    if ((rc = check_dev_ptr(b, "b_bits")) || (rc = check_dev_ptr(out, "out"))) return rc;
    if (ranges_overlap(out, (size_t)((lc + 63) / 64) * 8, b, (size_t)((len_b + 63) / 64) * 8))
        return fail(POLYMUL_EINVAL, "out overlaps an input");
    return resident_body(ctx, res->vals, res->log2n, b, len_b, out, lc, (hipStream_t)stream);
}

int polymul_set_large_field(polymul_ctx *ctx, int min_log2n)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (min_log2n < POLYMUL_LARGE_FIELD_MIN_LOG2N || min_log2n > M64_MAX_LOG2N + 1)
        return fail(POLYMUL_EINVAL, "large-field threshold must be in [7, 38]");
    ctx->large_field_log2n = min_log2n;
    return 0;
}

int polymul_set_small_field(polymul_ctx *ctx, int max_log2n)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (max_log2n < 0 || max_log2n > POLYMUL_SMALL_FIELD_MAX_LOG2N)
        return fail(POLYMUL_EINVAL, "small-field limit must be in [0, 20]");
    ctx->small_field_log2n = max_log2n;
    return 0;
}

int polymul_batch(polymul_ctx *ctx, uint32_t count, const uint64_t *a_pool, const uint64_t *a_word_off,
                  const uint64_t *len_a, const uint64_t *b_pool, const uint64_t *b_word_off, const uint64_t *len_b,
                  uint64_t *out_pool, const uint64_t *out_word_off, uint64_t max_product_bits, int32_t *status,
                  void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (count == 0) return 0;
    if (max_product_bits == 0 || max_product_bits > POLYMUL_BATCH_MAX_PRODUCT_BITS)
        return fail(POLYMUL_EINVAL, "max_product_bits must be in [1, 2^22]");
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(a_pool, "a_pool")) || (rc = check_dev_ptr(a_word_off, "a_word_off")) ||
        (rc = check_dev_ptr(len_a, "len_a")) || (rc = check_dev_ptr(b_pool, "b_pool")) ||
        (rc = check_dev_ptr(b_word_off, "b_word_off")) || (rc = check_dev_ptr(len_b, "len_b")) ||
        (rc = check_dev_ptr(out_pool, "out_pool")) || (rc = check_dev_ptr(out_word_off, "out_word_off")))
        return rc;
    if (status && (rc = check_dev_ptr(status, "status"))) return rc;
    return batch_body(ctx, count, a_pool, a_word_off, len_a, b_pool, b_word_off, len_b, out_pool, out_word_off,
                      nullptr, max_product_bits, status, (hipStream_t)stream);
}

int polymul_addfft(polymul_ctx *ctx, const uint64_t *a, uint64_t len_a, int log2n, uint64_t *values, void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (log2n < 6 || log2n > 37) return fail(POLYMUL_EINVAL, "log2n must be in [6, 37]");
    if (len_a > (1ull << log2n)) return fail(POLYMUL_EINVAL, "len_a exceeds 2^log2n");
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(values, "values"))) return rc;
    if (len_a && (rc = check_dev_ptr(a, "a_bits"))) return rc;
    return addfft_body(ctx, a, len_a, log2n, values, (hipStream_t)stream);
}

int polymul_pointwise(polymul_ctx *ctx, const uint64_t *fa, const uint64_t *fb, int log2n, uint64_t *fc,
                      void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (log2n < 6 || log2n > 37) return fail(POLYMUL_EINVAL, "log2n must be in [6, 37]");
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(fa, "fa")) || (rc = check_dev_ptr(fb, "fb")) || (rc = check_dev_ptr(fc, "fc"))) return rc;
    const uint64_t n = 1ull << (log2n - 6);
    const size_t bytes = (size_t)n * 8;
    if ((fc != fa && ranges_overlap(fc, bytes, fa, bytes)) || (fc != fb && ranges_overlap(fc, bytes, fb, bytes)))
        return fail(POLYMUL_EINVAL, "fc overlaps an input without being it");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t *other = fb;
    if (fc == fb) {
        other = fa;   // the product commutes: multiply fb in place by fa
    } else if (fc != fa) {
        HIP_TRY(hipMemcpyAsync(fc, fa, bytes, hipMemcpyDeviceToDevice, s));
    }
    if (fa == fb)   // a square: fc holds fa's values now
        KLAUNCH(ctx, s, "pointwise", k_square, square_grid(ctx, n), SQ_THREADS, fc, n, ctx->tables);
    else
        KLAUNCH(ctx, s, "pointwise", k_pointwise,
                (unsigned)std::min<uint64_t>((n + 1023) / 1024, (uint64_t)ctx->num_cu), 1024, fc, other, n,
                ctx->tables);
    return 0;
}

int polymul_iaddfft(polymul_ctx *ctx, const uint64_t *values, int log2n, uint64_t *out, uint64_t out_bits,
                    void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (log2n < 6 || log2n > 37) return fail(POLYMUL_EINVAL, "log2n must be in [6, 37]");
    if (out_bits > (1ull << log2n)) return fail(POLYMUL_EINVAL, "out_bits exceeds 2^log2n");
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(values, "values")) || (rc = check_dev_ptr(out, "out"))) return rc;
    if (out_bits == 0) return 0;
    return iaddfft_body(ctx, values, log2n, out, out_bits, (hipStream_t)stream);
}

int polymul_basiscvt(polymul_ctx *ctx, const uint64_t *in, uint64_t len, int log2n, int inverse, uint64_t *out,
                     void *stream)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (log2n < 0 || log2n > 37) return fail(POLYMUL_EINVAL, "log2n must be in [0, 37]");
    if (len > (1ull << log2n)) return fail(POLYMUL_EINVAL, "len exceeds 2^log2n");
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = check_dev_ptr(in, "in")) || (rc = check_dev_ptr(out, "out"))) return rc;
    return basiscvt_body(ctx, in, len, log2n, inverse, out, (hipStream_t)stream);
}

int polymul_profile_enable(polymul_ctx *ctx, int on)
{
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    DeviceGuard g(ctx->device);
    prof_collect(ctx);
    ctx->prof_acc.clear();
    ctx->prof = on != 0;
    return 0;
}

int polymul_profile_report(polymul_ctx *ctx, char *buf, size_t buflen)
{
    if (!ctx || !buf || !buflen) return fail(POLYMUL_EINVAL, "bad argument");
    DeviceGuard g(ctx->device);
    prof_collect(ctx);
    std::string txt;
    for (auto &kv : ctx->prof_acc) {
        char line[256];
        std::snprintf(line, sizeof line, "%s %llu %.6f\n", kv.first.c_str(), (unsigned long long)kv.second.first,
                      kv.second.second);
        txt += line;
    }
    if (txt.size() + 1 > buflen) return fail(POLYMUL_EINVAL, "report buffer too small");
    std::memcpy(buf, txt.c_str(), txt.size() + 1);
    return 0;
}

int polymul(const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b, uint64_t *out)
{
    static std::mutex mu;
    static std::map<int, polymul_ctx *> ctxs;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    polymul_ctx *ctx = nullptr;
    auto it = ctxs.find(dev);
    if (it == ctxs.end()) {
        int rc = polymul_ctx_create(&ctx, dev, 0);
        if (rc) return rc;
        ctxs[dev] = ctx;
    } else {
        ctx = it->second;
    }
    int rc = polymul_ex(ctx, a, len_a, b, len_b, out, nullptr);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(nullptr));
    return 0;
}

}  // extern "C"

#include "server.h"
