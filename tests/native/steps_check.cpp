// CPU checks of the word-level Taylor steps of BasisCvt (k_steps.h), the
// functions the per-step and batch kernels apply on the GPU, against the
// step written bit by bit from its definition (Alg. 1: on every S-bit
// segment with halves lo, hi of H = S/2 bits, hi[0, d) ^= hi[H-d, H), then
// lo[d, H) ^= hi[0, H-d); the inverse takes the two updates in the other
// order).  Covered: one step out of place (bcvt_wide_word), two steps
// composed through a lazily read intermediate array (StepView, the form of
// k_bcvt_wide2), and the in-register step for S <= 64 (bcvt_in_word).
// The header's device functions are plain host functions under a host
// compiler.  Each check prints "ok <name>"; the program exits non-zero on the
// first failure.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1803_11301_amd/csrc/k_steps.h"

#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            std::printf("FAIL %s:%d %s: ", __FILE__, __LINE__, #cond);    \
            std::printf(__VA_ARGS__);                                     \
            std::printf("\n");                                            \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

static uint64_t g_s = 0x243F6A8885A308D3ull;
static uint64_t rnd()
{
    g_s ^= g_s << 13;
    g_s ^= g_s >> 7;
    g_s ^= g_s << 17;
    return g_s;
}

struct Step {
    uint64_t S, d;
};

// the step list of BasisCvt for N bits (Alg. 1 with tau the largest 2^(2^k)
// whose square is at most N / 2), in units of e bits
static void step_list(uint64_t N, uint64_t e, std::vector<Step> &out)
{
    if (N <= 2) return;
    uint64_t tau = 2;
    while (tau < (1ull << 32) && tau * tau <= N / 2) tau *= tau;
    for (uint64_t S = N; S >= 2 * tau; S /= 2) out.push_back({S * e, (S / (2 * tau)) * e});
    step_list(N / tau, tau * e, out);
    step_list(tau, e, out);
}

static int bit(const std::vector<uint64_t> &x, uint64_t i) { return (int)((x[i / 64] >> (i % 64)) & 1); }
static void flip(std::vector<uint64_t> &x, uint64_t i, int v)
{
    if (v) x[i / 64] ^= 1ull << (i % 64);
}

// one step in place, bit by bit
static void step_bits(std::vector<uint64_t> &x, uint64_t nbits, Step st, bool inverse)
{
    const uint64_t H = st.S / 2, d = st.d;
    for (uint64_t seg = 0; seg < nbits; seg += st.S) {
        auto fix = [&]() {
            for (uint64_t i = 0; i < d; ++i) flip(x, seg + H + i, bit(x, seg + 2 * H - d + i));
        };
        // from the top down, so every bit of hi read is the step's input
        auto lo = [&]() {
            for (uint64_t i = H; i-- > d;) flip(x, seg + i, bit(x, seg + H + i - d));
        };
        if (!inverse) {
            fix();
            lo();
        } else {
            lo();
            fix();
        }
    }
}

static std::vector<uint64_t> random_words(uint64_t nw)
{
    std::vector<uint64_t> v(nw);
    for (auto &w : v) w = rnd();
    return v;
}

int main()
{
    int cases = 0;
    // one step out of place, every step with S >= 128 of the lists for 2^7 .. 2^16 bits
    for (int lg = 7; lg <= 16; ++lg) {
        const uint64_t N = 1ull << lg, nw = N / 64;
        std::vector<Step> st;
        step_list(N, 1, st);
        for (int inv = 0; inv < 2; ++inv)
            for (const Step &s : st) {
                if (s.S < 128) continue;
                std::vector<uint64_t> x = random_words(nw), want = x, got(nw);
                step_bits(want, N, s, inv);
                for (uint64_t w = 0; w < nw; ++w) got[w] = bcvt_wide_word(x.data(), w, s.S, s.d, inv);
                CHECK(got == want, "N=2^%d S=%lu d=%lu inverse=%d", lg, (unsigned long)s.S, (unsigned long)s.d, inv);
                ++cases;
            }
    }
    std::printf("ok wide_step (%d cases)\n", cases);

    // two consecutive steps of those lists (in the order each direction takes
    // them), composed without a pass between them
    cases = 0;
    for (int lg = 8; lg <= 16; ++lg) {
        const uint64_t N = 1ull << lg, nw = N / 64;
        std::vector<Step> st;
        step_list(N, 1, st);
        const size_t n = st.size();
        for (int inv = 0; inv < 2; ++inv)
            for (size_t k = 0; k + 1 < n; ++k) {
                const Step a = inv ? st[n - 1 - k] : st[k], b = inv ? st[n - 2 - k] : st[k + 1];
                if (a.S < 128 || b.S < 128) continue;
                std::vector<uint64_t> x = random_words(nw), want = x, got(nw);
                step_bits(want, N, a, inv);
                step_bits(want, N, b, inv);
                const StepView<WordArray> va{WordArray{x.data()}, a.S, a.d, inv};
                for (uint64_t w = 0; w < nw; ++w) got[w] = step_word(va, w, b.S, b.d, inv);
                CHECK(got == want, "pair N=2^%d inverse=%d", lg, inv);
                ++cases;
            }
    }
    // any two steps with S >= 128 and 0 < d <= S / 4, shifts not multiples of 64 included
    for (int it = 0; it < 300; ++it) {
        const uint64_t N = 1ull << 14, nw = N / 64;
        const Step a{128ull << (rnd() % 7), 0}, b{128ull << (rnd() % 7), 0};
        const Step a2{a.S, 1 + rnd() % (a.S / 4)}, b2{b.S, 1 + rnd() % (b.S / 4)};
        const int inv = (int)(rnd() & 1);
        std::vector<uint64_t> x = random_words(nw), want = x, got(nw);
        step_bits(want, N, a2, inv);
        step_bits(want, N, b2, inv);
        const StepView<WordArray> va{WordArray{x.data()}, a2.S, a2.d, inv};
        for (uint64_t w = 0; w < nw; ++w) got[w] = step_word(va, w, b2.S, b2.d, inv);
        CHECK(got == want, "pair Sa=%lu da=%lu Sb=%lu db=%lu inverse=%d", (unsigned long)a2.S, (unsigned long)a2.d,
              (unsigned long)b2.S, (unsigned long)b2.d, inv);
        ++cases;
    }
    std::printf("ok step_pair (%d cases)\n", cases);

    // steps inside one word: L = the low half of every segment, D = its low d bits
    cases = 0;
    for (uint64_t S = 4; S <= 64; S *= 2)
        for (uint64_t d = 1; d <= S / 4; ++d)
            for (int inv = 0; inv < 2; ++inv)
                for (int it = 0; it < 20; ++it) {
                    uint64_t L = 0, D = 0;
                    for (uint64_t seg = 0; seg < 64; seg += S) {
                        for (uint64_t i = 0; i < S / 2; ++i) L |= 1ull << (seg + i);
                        for (uint64_t i = 0; i < d; ++i) D |= 1ull << (seg + i);
                    }
                    std::vector<uint64_t> x = random_words(1), want = x;
                    step_bits(want, 64, Step{S, d}, inv);
                    const uint64_t got = bcvt_in_word(x[0], (int)(S / 2), (int)d, L, D, inv);
                    CHECK(got == want[0], "in-word S=%lu d=%lu inverse=%d", (unsigned long)S, (unsigned long)d, inv);
                    ++cases;
                }
    std::printf("ok in_word_step (%d cases)\n", cases);
    return 0;
}
