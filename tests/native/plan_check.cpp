// Host-only checks of the sizing rules of plan.h: for every product the
// server admits as a single launch, its arena reservation holds the workspace
// that the single-product path asks for; the fused path's buffers fit the
// workspace; and the transform length holds the product.  Prints "ok <name>"
// per check; exits non-zero on failure.
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1803_11301_amd/csrc/plan.h"
#include "../../paper_1803_11301_amd/csrc/server_policy.h"

using namespace fpmul_plan;

static int failures = 0;
#define CHECK(c, ...)                                                      \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::printf("FAIL %s:%d %s ", __FILE__, __LINE__, #c);         \
            std::printf(__VA_ARGS__);                                      \
            std::printf("\n");                                             \
            if (++failures > 20) return;                                   \
        }                                                                  \
    } while (0)

// product lengths: every 2^k - 1, 2^k, 2^k + 1 up to 2^37 and random ones
static std::vector<uint64_t> lengths()
{
    std::vector<uint64_t> v;
    for (int k = 0; k <= 37; ++k) {
        const uint64_t p = 1ull << k;
        for (uint64_t x : {p - 1, p, p + 1})
            if (x >= 1 && x <= (1ull << 37)) v.push_back(x);
    }
    std::mt19937_64 g(12345);
    for (int i = 0; i < 4000; ++i) v.push_back(1 + g() % (1ull << (1 + g() % 37)));
    return v;
}

static void ilog2_is_ceiling()
{
    for (int k = 0; k < 63; ++k) {
        const uint64_t p = 1ull << k;
        CHECK(ilog2(p) == k, "k %d", k);
        if (k >= 1) CHECK(ilog2(p + 1) == k + 1, "k %d", k);
        if (k >= 2) CHECK(ilog2(p - 1) == k, "k %d", k);
    }
    CHECK(ilog2(1) == 0 && ilog2(0) == 0, "small");
    std::printf("ok ilog2_is_ceiling\n");
}

static void transform_holds_the_product()
{
    for (uint64_t lc : lengths()) {
        const int k = product_log2n(lc);
        CHECK(k >= 6 && (1ull << k) >= lc, "lc %llu", (unsigned long long)lc);
        CHECK(k == 6 || (1ull << (k - 1)) < lc || k == 22, "lc %llu: transform not the smallest", (unsigned long long)lc);
        const int k2 = product128_log2n(lc);
        CHECK(k2 >= 7 && (1ull << k2) >= lc, "lc %llu", (unsigned long long)lc);
    }
    std::printf("ok transform_holds_the_product\n");
}

// the server reserves single_launch_bytes(lc) for a single launch; the
// single-product path (with the server's field routing: m = 64 up to 2^37)
// asks for four buffers of product_ws_words(la, lb) words, for every split
// of lc into la + lb - 1
static void server_reservation_holds_the_workspace()
{
    std::mt19937_64 g(777);
    for (uint64_t lc : lengths()) {
        const uint64_t res = single_launch_bytes(lc);
        std::vector<uint64_t> las = {1, lc, (lc + 1) / 2, lc > 1 ? lc - 1 : 1};
        for (int i = 0; i < 4; ++i) las.push_back(1 + g() % lc);
        for (uint64_t la : las) {
            const uint64_t lb = lc + 1 - la;
            CHECK(!routes_m128(lc, M64_MAX_LOG2N + 1), "lc %llu routed to m = 128", (unsigned long long)lc);
            const uint64_t need = 4 * product_ws_words(la, lb, M64_MAX_LOG2N + 1) * 8;
            CHECK(need <= res, "lc %llu la %llu: needs %llu, reserved %llu", (unsigned long long)lc,
                  (unsigned long long)la, (unsigned long long)need, (unsigned long long)res);
            // the arena rounds the reservation up, never down
            CHECK(fpmul_srv::Arena::round(res) >= need, "rounding");
        }
    }
    std::printf("ok server_reservation_holds_the_workspace\n");
}

// every routing threshold of the single-product path: the workspace it asks
// for holds the transform of the route it takes
static void workspace_holds_every_route()
{
    for (int thr = 7; thr <= M64_MAX_LOG2N + 1; ++thr)
        for (uint64_t lc : lengths()) {
            const uint64_t w = product_ws_words(1, lc, thr);
            if (routes_m128(lc, thr)) {
                CHECK(w >= (1ull << (product128_log2n(lc) - 6)), "m128 lc %llu", (unsigned long long)lc);
            } else {
                const int k = product_log2n(lc);
                CHECK(w >= (1ull << (k - 6)), "m64 lc %llu", (unsigned long long)lc);
                CHECK(k <= M64_MAX_LOG2N, "m64 beyond its bound: lc %llu thr %d", (unsigned long long)lc, thr);
            }
        }
    std::printf("ok workspace_holds_every_route\n");
}

// the fused path: the skewed rows of an operand of N <= 2^30 bits (R = N /
// 2^16 rows of bc_ew(lgR) words) and the n_p transform values fit a buffer
static void fused_buffers_fit()
{
    for (int k = FUSED_MIN_LOG2N; k <= FUSED_MAX_LOG2N; ++k) {
        const uint64_t ws = ws_words_for(k), np = 1ull << (k - 6);
        CHECK(ws >= np, "k %d", k);
        for (int lgN = 0; lgN <= std::min(k, 30); ++lgN) {
            const int lgR = lgN <= 16 ? 0 : lgN - 16;
            CHECK((1ull << lgR) * (uint64_t)bc_ew(lgR) <= ws, "k %d lgN %d", k, lgN);
            CHECK(bc_ew(lgR) % 64 == 0 && (uint64_t)(bc_ew(lgR) - TAU_WORDS) * 64 >= (1ull << lgR), "k %d", k);
        }
        // the inverse: 2^(k-16) rows of the product
        CHECK((1ull << (k - 16)) * (uint64_t)bc_ew(k - 16) <= ws, "k %d", k);
    }
    std::printf("ok fused_buffers_fit\n");
}

// the tuner's schedule space: every candidate split of the upper butterfly
// layers is valid (parts 1..7 leaving 7 or 6 layers to the bottom pass, the
// lowest at least 12 minus the bottom's layers), the default split is among
// them, both bottom passes occur, no candidate repeats, and a cache line
// written for a schedule parses back to it (and only for its own device)
static void schedule_space()
{
    for (int l = 16; l <= 25; ++l) {
        const auto cands = upper_candidates(l);
        const auto def = default_upper(l);
        CHECK(upper_valid(l, def), "l=%d default split invalid", l);
        bool has_def = false, has6 = false, has7 = false;
        for (size_t i = 0; i < cands.size(); ++i) {
            CHECK(upper_valid(l, cands[i]), "l=%d candidate %zu invalid", l, i);
            const int b = bottom_layers(l, cands[i]);
            CHECK(b == 6 || b == 7, "l=%d candidate %zu leaves %d bottom layers", l, i, b);
            CHECK(cands[i][0] >= 12 - b, "l=%d candidate %zu: lowest pass too short", l, i);
            has6 = has6 || b == 6;
            has7 = has7 || b == 7;
            has_def = has_def || cands[i] == def;
            for (size_t j = i + 1; j < cands.size(); ++j) CHECK(cands[i] != cands[j], "l=%d repeated candidate", l);
        }
        CHECK(has_def, "l=%d default split not among the candidates", l);
        CHECK(has6 && has7, "l=%d candidates miss a bottom pass size", l);
        CHECK(bottom_layers(l, def) == 7, "l=%d default bottom pass", l);
        for (const auto &u : cands) {
            Schedule s;
            s.upper = u;
            s.rows_mult = 1 + (int)(u.size() % 4);
            s.zeta_mult = 4 << (u[0] % 3);
            const std::string line = schedule_line("gfx950", 256, l + 6, s, 1.25);
            int lg = 0;
            Schedule r;
            CHECK(schedule_parse(line.c_str(), "gfx950", 256, lg, r), "%s does not parse", line.c_str());
            CHECK(lg == l + 6 && r.upper == s.upper && r.rows_mult == s.rows_mult && r.zeta_mult == s.zeta_mult,
                  "%s parses to another schedule", line.c_str());
            CHECK(!schedule_parse(line.c_str(), "gfx942", 256, lg, r), "%s applied to another arch", line.c_str());
            CHECK(!schedule_parse(line.c_str(), "gfx950", 304, lg, r), "%s applied to another CU count", line.c_str());
        }
    }
    int lg = 0;
    Schedule r;
    // malformed or invalid lines are refused
    CHECK(schedule_parse("gfx950 cu=256 log2n=31 upper=7,6,6 rows=2 zeta=8 ms=1", "gfx950", 256, lg, r) &&
              bottom_layers(25, r.upper) == 6,
          "a six-layer bottom split refused");
    for (const char *bad : {"gfx950 cu=256 log2n=31 upper=4,7,7 rows=2 zeta=8 ms=1",   // lowest pass below 5
                            "gfx950 cu=256 log2n=31 upper=5,7,7 rows=2 zeta=8 ms=1",   // bottom 6, lowest below 6
                            "gfx950 cu=256 log2n=31 upper=6,6,7,1 rows=2 zeta=8 ms=1", // 20 layers, bottom 5
                            "gfx950 cu=256 log2n=31 upper=6,6,5 rows=2 zeta=8 ms=1",   // 17 layers, not 18
                            "gfx950 cu=256 log2n=31 upper=6,6,6 rows=0 zeta=8 ms=1",   // no row workgroups
                            "gfx950 cu=256 log2n=21 upper=- rows=2 zeta=8 ms=1",       // outside the fused path
                            "gfx950 cu=256 log2n=31 upper=6,x,6 rows=2 zeta=8 ms=1", "garbage"})
        CHECK(!schedule_parse(bad, "gfx950", 256, lg, r), "accepted: %s", bad);
    if (!failures) std::printf("ok schedule_space\n");
}

int main()
{
    schedule_space();
    ilog2_is_ceiling();
    transform_holds_the_product();
    server_reservation_holds_the_workspace();
    workspace_holds_every_route();
    fused_buffers_fit();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    return 0;
}
