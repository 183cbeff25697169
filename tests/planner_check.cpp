// Host-only check of the pass planner (paper_quant_ph_0308158_amd/csrc/planner.cpp),
// built by tests/test_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer: random diagrams under many planner settings,
// and for every plan
//   * each step appears exactly once;
//   * every NOT step of a pass targets a tile bit or has no control among the
//     tile bits (the condition under which steps share a pass, Sec. 2(i));
//   * no tile has more than tile_bits bits, and the first and last passes hold
//     the low address bits and no bit at or above 32;
//   * two steps that do not commute keep their order;
//   * for M <= 14 the reordered list applied to an address-tag vector gives
//     the same vector as the original list (plain pair-swap loop).
// Exit status 0 and a line "planner ok ..." when all hold.
#include <stdint.h>
#include <stdio.h>

#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../paper_quant_ph_0308158_amd/csrc/planner.h"

using namespace qsim;

static int fail_count = 0;
static int rejected = 0;

#define CHECK(cond, ...)                                         \
    do {                                                         \
        if (!(cond)) {                                           \
            fprintf(stderr, "planner check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                               \
            ++fail_count;                                        \
            return;                                              \
        }                                                        \
    } while (0)

// k <- U_s k for each step in `order` (address tags: entry i starts as i).
static std::vector<uint32_t> run(uint32_t M, const std::vector<uint32_t> &order, const uint32_t *tg,
                                 const uint64_t *cm, const uint8_t *kd) {
    std::vector<uint32_t> v(1u << M);
    for (uint32_t i = 0; i < v.size(); ++i) v[i] = i;
    for (uint32_t s : order) {
        const uint64_t T = 1ull << tg[s], C = cm[s];
        for (uint64_t i = 0; i < v.size(); ++i) {
            if (kd[s]) {
                if ((i & (C | T)) == (C | T)) v[i] ^= 0x80000000u;   // a sign bit on the tag
            } else if (!(i & T) && (i & C) == C) {
                std::swap(v[i], v[i | T]);
            }
        }
    }
    return v;
}

static void check_one(std::mt19937_64 &rng, uint32_t M, uint64_t L, const PlanConfig &cfg, bool phases) {
    std::vector<uint32_t> tg(L);
    std::vector<uint64_t> cm(L);
    std::vector<uint8_t> kd(L, 0);
    for (uint64_t s = 0; s < L; ++s) {
        tg[s] = (uint32_t)(rng() % M);
        const uint32_t n = (uint32_t)(rng() % 4);
        uint64_t c = 0;
        for (uint32_t k = 0; k < n && M > 1; ++k) {
            const uint32_t b = (uint32_t)(rng() % M);
            if (b != tg[s]) c |= 1ull << b;
        }
        cm[s] = c;
        if (phases) kd[s] = (rng() % 4) == 0;
    }
    std::vector<Pass> passes;
    try {
        passes = plan_passes(M, tg.data(), cm.data(), kd.data(), L, cfg);
    } catch (const std::exception &e) {
        // Without permuted layouts every tile bit lies below 32 and every
        // tile holds the low bits: a step on a bit at or above 32 controlled
        // by a low bit fits no pass, and the planner must say so.
        bool stuck = false;
        for (uint64_t s = 0; s < L; ++s)
            if (!kd[s] && tg[s] >= 32 && (cm[s] & 31ull)) stuck = true;
        CHECK(!cfg.remap && M > 32 && stuck && std::string(e.what()).find("remap") != std::string::npos,
              "M=%u: planner failed: %s", M, e.what());
        ++rejected;
        return;
    }
    std::vector<uint32_t> order, pos(L, UINT32_MAX);
    const int K = cfg.tile_bits < (int)M ? cfg.tile_bits : (int)M;
    // the forced low bits leave one tile bit free when the state exceeds a tile
    const int low_cap = (int)M > K ? K - 1 : K;
    const uint32_t lowb = (uint32_t)(cfg.low_bits < low_cap ? cfg.low_bits : low_cap);
    const uint64_t low = lowb >= 64 ? ~0ull : ((1ull << lowb) - 1ull);
    for (size_t p = 0; p < passes.size(); ++p) {
        const uint64_t I = passes[p].tile_mask;
        CHECK(__builtin_popcountll(I) <= K, "M=%u pass %zu has %d tile bits > %d", M, p, __builtin_popcountll(I), K);
        CHECK(M >= 64 || (I >> M) == 0, "M=%u pass %zu tiles a bit >= M", M, p);
        if (p == 0 || p + 1 == passes.size()) {
            CHECK((I & low) == low, "M=%u pass %zu lacks the low bits", M, p);
            CHECK((I >> 32) == 0, "M=%u pass %zu (first/last) tiles a bit >= 32", M, p);
        }
        for (uint32_t s : passes[p].steps) {
            CHECK(s < L, "step index %u out of range", s);
            CHECK(pos[s] == UINT32_MAX, "step %u planned twice", s);
            pos[s] = (uint32_t)order.size();
            order.push_back(s);
            if (!kd[s]) CHECK(((I >> tg[s]) & 1ull) || !(cm[s] & I), "M=%u step %u inadmissible in pass %zu", M, s, p);
        }
    }
    CHECK(order.size() == L, "M=%u: %zu of %llu steps planned", M, order.size(), (unsigned long long)L);
    for (uint64_t i = 0; i < L; ++i) {
        const uint64_t Wi = kd[i] ? 0 : 1ull << tg[i], Ri = cm[i] | (kd[i] ? 1ull << tg[i] : 0);
        for (uint64_t j = i + 1; j < L; ++j) {
            const uint64_t Wj = kd[j] ? 0 : 1ull << tg[j], Rj = cm[j] | (kd[j] ? 1ull << tg[j] : 0);
            const bool commute = !(Wi & Rj) && !(Wj & Ri);
            if (!commute) CHECK(pos[i] < pos[j], "M=%u steps %llu and %llu swapped", M, (unsigned long long)i,
                                (unsigned long long)j);
        }
    }
    if (M <= 14) {
        std::vector<uint32_t> orig(L);
        for (uint64_t s = 0; s < L; ++s) orig[s] = (uint32_t)s;
        CHECK(run(M, orig, tg.data(), cm.data(), kd.data()) == run(M, order, tg.data(), cm.data(), kd.data()),
              "M=%u: reordered plan gives another result", M);
    }
}

int main() {
    std::mt19937_64 rng(20261203);
    int plans = 0;
    const uint32_t Ms[] = {3, 6, 10, 14, 18, 24, 32, 34};
    for (uint32_t M : Ms)
        for (int tb : {5, 8, 13, 14})
            for (int search : {0, 1, 2})
                for (int variant = 0; variant < 4; ++variant) {
                    PlanConfig cfg;
                    cfg.tile_bits = tb;
                    cfg.low_bits = tb < 5 ? tb : (variant & 1 ? 4 : 5);
                    cfg.mid_low_bits = variant & 2 ? 1 : 2;
                    cfg.reorder = variant != 3;
                    cfg.remap = variant != 2;
                    cfg.search = search;
                    cfg.threads = 2;
                    cfg.max_seg_steps = variant == 1 ? 7 : 1024;
                    cfg.line_bits = variant & 1 ? 3 : 4;
                    const uint64_t L = M >= 24 ? (search == 2 ? 120 : 300) : (uint64_t)(rng() % 200);
                    check_one(rng, M, L, cfg, variant >= 2);
                    ++plans;
                    if (fail_count) return 1;
                }
    // empty and one-step diagrams
    for (uint32_t M : {1u, 2u, 5u, 20u}) {
        PlanConfig cfg;
        cfg.tile_bits = 13;
        check_one(rng, M, 0, cfg, false);
        check_one(rng, M, 1, cfg, true);
        plans += 2;
    }
    if (fail_count) return 1;
    printf("planner ok: %d plans (%d rejected: no layout can place them)\n", plans, rejected);
    return 0;
}
