// Pass planner of the fused path: host-only declarations (no HIP), so the
// planner also builds with a plain C++ compiler (the sanitizer checks).
#pragma once

#include <stdint.h>

#include <vector>

namespace qsim {

// Step kinds as the library stores them (the public qsim_step_kind values).
constexpr uint8_t kStepNot = 0;
constexpr uint8_t kStepPhase = 1;

// Host-side plan of the fused path.
struct Pass {
    uint64_t tile_mask = 0;          // address bits inside a tile
    std::vector<uint32_t> steps;     // original step indices, execution order
};

struct PlanConfig {
    int tile_bits = 13;
    int low_bits = 5;       // low address bits in the tiles of the first and last pass
    int mid_low_bits = 0;   // same for the passes in between (0 = low_bits)
    int min_overlap = 0;    // tile bits a middle pass shares with the previous one
    int max_seg_steps = 1024;
    bool reorder = true;
    int search = -1;        // tile-mask search: 0 off, 1 hill climb per pass, 2 climb + beam
                            // search over whole plans, -1 by size: climb + beam for M >= 30,
                            // search_small below
    int search_small = 0;   // the search level of -1 below M = 30
    bool remap = true;      // permuted layouts between passes (middle tiles may use bits >= 32)
    int threads = 0;        // host threads of the beam search (0 = hardware threads, at most 16)
    int line_bits = 4;      // address bits a 128-byte line spans (4: 8-byte entries, 3: 16-byte)
};

// Split steps into passes (see planner.cpp).
// kind may be null (every step a controlled NOT).
std::vector<Pass> plan_passes(uint32_t M, const uint32_t *target, const uint64_t *cmask, const uint8_t *kind,
                              uint64_t L, const PlanConfig &cfg);

}  // namespace qsim
