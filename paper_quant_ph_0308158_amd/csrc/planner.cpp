// Pass planner of the fused path (host only).
//
// A pass streams the whole state once through LDS tiles.  A tile is the set
// of 2^K rows that agree on every address bit outside a mask I of K bits.  A
// step (target t, controls C) can join a pass with mask I when
//   * t is in I: it permutes rows inside each tile (inner step), or
//   * C has no bit in I: it moves whole tiles, or leaves them, depending on
//     bits that are constant over a tile (outer step).
// A step with t outside I and a control inside I would split tiles, so it
// waits for a later pass.  This is the paper's question of which sequential
// steps can be processed together (Sec. 2(i) Parallelism), answered for
// tiles rather than single sub-matrices.
//
// Steps may be taken out of order, but only past steps they commute with:
// (t1, C1) and (t2, C2) commute when t1 is not in C2 and t2 is not in C1
// (equal targets always commute, the premise of the same-target shortcut of
// Sec. 2(i)).  The scan below keeps every step behind each earlier step it
// does not commute with, so the product of the reordered list is the
// product of the original one.
//
// A phase step (a diagonal matrix: -1 on the rows whose bits t and C are
// all 1) moves nothing, so it joins any pass: inside a tile it flips the
// sign of the rows its tile bits select, for the tiles its outside bits
// select.  In terms of commutation it writes no address bit and reads all
// of C and t: it commutes with a NOT step unless that step's target is one
// of its bits, and with every other phase step.  With write mask W (the
// NOT's target bit, none for a phase step) and read mask R (the controls,
// plus the target for a phase step), two steps commute iff neither writes
// a bit the other reads.
#include <algorithm>
#include <stdexcept>

#include "qsim_internal.h"

namespace qsim {

namespace {

inline int popc(uint64_t x) { return __builtin_popcountll(x); }

inline bool is_phase(const uint8_t *kind, uint32_t s) { return kind && kind[s] == kStepPhase; }

// Smallest mask containing `I` under which every step of `taken` (plus the
// candidate step, if any) is admissible; returns 0 if that needs more than
// `K` bits or a bit outside `allowed`.
uint64_t close_mask(uint64_t I, const std::vector<uint32_t> &taken, int cand, const uint32_t *target,
                    const uint64_t *cmask, const uint8_t *kind, int K, uint64_t allowed) {
    bool changed = true;
    while (changed) {
        changed = false;
        auto visit = [&](uint32_t q) {
            if (is_phase(kind, q)) return;
            const uint64_t T = 1ull << target[q];
            if (!(I & T) && (cmask[q] & I)) {
                I |= T;
                changed = true;
            }
        };
        for (uint32_t q : taken) visit(q);
        if (cand >= 0) visit((uint32_t)cand);
        if (popc(I) > K || (I & ~allowed)) return 0;
    }
    return I;
}

}  // namespace

std::vector<Pass> plan_passes(uint32_t M, const uint32_t *target, const uint64_t *cmask, const uint8_t *kind,
                              uint64_t L, const PlanConfig &cfg) {
    std::vector<Pass> passes;
    if (L == 0) return passes;
    const int K = std::min<int>(cfg.tile_bits, (int)M);
    const uint64_t all = (M >= 64) ? ~0ull : ((1ull << M) - 1ull);
    // Tile bits address entries inside a tile with 32-bit offsets, so their
    // physical positions lie below 32.  The first pass reads and the last
    // pass writes the natural layout (physical = logical), so their tile
    // bits are logical bits below 32; with permuted layouts between passes
    // a middle pass's tile bits sit at the bottom of both its layouts, so
    // any bit will do (this lets steps on bits 32 and up become inner).
    const uint64_t low32 = all & 0xFFFFFFFFull;
    uint64_t allowed = low32;
    auto set_allowed = [&](bool natural) { allowed = (natural || !cfg.remap) ? low32 : all; };
    const int low = std::min<int>(std::max(cfg.low_bits, 1), K);
    const uint64_t base = (1ull << low) - 1ull;
    const int cap = std::max(cfg.max_seg_steps, 1);

    // state: 0 = pending, 1 = done in an earlier pass, 2 = taken now, 3 = blocked now
    std::vector<uint8_t> state(L, 0);
    std::vector<uint32_t> pending;
    pending.reserve(L);
    for (uint64_t s = 0; s < L; ++s) pending.push_back((uint32_t)s);

    // Write and read masks (see the top of the file).
    auto WM = [&](uint32_t s) { return is_phase(kind, s) ? 0ull : 1ull << target[s]; };
    auto RM = [&](uint32_t s) { return is_phase(kind, s) ? (cmask[s] | (1ull << target[s])) : cmask[s]; };
    // Admissible in a pass with tile mask I.
    auto admissible = [&](uint32_t s, uint64_t I) {
        return is_phase(kind, s) || ((I >> target[s]) & 1ull) || !(cmask[s] & I);
    };
    // Controls of the taken NOT steps whose target lies outside mask I: bits
    // that cannot join the tile any more without pulling those targets in.
    auto outer_controls = [&](const std::vector<uint32_t> &taken, int cand, uint64_t I) {
        uint64_t U = 0;
        for (uint32_t q : taken)
            if (!is_phase(kind, q) && !((I >> target[q]) & 1ull)) U |= cmask[q];
        if (cand >= 0 && !is_phase(kind, (uint32_t)cand) && !((I >> target[cand]) & 1ull)) U |= cmask[cand];
        return U;
    };
    // A pass must still be able to grow its tile to K bits with bits that no
    // taken outer step is controlled by.
    auto completable = [&](uint64_t I, uint64_t U) {
        return popc(allowed & ~I & ~U) >= K - popc(I);
    };

    // Mask search: the greedy scan commits to tile bits in the order the
    // pending steps ask for them.  Afterwards one tile bit (not one the
    // pass must hold) is swapped for one outside bit while a scan with the
    // fixed mask admits more pending steps; that scan keeps the same
    // commutation blocking, so its steps form a valid pass.
    const bool search = cfg.search > 0 || (cfg.search < 0 && M >= 30);
    auto scan_fixed = [&](uint64_t I, std::vector<uint32_t> *take) {
        uint64_t BT = 0, BC = 0;
        bool any_blocked = false;
        int n = 0;
        for (uint32_t s : pending) {
            const bool ready = n < cap && (cfg.reorder ? !((RM(s) & BT) || (WM(s) & BC)) : !any_blocked);
            if (ready && admissible(s, I)) {
                ++n;
                if (take) take->push_back(s);
            } else {
                BT |= WM(s);
                BC |= RM(s);
                any_blocked = true;
            }
        }
        return n;
    };
    auto climb = [&](uint64_t I, uint64_t keep) {
        int best = scan_fixed(I, nullptr);
        for (int round = 0; round < 4; ++round) {
            uint64_t bestI = I;
            for (uint32_t b = 0; b < M; ++b) {
                if (!((I >> b) & 1ull) || ((keep >> b) & 1ull)) continue;
                for (uint32_t c = 0; c < M; ++c) {
                    if (((I >> c) & 1ull) || !((allowed >> c) & 1ull)) continue;
                    const uint64_t J = (I & ~(1ull << b)) | (1ull << c);
                    const int n = scan_fixed(J, nullptr);
                    if (n > best) {
                        best = n;
                        bestI = J;
                    }
                }
            }
            if (bestI == I) break;
            I = bestI;
        }
        return I;
    };

    // One pass over the pending steps, starting from tile mask `start`.
    // A step may join the pass only if it commutes with every earlier
    // pending step left behind in this scan: with BT the targets and BC the
    // controls of the steps left behind, step s is blocked exactly when one
    // of its controls is in BT or its target is in BC.
    auto build_pass = [&](uint64_t start) {
        uint64_t I = start;
        uint64_t U = 0;
        uint64_t BT = 0, BC = 0;
        bool any_blocked = false;
        std::vector<uint32_t> taken;
        for (uint32_t s : pending) {
            if ((int)taken.size() >= cap) break;
            const bool ready = cfg.reorder ? !((RM(s) & BT) || (WM(s) & BC)) : !any_blocked;
            if (!ready) {
                state[s] = 3;
                BT |= WM(s);
                BC |= RM(s);
                any_blocked = true;
                continue;
            }
            const uint64_t T = 1ull << target[s];
            bool took = false;
            if (is_phase(kind, s)) {
                took = true;                       // moves nothing: any tile
            } else if (I & T) {
                took = true;                       // inner step: U unchanged
            } else if (!(cmask[s] & I) && completable(I, U | cmask[s])) {
                U |= cmask[s];                     // outer step
                took = true;
            } else {
                // make it an inner step by adding its target (and the closure)
                const uint64_t J = close_mask(I | T, taken, (int)s, target, cmask, kind, K, allowed);
                if (J) {
                    const uint64_t UJ = outer_controls(taken, (int)s, J);
                    if (completable(J, UJ)) {
                        I = J;
                        U = UJ;
                        took = true;
                    }
                }
            }
            if (took) {
                taken.push_back(s);
                state[s] = 2;
            } else {
                state[s] = 3;
                BT |= WM(s);
                BC |= RM(s);
                any_blocked = true;
            }
        }
        if (taken.empty()) {
            for (uint32_t s : pending) state[s] = 0;
            return Pass{};
        }
        // Widen the tile to K bits with the lowest bits that no outer step of
        // the pass is controlled by; every taken step stays admissible.
        for (uint32_t b = 0; b < M && popc(I) < K; ++b) {
            const uint64_t B = 1ull << b;
            if ((I & B) || (U & B) || !(allowed & B)) continue;
            I |= B;
        }
        Pass p;
        p.tile_mask = I;
        if (search) {
            // A fixed-mask scan admits every step the greedy scan took (the
            // final mask only added bits no outer step is controlled by), so
            // the climb can only add steps.
            p.tile_mask = climb(I, start);
            for (uint32_t s : pending) state[s] = 0;
            scan_fixed(p.tile_mask, &p.steps);
            for (uint32_t s : p.steps) state[s] = 2;
        } else {
            p.steps = taken;
        }
        std::vector<uint32_t> next;
        next.reserve(pending.size());
        for (uint32_t s : pending) {
            if (state[s] == 2) state[s] = 1;
            else { state[s] = 0; next.push_back(s); }
        }
        pending.swap(next);
        return p;
    };

    // The first pass reads, and the last pass writes, the state in its
    // natural bit order, so their tiles must hold the low address bits that
    // make each tile a set of long contiguous runs.  Passes in between see
    // layouts permuted to suit them and may start from fewer low bits.
    const int mid_low = std::min<int>(std::max(cfg.mid_low_bits > 0 ? cfg.mid_low_bits : low, 1), low);
    const uint64_t mid_base = (1ull << mid_low) - 1ull;
    // Consecutive tiles must share at least min_overlap bits: between passes
    // the state is laid out with the shared bits lowest, so the pass that
    // writes it does so in runs of 2^(shared bits) entries, which should fill
    // whole cache lines.  A middle pass therefore starts from the low bits
    // plus bits of the previous tile, preferring the targets of the next
    // pending steps (which the tile would take in anyway).
    const int min_ov = std::min(cfg.min_overlap, K - 1);
    auto seed_from = [&](uint64_t prev) {
        uint64_t I = mid_base;
        for (uint32_t s : pending) {
            if (popc(I & prev) >= min_ov) break;
            if (is_phase(kind, s)) continue;
            const uint64_t T = 1ull << target[s];
            if ((prev & T) && (allowed & T)) I |= T;
        }
        for (uint32_t b = 0; b < M && popc(I & prev) < min_ov; ++b)
            if ((prev >> b) & 1ull) I |= 1ull << b;
        return I;
    };
    // A seeded start can leave no step admissible; the plain start always
    // admits the first pending step.
    auto next_pass = [&](uint64_t start, uint64_t fallback) {
        Pass p = build_pass(start);
        if (p.steps.empty() && start != fallback) p = build_pass(fallback);
        if (p.steps.empty()) throw std::logic_error("planner made no progress");
        return p;
    };
    while (!pending.empty()) {
        set_allowed(passes.empty());
        passes.push_back(passes.empty() ? next_pass(base, base)
                                        : next_pass(seed_from(passes.back().tile_mask), mid_base));
    }
    if ((passes.back().tile_mask & base) != base || (passes.back().tile_mask & ~low32)) {
        // The last pass writes the natural layout: re-plan its steps from
        // the full base with tile bits below 32.  Should that leave a step
        // no such tile admits (a target above bit 31 with a control among
        // the base bits), keep the pass and end with a pass without steps
        // that only moves the state back to the natural layout.
        const Pass last = passes.back();
        passes.pop_back();
        for (uint32_t s : last.steps) state[s] = 0;
        pending = last.steps;
        set_allowed(true);
        std::vector<Pass> redo;
        bool ok = true;
        while (!pending.empty() && ok) {
            Pass p = build_pass(base);
            if (p.steps.empty()) ok = false;
            else redo.push_back(std::move(p));
        }
        if (ok) {
            for (Pass &p : redo) passes.push_back(std::move(p));
        } else {
            for (uint32_t s : last.steps) state[s] = 1;
            pending.clear();
            passes.push_back(last);
            Pass tail;
            tail.tile_mask = base;
            for (uint32_t b = 0; b < 32 && b < M && popc(tail.tile_mask) < K; ++b) tail.tile_mask |= 1ull << b;
            passes.push_back(tail);
        }
    }
    return passes;
}

}  // namespace qsim
