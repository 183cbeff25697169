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
#include <atomic>
#include <set>
#include <stdexcept>
#include <thread>

#include "host_threads.h"
#include "planner.h"

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

// The diagram and the planner's settings, with each step's write mask W
// (a NOT's target bit, none for a phase step) and read mask R (the
// controls, plus the target for a phase step).
struct Diagram {
    uint32_t M;
    int K;
    const uint32_t *target;
    const uint64_t *cmask;
    const uint8_t *kind;
    const PlanConfig &cfg;
    int cap;
    std::vector<uint64_t> W, R;

    Diagram(uint32_t M_, const uint32_t *t, const uint64_t *c, const uint8_t *k, uint64_t L, const PlanConfig &cf)
        : M(M_), K(std::min<int>(cf.tile_bits, (int)M_)), target(t), cmask(c), kind(k), cfg(cf),
          cap(std::max(cf.max_seg_steps, 1)), W(L), R(L) {
        for (uint64_t s = 0; s < L; ++s) {
            W[s] = is_phase(kind, (uint32_t)s) ? 0ull : 1ull << target[s];
            R[s] = is_phase(kind, (uint32_t)s) ? (cmask[s] | (1ull << target[s])) : cmask[s];
        }
    }
    // Admissible in a pass with tile mask I: a phase step always; a NOT step
    // if its target is in I or none of its controls is.
    bool admissible(uint32_t s, uint64_t I) const { return !((W[s] & ~I) && (R[s] & I)); }
    // Step s may run ahead of the steps left behind so far in a scan, whose
    // write masks OR to BT and read masks to BC, iff it commutes with all of
    // them: it reads none of BT and writes none of BC.  Without reordering
    // any step left behind blocks every later one.
    bool ready(uint32_t s, uint64_t BT, uint64_t BC, bool any_blocked) const {
        return cfg.reorder ? !((R[s] & BT) || (W[s] & BC)) : !any_blocked;
    }
};

// Scan the pending steps in order with a fixed tile mask I: a step joins
// the pass when it is ready and admissible.  Returns the number taken;
// `take` and `rest` (if given) receive the taken and the remaining steps.
int scan_fixed(const Diagram &d, const std::vector<uint32_t> &pending, uint64_t I, std::vector<uint32_t> *take,
               std::vector<uint32_t> *rest) {
    uint64_t BT = 0, BC = 0;
    bool any_blocked = false;
    int n = 0;
    for (uint32_t s : pending) {
        if (n < d.cap && d.ready(s, BT, BC, any_blocked) && d.admissible(s, I)) {
            ++n;
            if (take) take->push_back(s);
        } else {
            BT |= d.W[s];
            BC |= d.R[s];
            any_blocked = true;
            if (rest) rest->push_back(s);
        }
    }
    return n;
}

// The pending steps' masks in scan order, for scan_many.  A step left
// behind adds Wb to BT and Rb to BC: its own masks when reordering, all
// bits otherwise (every later step then counts as blocked, since each step
// writes or reads at least one bit).
struct PendingMasks {
    std::vector<uint64_t> W, R, Wb, Rb;
    PendingMasks(const Diagram &d, const std::vector<uint32_t> &pending) {
        W.reserve(pending.size());
        R.reserve(pending.size());
        Wb.reserve(pending.size());
        Rb.reserve(pending.size());
        for (uint32_t s : pending) {
            W.push_back(d.W[s]);
            R.push_back(d.R[s]);
            Wb.push_back(d.cfg.reorder ? d.W[s] : ~0ull);
            Rb.push_back(d.cfg.reorder ? d.R[s] : ~0ull);
        }
    }
};

// scan_fixed's count for each of `nm` masks, 64 masks side by side per
// sweep over the steps (branch-free, so the inner loop vectorises).  The
// same code is compiled for AVX-512, AVX2 and the baseline instruction set
// and picked by what the host CPU supports.
template <int kLanes>
__attribute__((always_inline)) inline void scan_lanes(const PendingMasks &p, int cap, const uint64_t *masks, size_t nm, int *counts) {
    const size_t L = p.W.size();
    for (size_t j0 = 0; j0 < nm; j0 += kLanes) {
        const int n = (int)std::min<size_t>(kLanes, nm - j0);
        uint64_t I[kLanes], BT[kLanes], BC[kLanes], cnt[kLanes];
        for (int j = 0; j < kLanes; ++j) {
            I[j] = j < n ? masks[j0 + j] : 0ull;
            BT[j] = BC[j] = cnt[j] = 0;
        }
        for (size_t s = 0; s < L; ++s) {
            const uint64_t W = p.W[s], R = p.R[s], Wb = p.Wb[s], Rb = p.Rb[s];
            for (int j = 0; j < kLanes; ++j) {
                const uint64_t blocked = (R & BT[j]) | (W & BC[j]);
                const uint64_t inadm = (uint64_t)((W & ~I[j]) != 0) & (uint64_t)((R & I[j]) != 0);
                const uint64_t take = (uint64_t)(blocked == 0) & (inadm ^ 1ull) & (uint64_t)(cnt[j] < (uint64_t)cap);
                const uint64_t left = take - 1ull;   // all ones when the step is left behind
                BT[j] |= Wb & left;
                BC[j] |= Rb & left;
                cnt[j] += take;
            }
        }
        for (int j = 0; j < n; ++j) counts[j0 + j] = (int)cnt[j];
    }
}

__attribute__((target("avx512f,avx512vl,avx512bw,avx512dq")))
void scan_many_avx512(const PendingMasks &p, int cap, const uint64_t *masks, size_t nm, int *counts) {
    scan_lanes<64>(p, cap, masks, nm, counts);
}

__attribute__((target("avx2")))
void scan_many_avx2(const PendingMasks &p, int cap, const uint64_t *masks, size_t nm, int *counts) {
    scan_lanes<64>(p, cap, masks, nm, counts);
}

void scan_many(const PendingMasks &p, int cap, const uint64_t *masks, size_t nm, int *counts) {
    static const int isa = __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512vl") &&
                                   __builtin_cpu_supports("avx512bw") && __builtin_cpu_supports("avx512dq")
                               ? 2
                               : (__builtin_cpu_supports("avx2") ? 1 : 0);
    if (isa == 2) scan_many_avx512(p, cap, masks, nm, counts);
    else if (isa == 1) scan_many_avx2(p, cap, masks, nm, counts);
    else scan_lanes<64>(p, cap, masks, nm, counts);
}

// Hill climb on the tile mask: in each round every swap of one tile bit
// (not in `keep`) for one outside bit in `allowed` is scanned, and the
// first swap that admits the most pending steps is taken if it beats the
// current mask.  `alts` (if given) receives the best other masks of the
// last round scanned, most steps first.
uint64_t climb(const Diagram &d, const PendingMasks &p, uint64_t I, uint64_t keep, uint64_t allowed, int rounds,
               size_t n_alts, std::vector<uint64_t> *alts) {
    int best = 0;
    scan_many(p, d.cap, &I, 1, &best);
    std::vector<uint64_t> cand;
    std::vector<int> cnt;
    for (int round = 0; round < rounds; ++round) {
        cand.clear();
        for (uint32_t b = 0; b < d.M; ++b) {
            if (!((I >> b) & 1ull) || ((keep >> b) & 1ull)) continue;
            for (uint32_t c = 0; c < d.M; ++c) {
                if (((I >> c) & 1ull) || !((allowed >> c) & 1ull)) continue;
                cand.push_back((I & ~(1ull << b)) | (1ull << c));
            }
        }
        cnt.assign(cand.size(), 0);
        scan_many(p, d.cap, cand.data(), cand.size(), cnt.data());
        size_t arg = cand.size();
        for (size_t k = 0; k < cand.size(); ++k)
            if (cnt[k] > best) {
                best = cnt[k];
                arg = k;
            }
        const bool last = arg == cand.size() || round + 1 == rounds;
        if (last && alts) {
            std::vector<size_t> order(cand.size());
            for (size_t k = 0; k < order.size(); ++k) order[k] = k;
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cnt[a] > cnt[b]; });
            const uint64_t chosen = arg == cand.size() ? I : cand[arg];
            for (size_t k = 0; k < order.size() && alts->size() < n_alts; ++k)
                if (cand[order[k]] != chosen) alts->push_back(cand[order[k]]);
        }
        if (arg == cand.size()) break;
        I = cand[arg];
    }
    return I;
}

// Greedy scan from tile mask `start`: steps are taken in order (those left
// behind block the ones they do not commute with); a NOT step whose target
// is outside the mask and which has a control inside it adds its target
// (with the closure over the steps already taken) while the mask has room.
// The mask is then widened to K bits with the lowest bits that no outer
// step is controlled by.  Returns 0 if no step was taken.
uint64_t greedy_scan(const Diagram &d, const std::vector<uint32_t> &pending, uint64_t start, uint64_t allowed,
                     std::vector<uint32_t> &taken) {
    const int K = d.K;
    // Controls of the taken NOT steps whose target lies outside mask I: bits
    // that cannot join the tile any more without pulling those targets in.
    auto outer_controls = [&](int cand, uint64_t I) {
        uint64_t U = 0;
        for (uint32_t q : taken)
            if (!is_phase(d.kind, q) && !((I >> d.target[q]) & 1ull)) U |= d.cmask[q];
        if (cand >= 0 && !is_phase(d.kind, (uint32_t)cand) && !((I >> d.target[cand]) & 1ull)) U |= d.cmask[cand];
        return U;
    };
    // A pass must still be able to grow its tile to K bits with bits that no
    // taken outer step is controlled by.
    auto completable = [&](uint64_t I, uint64_t U) { return popc(allowed & ~I & ~U) >= K - popc(I); };
    uint64_t I = start, U = 0, BT = 0, BC = 0;
    bool any_blocked = false;
    taken.clear();
    for (uint32_t s : pending) {
        if ((int)taken.size() >= d.cap) break;
        bool took = false;
        if (d.ready(s, BT, BC, any_blocked)) {
            const uint64_t T = 1ull << d.target[s];
            if (is_phase(d.kind, s)) {
                took = true;                       // moves nothing: any tile
            } else if (I & T) {
                took = true;                       // inner step: U unchanged
            } else if (!(d.cmask[s] & I) && completable(I, U | d.cmask[s])) {
                U |= d.cmask[s];                   // outer step
                took = true;
            } else {
                // make it an inner step by adding its target (and the closure)
                const uint64_t J = close_mask(I | T, taken, (int)s, d.target, d.cmask, d.kind, K, allowed);
                if (J) {
                    const uint64_t UJ = outer_controls((int)s, J);
                    if (completable(J, UJ)) {
                        I = J;
                        U = UJ;
                        took = true;
                    }
                }
            }
        }
        if (took) {
            taken.push_back(s);
        } else {
            BT |= d.W[s];
            BC |= d.R[s];
            any_blocked = true;
        }
    }
    if (taken.empty()) return 0;
    for (uint32_t b = 0; b < d.M && popc(I) < K; ++b) {
        const uint64_t B = 1ull << b;
        if ((I & B) || (U & B) || !(allowed & B)) continue;
        I |= B;
    }
    return I;
}

uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

namespace {

// Beam search over whole plans.  Taking the most steps in every pass is
// not the fewest passes overall: which of several equally good masks a pass
// takes decides what the later passes can take together.  The search keeps
// the `kBeam` cheapest partial plans (pending steps, plus a charge for each
// thin boundary, below) after each number of passes; each is extended by
// the masks of a hill climb from its greedy mask (the best mask and the
// next best of its last round) and by climbs from seeded random masks.  A
// plan ends with a pass whose tile holds the low bits and lies below bit 32
// (it writes the natural layout).  The search runs only while it can still
// beat `limit` passes; random draws are seeded from the pass number and the
// plan's rank, so the result does not depend on the thread count.
std::vector<Pass> beam_plan(const Diagram &d, uint64_t L, uint64_t base, uint64_t mid_base, uint64_t low32,
                            uint64_t all, size_t limit) {
    constexpr size_t kBeam = 6, kAlts = 4;
    constexpr int kRestarts = 4, kRounds = 4, kRestartRounds = 8;
    const int threads = d.cfg.threads > 0 ? d.cfg.threads
                                          : (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    const uint64_t mid_allowed = d.cfg.remap ? all : low32;
    if (popc(low32) < d.K || popc(mid_allowed) < d.K) return {};
    // Consecutive tiles that share fewer bits than a 128-byte line spans
    // make the pass between them read part lines (measured: such a pair of
    // passes costs about a fifth of a pass more), so partial plans are
    // ranked by pending steps plus, per such boundary, a quarter of the
    // steps an average pass of the greedy plan takes.
    const size_t thin_cost = std::max<size_t>(1, L / (4 * limit));
    struct Node {
        std::vector<uint32_t> pending;
        std::vector<uint64_t> masks;
        size_t thin = 0;
    };
    auto cost = [&](const Node &n) { return n.pending.size() + thin_cost * n.thin; };
    auto is_thin = [&](uint64_t a, uint64_t b) { return popc(a & b) < d.cfg.line_bits; };
    std::vector<Node> beam(1);
    beam[0].pending.resize(L);
    for (uint64_t s = 0; s < L; ++s) beam[0].pending[s] = (uint32_t)s;
    for (size_t level = 0; level + 1 < limit; ++level) {
        // Candidate masks of every partial plan, as independent tasks: the
        // climb from the greedy mask (with its alternatives), the climbs from
        // random masks, and the check whether one last pass can finish it.
        std::vector<PendingMasks> pms;
        pms.reserve(beam.size());
        for (const Node &n : beam) pms.emplace_back(d, n.pending);
        constexpr size_t kTasks = kRestarts + 2;
        std::vector<std::vector<uint64_t>> out(beam.size() * kTasks);
        parallel_for(beam.size() * kTasks, threads, [&](size_t q) {
            const size_t k = q / kTasks, task = q % kTasks;
            const Node &n = beam[k];
            const PendingMasks &pm = pms[k];
            const uint64_t start = level == 0 ? base : mid_base;
            const uint64_t allowed = level == 0 ? low32 : mid_allowed;
            std::vector<uint32_t> taken;
            if (task == 0) {
                const uint64_t g = greedy_scan(d, n.pending, start, allowed, taken);
                if (g) {
                    std::vector<uint64_t> alts;
                    out[q].push_back(climb(d, pm, g, start, allowed, kRounds, kAlts - 1, &alts));
                    out[q].insert(out[q].end(), alts.begin(), alts.end());
                }
            } else if (task <= (size_t)kRestarts) {
                uint64_t seed = ((uint64_t)level << 40) ^ ((uint64_t)k << 8) ^ (uint64_t)task;
                uint64_t I = start;
                while (popc(I) < d.K) {
                    const uint32_t b = (uint32_t)(splitmix64(seed) % d.M);
                    if ((allowed >> b) & 1ull) I |= 1ull << b;
                }
                out[q].push_back(climb(d, pm, I, start, allowed, kRestartRounds, 0, nullptr));
            } else if (level > 0) {
                // a last pass: the low bits, below bit 32 (the first pass's
                // masks hold them already)
                const uint64_t gf = greedy_scan(d, n.pending, base, low32, taken);
                if (gf) out[q].push_back(climb(d, pm, gf, base, low32, kRounds, 0, nullptr));
            }
        });
        std::vector<std::vector<uint64_t>> cands(beam.size());
        std::vector<uint64_t> final_mask(beam.size(), 0);
        for (size_t k = 0; k < beam.size(); ++k) {
            for (size_t task = 0; task + 1 < kTasks; ++task)
                cands[k].insert(cands[k].end(), out[k * kTasks + task].begin(), out[k * kTasks + task].end());
            const std::vector<uint64_t> &f = level == 0 ? out[k * kTasks] : out[k * kTasks + kTasks - 1];
            if (!f.empty() && (size_t)scan_fixed(d, beam[k].pending, f[0], nullptr, nullptr) == beam[k].pending.size())
                final_mask[k] = f[0];
        }
        // Of the plans that can end with this pass, the one with the fewest
        // thin boundaries (the first such in rank order).
        auto thin_at_end = [&](size_t j) {
            return beam[j].thin + (level > 0 && is_thin(beam[j].masks.back(), final_mask[j]) ? 1 : 0);
        };
        size_t end = beam.size();
        for (size_t k = 0; k < beam.size(); ++k)
            if (final_mask[k] && (end == beam.size() || thin_at_end(k) < thin_at_end(end))) end = k;
        if (end < beam.size()) {
            // replay its masks into passes
            const size_t k = end;
            std::vector<Pass> plan;
            std::vector<uint32_t> pending(L);
            for (uint64_t s = 0; s < L; ++s) pending[s] = (uint32_t)s;
            std::vector<uint64_t> masks = beam[k].masks;
            masks.push_back(final_mask[k]);
            for (uint64_t I : masks) {
                Pass p;
                p.tile_mask = I;
                std::vector<uint32_t> rest;
                scan_fixed(d, pending, I, &p.steps, &rest);
                pending.swap(rest);
                plan.push_back(std::move(p));
            }
            if (!pending.empty()) throw std::logic_error("beam plan left steps behind");
            return plan;
        }
        // Extend every partial plan by its candidate masks; keep the kBeam
        // cheapest extensions, one per set of pending steps.
        std::vector<Node> next;
        for (size_t k = 0; k < beam.size(); ++k) {
            for (uint64_t I : cands[k]) {
                Node x;
                std::vector<uint32_t> take;
                scan_fixed(d, beam[k].pending, I, &take, &x.pending);
                if (take.empty() || x.pending.empty()) continue;
                x.masks = beam[k].masks;
                x.thin = beam[k].thin + (level > 0 && is_thin(x.masks.back(), I) ? 1 : 0);
                x.masks.push_back(I);
                next.push_back(std::move(x));
            }
        }
        if (next.empty()) return {};
        std::stable_sort(next.begin(), next.end(), [&](const Node &a, const Node &b) { return cost(a) < cost(b); });
        std::vector<Node> kept;
        std::set<std::vector<uint32_t>> seen;
        for (Node &x : next) {
            if (kept.size() == kBeam) break;
            if (seen.insert(x.pending).second) kept.push_back(std::move(x));
        }
        beam.swap(kept);
    }
    return {};
}

}  // namespace

std::vector<Pass> plan_passes(uint32_t M, const uint32_t *target, const uint64_t *cmask, const uint8_t *kind,
                              uint64_t L, const PlanConfig &cfg) {
    std::vector<Pass> passes;
    if (L == 0) return passes;
    const Diagram d(M, target, cmask, kind, L, cfg);
    const int K = d.K;
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
    // The forced low bits leave a tile bit free whenever the state is larger
    // than one tile: a step whose target lies outside them and whose control
    // lies among them needs its target in the tile.
    const int low = std::min<int>(std::max(cfg.low_bits, 1), (int)M > K ? K - 1 : K);
    const uint64_t base = (1ull << low) - 1ull;
    std::vector<uint32_t> pending(L);
    for (uint64_t s = 0; s < L; ++s) pending[s] = (uint32_t)s;

    // Mask search: the greedy scan commits to tile bits in the order the
    // pending steps ask for them.  Afterwards one tile bit (not one the
    // pass must hold) is swapped for one outside bit while a scan with the
    // fixed mask admits more pending steps; that scan keeps the same
    // commutation blocking, so its steps form a valid pass.  Level 2 adds a
    // beam search over whole plans (beam_plan); both are on by default from
    // M = 30, where a pass takes tens of milliseconds.
    const int search = cfg.search >= 0 ? cfg.search : (M >= 30 ? 2 : cfg.search_small);

    // One pass over the pending steps, starting from tile mask `start`.
    auto build_pass = [&](uint64_t start) {
        Pass p;
        const uint64_t I = greedy_scan(d, pending, start, allowed, p.steps);
        if (!I) return Pass{};
        p.tile_mask = I;
        if (search) {
            // A fixed-mask scan admits every step the greedy scan took (the
            // final mask only added bits no outer step is controlled by), so
            // the climb can only add steps.
            const PendingMasks pm(d, pending);
            p.tile_mask = climb(d, pm, I, start, allowed, 4, 0, nullptr);
            p.steps.clear();
        }
        std::vector<uint32_t> take, rest;
        scan_fixed(d, pending, p.tile_mask, &take, &rest);
        if (search) p.steps = take;
        else {
            // keep the greedy scan's own steps; the rest stay pending
            std::vector<uint8_t> in(L, 0);
            for (uint32_t s : p.steps) in[s] = 1;
            rest.clear();
            for (uint32_t s : pending)
                if (!in[s]) rest.push_back(s);
        }
        pending.swap(rest);
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
        if (p.steps.empty() && passes.empty() && cfg.remap && (allowed & ~low32) == 0 && all != low32) {
            // The first pass reads the natural layout, so its tile bits lie
            // below 32; when every step it could take waits behind one that
            // targets a bit at or above 32 with a control among the low
            // bits, a pass without steps moves the state into a permuted
            // layout in which the next pass may tile that bit.
            Pass head;
            head.tile_mask = base;
            for (uint32_t b = 0; b < 32 && b < M && popc(head.tile_mask) < K; ++b) head.tile_mask |= 1ull << b;
            return head;
        }
        if (p.steps.empty())
            throw std::logic_error(cfg.remap ? "planner made no progress"
                                             : "a step targets an address bit at or above 32 with a control that "
                                               "every tile holds; this needs permuted layouts (remap on)");
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
            pending.clear();
            passes.push_back(last);
            Pass tail;
            tail.tile_mask = base;
            for (uint32_t b = 0; b < 32 && b < M && popc(tail.tile_mask) < K; ++b) tail.tile_mask |= 1ull << b;
            passes.push_back(tail);
        }
    }
    // Every tile holds the middle low bits, so consecutive tiles share at
    // least those; the beam search keeps no other overlap.  Its host time
    // grows with L times the number of passes (each pass level scans the
    // pending steps): long diagrams keep the climb's plan.
    constexpr double kBeamWork = 4e6;
    if (search >= 2 && min_ov <= mid_low && passes.size() > 2 && (double)L * (double)passes.size() <= kBeamWork) {
        std::vector<Pass> b = beam_plan(d, L, base, mid_base, low32, all, passes.size());
        if (!b.empty() && b.size() < passes.size()) return b;
    }
    return passes;
}

}  // namespace qsim
