// C ABI of libqsim (declared in include/qsim.h): state handles, argument
// validation, the choice between the small-state, fused-pass and direct
// kernels, plan upload and the read/write of contiguous portions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <chrono>
#include <array>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <functional>
#include <cmath>
#include <new>
#include <string>
#include <stdexcept>
#include <system_error>
#include <vector>
#include <unordered_set>
#include <exception>
#include <memory>
#include <thread>

#include <unistd.h>

#include "../../include/qsim.h"
#include "host_threads.h"
#include "qsim_internal.h"

using namespace qsim;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

// Host-side fault injection for tests of the error paths.  With
// QSIM_FAULT_INJECT = "<site>:<n>" the n-th check of <site> (counted from 1
// since the variable last changed) reports a HIP error after the real call
// has succeeded, so the error handling runs while the device sees nothing
// unusual.  Sites: "launch" (each kernel launch of an apply), "upload" (the
// plan upload of an apply), "read" (a portion read), "batch" (a batched
// launch).  A site is matched by its whole name.
hipError_t injected(const char *site) {
    const char *v = std::getenv("QSIM_FAULT_INJECT");
    if (!v || !*v) return hipSuccess;
    static std::mutex mu;
    static std::string spec;
    static uint64_t count = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (spec != v) {
        spec = v;
        count = 0;
    }
    const char *colon = std::strchr(v, ':');
    if (!colon || (size_t)(colon - v) != std::strlen(site) || std::strncmp(v, site, colon - v) != 0) return hipSuccess;
    const uint64_t n = std::strtoull(colon + 1, nullptr, 10);
    return ++count == n ? hipErrorUnknown : hipSuccess;
}

// The same for host exceptions: throws std::bad_alloc, as an allocation that
// fails would, at the n-th check of `site`.  Sites: "host" (each planning of
// a diagram, on the planning threads of a batch too), "host-launch" (after
// each kernel launch of an apply, where a timing record would be stored).
void injected_throw(const char *site) {
    if (injected(site) != hipSuccess) throw std::bad_alloc();
}

std::atomic<uint64_t> g_allocated{0};

// Optional cap on the bytes that qsim_state_create may allocate, from the
// environment (QSIM_HBM_BUDGET_BYTES); 0 = no cap beyond the device's.
uint64_t budget_bytes() {
    const char *s = std::getenv("QSIM_HBM_BUDGET_BYTES");
    if (!s || !*s) return 0;
    return std::strtoull(s, nullptr, 10);
}

uint32_t elem_of(qsim_dtype d) { return d == QSIM_C64 ? 8u : (d == QSIM_C128 ? 16u : 0u); }

int validate_steps(uint32_t M, const qsim_step *steps, uint64_t L) {
    if (L > 0 && steps == nullptr) return fail(QSIM_ERR_INVALID, "steps is NULL with L > 0");
    if (L > 0xFFFFFFFFull) return fail(QSIM_ERR_INVALID, "too many steps");
    const uint64_t all = (M >= 64) ? ~0ull : ((1ull << M) - 1ull);
    for (uint64_t s = 0; s < L; ++s) {
        const qsim_step &st = steps[s];
        if (st.kind != QSIM_STEP_NOT && st.kind != QSIM_STEP_PHASE)
            return fail(QSIM_ERR_INVALID, "step " + std::to_string(s) + ": unknown kind " + std::to_string(st.kind));
        if (st.target >= M)
            return fail(QSIM_ERR_INVALID, "step " + std::to_string(s) + ": target " + std::to_string(st.target) +
                                              " >= M = " + std::to_string(M));
        if (st.control_mask & ~all)
            return fail(QSIM_ERR_INVALID, "step " + std::to_string(s) + ": control bit >= M");
        if ((st.control_mask >> st.target) & 1ull)
            return fail(QSIM_ERR_INVALID, "step " + std::to_string(s) + ": target is one of its own controls");
    }
    return QSIM_OK;
}

// The steps as separate arrays (planner input).
struct StepLists {
    std::vector<uint32_t> tg;
    std::vector<uint64_t> cm;
    std::vector<uint8_t> kd;
    bool any_phase = false;
};

StepLists split_steps(const qsim_step *steps, uint64_t L) {
    injected_throw("host");
    StepLists o;
    o.tg.resize(L);
    o.cm.resize(L);
    o.kd.resize(L);
    for (uint64_t i = 0; i < L; ++i) {
        o.tg[i] = steps[i].target;
        o.cm[i] = steps[i].control_mask;
        o.kd[i] = steps[i].kind == QSIM_STEP_PHASE ? kStepPhase : kStepNot;
        o.any_phase |= o.kd[i] == kStepPhase;
    }
    return o;
}

// Bits a step reads at its place in the walk: the controls, plus the target
// for a phase step (whose rows are those with target and controls all 1).
inline uint64_t phase_mask(const qsim_step &st) { return st.control_mask | (1ull << st.target); }

struct Tuning {
    int tile_bits;
    int low_bits;
    int max_seg_steps;
    bool reorder;
    int small_bits;
    uint32_t variant;     // 0 = one tile per workgroup, 1 = persistent
    uint32_t wg_per_cu;
    uint32_t outer_order; // 0 = lowest outside bit fastest, 1 = highest fastest
    bool remap;           // permuted layouts between passes
    int mid_low_bits;     // forced low bits of the passes in between
    int min_overlap;      // tile bits shared by consecutive passes
    uint32_t rows_eb;     // log2 of the tile rows each thread owns
    int plan_search;      // -1 = by size, 0 = off, 1 = climb, 2 = climb + beam search
    bool xcd_swizzle;     // consecutive tiles on one XCD (one-tile-per-workgroup kernel)
    uint32_t product_cut; // product first pass: partials staged down to just above bit cut - 1
};

Tuning default_tuning(uint32_t elem) {
    // 16-byte entries: 2^12-entry tiles (64 KiB, two one-tile workgroups
    // per CU) planned with the mask climb and one forced low bit in the
    // middle passes reach the pass count of 2^13-entry tiles with faster
    // passes (M = 26, L = 200: 7 passes at 71.1 % of peak, 2.80 ms per
    // apply, against 7 persistent passes of 2^13 entries at 68.9 %, 2.88 ms).
    Tuning t;
    t.tile_bits = elem == 8 ? 13 : 12;   // 64 KiB of LDS per tile
    t.low_bits = elem == 8 ? 5 : 4;      // >= 256 contiguous bytes per tile row run
    t.max_seg_steps = 1024;
    t.reorder = true;
    t.small_bits = elem == 8 ? 14 : 13;  // whole state in 128 KiB of LDS
    t.variant = 0;                       // two one-tile workgroups per CU
    t.wg_per_cu = 0;
    t.outer_order = 0;
    t.remap = true;
    t.mid_low_bits = elem == 8 ? 2 : 1;
    t.min_overlap = 1;                   // no overlap requirement (measured best)
    t.rows_eb = 5;
    t.plan_search = -1;
    t.xcd_swizzle = true;
    // Product first pass: a quarter-tile table (16 KiB for 2^13 8-byte
    // entries) and two products per entry at the store; at M = 32 the
    // pass takes 6.25 ms against 9.8 ms with the whole tile staged.
    t.product_cut = 2;
    return t;
}

// The external form of a tuning (every field set).
void export_tuning_to(const Tuning &t, qsim_tuning *out) {
    std::memset(out, 0, sizeof(*out));
    out->tile_bits = (uint32_t)t.tile_bits;
    out->low_bits = (uint32_t)t.low_bits;
    out->max_seg_steps = (uint32_t)t.max_seg_steps;
    out->reorder = t.reorder ? 1u : 2u;
    out->small_bits = (uint32_t)t.small_bits;
    out->kernel_variant = t.variant + 1;
    out->wg_per_cu = t.wg_per_cu;
    out->outer_order = t.outer_order + 1;
    out->remap = t.remap ? 1u : 2u;
    out->mid_low_bits = (uint32_t)t.mid_low_bits;
    out->min_overlap = (uint32_t)t.min_overlap;
    out->rows_per_thread = 1u << t.rows_eb;
    out->plan_search = t.plan_search < 0 ? 0u : (uint32_t)t.plan_search + 1u;
    out->xcd_swizzle = t.xcd_swizzle ? 2u : 1u;
    out->product_stage = t.product_cut + 1u;
}

int tuning_from(const qsim_tuning *in, uint32_t elem, Tuning *out) {
    Tuning t = default_tuning(elem);
    if (in) {
        if (in->tile_bits) t.tile_bits = (int)in->tile_bits;
        if (in->low_bits) t.low_bits = (int)in->low_bits;
        if (in->max_seg_steps) t.max_seg_steps = (int)in->max_seg_steps;
        if (in->reorder) t.reorder = (in->reorder == 1);
        if (in->small_bits) t.small_bits = (int)in->small_bits;
        if (in->kernel_variant) t.variant = in->kernel_variant - 1;
        if (in->wg_per_cu) t.wg_per_cu = in->wg_per_cu;
        if (in->outer_order) t.outer_order = in->outer_order - 1;
        if (in->remap) t.remap = (in->remap == 1);
        if (in->mid_low_bits) t.mid_low_bits = (int)in->mid_low_bits;
        if (in->min_overlap) t.min_overlap = (int)in->min_overlap;
        if (in->rows_per_thread) {
            if (in->rows_per_thread != 8 && in->rows_per_thread != 16 && in->rows_per_thread != 32)
                return fail(QSIM_ERR_INVALID, "rows_per_thread must be 8, 16 or 32");
            t.rows_eb = (uint32_t)__builtin_ctz(in->rows_per_thread);
        }
        if (in->plan_search) {
            if (in->plan_search > 3) return fail(QSIM_ERR_INVALID, "plan_search out of range");
            t.plan_search = (int)in->plan_search - 1;
        }
        if (in->xcd_swizzle) {
            if (in->xcd_swizzle > 2) return fail(QSIM_ERR_INVALID, "xcd_swizzle out of range");
            t.xcd_swizzle = in->xcd_swizzle == 2;
        }
        if (in->product_stage) {
            if (in->product_stage > 3) return fail(QSIM_ERR_INVALID, "product_stage out of range");
            t.product_cut = in->product_stage - 1;
        }
    }
    if (t.mid_low_bits < 1 || t.mid_low_bits > t.low_bits) t.mid_low_bits = t.low_bits;
    if (t.outer_order > 1) return fail(QSIM_ERR_INVALID, "outer_order out of range");
    if (t.variant > 2) return fail(QSIM_ERR_INVALID, "kernel_variant out of range");
    if (t.wg_per_cu > 8) return fail(QSIM_ERR_INVALID, "wg_per_cu out of range");
    const int max_tile = elem == 8 ? kMaxTileBits : kMaxTileBits - 1;
    if (t.tile_bits < 5 || t.tile_bits > max_tile)
        return fail(QSIM_ERR_INVALID, "tile_bits out of range");
    if ((uint32_t)t.tile_bits < t.rows_eb || (uint32_t)t.tile_bits - t.rows_eb > 10)
        return fail(QSIM_ERR_INVALID, "tile_bits and rows_per_thread need 1..1024 threads per tile");
    if (t.low_bits < 1 || t.low_bits > t.tile_bits) return fail(QSIM_ERR_INVALID, "low_bits out of range");
    if (t.max_seg_steps < 1 || t.max_seg_steps > 4096) return fail(QSIM_ERR_INVALID, "max_seg_steps out of range");
    if (t.small_bits < 4 || t.small_bits > max_tile) return fail(QSIM_ERR_INVALID, "small_bits out of range");
    *out = t;
    return QSIM_OK;
}

PlanConfig plan_config(const Tuning &t, uint32_t elem) {
    PlanConfig c;
    c.line_bits = elem == 8 ? 4 : 3;   // 128-byte lines
    c.tile_bits = t.tile_bits;
    c.low_bits = t.low_bits;
    c.mid_low_bits = t.remap ? t.mid_low_bits : t.low_bits;
    c.min_overlap = t.remap ? t.min_overlap : 0;
    c.max_seg_steps = t.max_seg_steps;
    c.reorder = t.reorder;
    c.search = t.plan_search;
    c.search_small = elem == 8 ? 0 : 1;   // by size, below M = 30: greedy (8 B), climb (16 B)
    c.remap = t.remap;
    return c;
}

uint64_t pdep(uint64_t x, const uint8_t *pos, uint32_t n) {
    uint64_t r = 0;
    for (uint32_t q = 0; q < n; ++q)
        if ((x >> q) & 1ull) r |= 1ull << pos[q];
    return r;
}

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n) {
        if (n <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            cap = 0;
            if (e != hipSuccess) return e;
        }
        size_t want = std::max<size_t>(n, 4096);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Grow-only pinned host staging buffer; `ev` marks when the last copy out
// of it has been consumed by the device.
struct HostStage {
    void *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    hipError_t wait() {
        if (pending) {
            pending = false;
            return hipEventSynchronize(ev);
        }
        return hipSuccess;
    }
    hipError_t ensure(size_t n) {
        hipError_t e = wait();
        if (e != hipSuccess) return e;
        if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
        if (n <= cap) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(n, 65536);
        e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        (void)wait();
        if (p) (void)hipHostFree(p);
        if (ev) (void)hipEventDestroy(ev);
        p = nullptr;
        ev = nullptr;
        cap = 0;
    }
};

}  // namespace

struct qsim_state {
    uint32_t M = 0;
    qsim_dtype dtype = QSIM_C64;
    uint32_t elem = 8;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    bool owned = false;
    bool poisoned = false;
    int device = 0;
    hipStream_t last_stream = nullptr;
    Tuning tune{};
    DevBuf plan;   // uploaded step descriptors
    DevBuf rec;    // per-tile records of a pass
    HostStage stage;
    // timing (qsim_state_profile)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    struct Timed { int kind; hipEvent_t a, b; uint64_t bytes; };
    std::vector<Timed> timed;
    qsim_profile prof{};
};

namespace {

int device_fail(qsim_state *s, hipError_t e, const char *what) {
    if (s) s->poisoned = true;
    return fail(QSIM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

// Host-side plan of one apply call: a blob to upload and the launches to
// make with pointers into the uploaded copy.
struct Launch {
    enum Kind { DIRECT, SMALL, TILEMAP, TILE } kind;
    size_t steps_off = 0;    // byte offset of the launch's step array in the blob
    size_t inner_off = 0;
    uint32_t n = 0;          // steps (DIRECT / TILEMAP)
    uint64_t n_tiles = 0;
    TileArgs ta{};
    TileMapArgs tm{};
    bool product = false;    // TILE: form the source tile from qubits (first pass only)
    size_t q_off = 0;        // byte offset of the qubits in the blob
    ProductTileArgs pa{};
};

struct Prepared {
    std::vector<uint8_t> blob;
    std::vector<Launch> launches;
    size_t rec_bytes = 0;
};

size_t blob_push(std::vector<uint8_t> &blob, const void *data, size_t bytes) {
    size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + bytes);
    if (bytes) std::memcpy(blob.data() + off, data, bytes);
    return off;
}

// Inner step arrays are read eight entries at a time by the tile kernels:
// pad with zero entries (never executed) to a multiple of eight.
size_t push_inner(std::vector<uint8_t> &blob, std::vector<uint32_t> inner) {
    inner.resize((inner.size() + 7) & ~size_t(7), 0u);
    if (inner.empty()) inner.resize(8, 0u);
    return blob_push(blob, inner.data(), inner.size() * 4);
}

// Small-state path: the whole state is one tile; every step is inner.
void prepare_small(uint32_t M, uint32_t elem, const qsim_step *steps, uint64_t L, Prepared &pr) {
    std::vector<uint32_t> inner(L);
    bool sign = false;
    for (uint64_t s = 0; s < L; ++s) {
        const qsim_step &st = steps[L - 1 - s];
        if (st.kind == QSIM_STEP_PHASE) {
            inner[s] = pack_inner(kSignPlane, (uint32_t)phase_mask(st));
            sign = true;
        } else {
            inner[s] = pack_inner(st.target, (uint32_t)st.control_mask);
        }
    }
    Launch l;
    l.kind = Launch::SMALL;
    l.ta.sign = sign ? 1u : 0u;
    l.inner_off = push_inner(pr.blob, inner);
    l.ta.n_inner = (uint32_t)L;
    l.ta.tb = M - 5;
    l.ta.eb = 5;
    l.ta.n_out = 0;
    const uint32_t LO = elem == 8 ? 1 : 0;
    for (uint32_t b = 0; b < 16; ++b) l.ta.pos_src[b] = l.ta.pos_dst[b] = (uint8_t)b;
    const uint32_t vpt = 32u >> LO;
    for (uint32_t r = 0; r < 32; ++r)
        l.ta.off_r_src[r] = l.ta.off_r_dst[r] = r < vpt ? (uint32_t)(r << (LO + l.ta.tb)) : 0u;
    pr.launches.push_back(l);
}

void prepare_direct(const qsim_step *steps, uint64_t L, Prepared &pr) {
    std::vector<TmStep> rev(L);
    for (uint64_t s = 0; s < L; ++s) {
        const qsim_step &st = steps[L - 1 - s];
        const bool ph = st.kind == QSIM_STEP_PHASE;
        rev[s].cm = ph ? phase_mask(st) : st.control_mask;
        rev[s].tbit = st.target;
        rev[s].inner = ph ? 1u : 0u;
    }
    Launch l;
    l.kind = Launch::DIRECT;
    l.steps_off = blob_push(pr.blob, rev.data(), rev.size() * sizeof(TmStep));
    l.n = (uint32_t)L;
    pr.launches.push_back(l);
}

// Layout of the state between pass p-1 (tile mask A) and pass p (tile mask
// B): physical bit i holds logical bit order[i].  The bits every pass keeps
// in its tile stay at the bottom in place; above them come the bits both
// neighbours tile, then the rest of B (read side of pass p), then the rest
// of A (write side of pass p-1), then everything else, so that both passes
// see their tiles as a few long contiguous runs in few pages.
void make_layout(uint32_t M, uint32_t fixed, uint64_t A, uint64_t B, uint8_t *lam, uint32_t line_bits) {
    std::vector<uint32_t> order;
    for (uint32_t b = 0; b < fixed; ++b) order.push_back(b);
    auto add = [&](uint64_t set) {
        for (uint32_t b = fixed; b < M; ++b)
            if ((set >> b) & 1ull) order.push_back(b);
    };
    const uint64_t all = (1ull << M) - 1ull;
    add(A & B);
    // When the two tiles share fewer bits than address one 128-byte line,
    // bits of A take the rest of the line's positions: pass p-1 then writes
    // whole lines and pass p reads part lines (measured cheaper than the
    // other way round: 14.1 + 14.9 ms against 18.3 + 12.0 ms for the two
    // passes around such a boundary at M = 32).
    uint64_t a_only = A & ~B;
    const uint32_t shared = (uint32_t)__builtin_popcountll(A & B);
    uint32_t need = line_bits > shared ? line_bits - shared : 0u;
    uint64_t lift = 0;
    for (uint32_t b = fixed; b < M && need; ++b)
        if ((a_only >> b) & 1ull) {
            lift |= 1ull << b;
            --need;
        }
    add(lift);
    add(B & ~A);
    add(a_only & ~lift);
    add(all & ~(A | B));
    for (uint32_t i = 0; i < M; ++i) lam[order[i]] = (uint8_t)i;
}

int prepare_passes(uint32_t M, uint32_t elem, const std::vector<Pass> &passes,
                   const uint32_t *target, const uint64_t *cmask, const uint8_t *kind, uint32_t outer_order,
                   bool remap, uint32_t eb, Prepared &pr, bool xcd_swizzle = true) {
    const uint32_t LO = elem == 8 ? 1 : 0;
    const size_t P = passes.size();
    // Layouts at the pass boundaries; the state enters and leaves in the
    // natural order.
    std::vector<std::array<uint8_t, 64>> lam(P + 1);
    for (auto &l : lam)
        for (uint32_t b = 0; b < 64; ++b) l[b] = (uint8_t)b;
    if (remap && P > 1) {
        uint64_t common = ~0ull;
        for (const Pass &p : passes) common &= p.tile_mask;
        uint32_t fixed = 0;
        while (fixed < M && ((common >> fixed) & 1ull)) ++fixed;
        for (size_t p = 1; p < P; ++p)
            make_layout(M, fixed, passes[p - 1].tile_mask, passes[p].tile_mask, lam[p].data(), elem == 8 ? 4u : 3u);
    }
    for (size_t pi = 0; pi < P; ++pi) {
        const Pass &p = passes[pi];
        const uint64_t I = p.tile_mask;
        const uint32_t K = (uint32_t)__builtin_popcountll(I);
        // The tile kernel needs 32 entries per thread, at most 2^14 entries,
        // tile offsets below 2^32 and, for 8-byte entries, address bit 0 in
        // the tile (entries travel in adjacent pairs).
        if (K < eb || K - eb > 10 || K > (uint32_t)kMaxTileBits || (M - K) > (uint32_t)kMaxOuterBits ||
            (elem == 8 && !(I & 1ull)) || (elem == 16 && K > (uint32_t)kMaxTileBits - 1))
            return fail(QSIM_ERR_INVALID, "planner produced a tile the kernel cannot run");
        const uint8_t *ls = lam[pi].data(), *ld = lam[pi + 1].data();
        uint8_t in_log[16] = {0}, out_log[kMaxOuterBits] = {0};
        uint8_t jpos[64];
        uint32_t ni = 0, no = 0;
        for (uint32_t b = 0; b < M; ++b) {
            if ((I >> b) & 1ull) in_log[ni++] = (uint8_t)b;
            else out_log[no++] = (uint8_t)b;
        }
        // Tile-index bit j of the kernel is tile bit in_log[j].  Kernel index
        // bits: the LO pair bit and 6 lane bits (one wave instruction moves
        // these 2^(LO+6) rows), then the wave bits, then the per-thread row
        // bits.  The lane bits hold the tile bits at the lowest physical
        // positions of both layouts (the bits inside one 128-byte line), so
        // every load and every store instruction covers whole lines: a line
        // split across instructions can leave L2 before its last part is
        // read, and is then fetched twice.  The rest of the lanes, and the
        // order within them, follow the written layout so a wave store
        // covers contiguous lines; bit 0 stays first (its physical position
        // is 0 in every layout, which the 8-byte pairs need).  The wave bits
        // take the highest written positions and the row bits the ones
        // between, so that each wave's stores cover one compact block
        // (measured faster than rows spread over the whole tile).
        std::sort(in_log, in_log + ni, [&](uint8_t x, uint8_t y) { return ld[x] < ld[y]; });
        {
            const uint32_t lanes = std::min<uint32_t>(LO + 6, K), tb = K - eb;
            const uint32_t line_bits = elem == 8 ? 4u : 3u;
            uint8_t by_pos[16];
            std::memcpy(by_pos, in_log, sizeof(by_pos));
            bool lane[16] = {false};
            uint32_t nl = 0;
            // written-side line bits first, then read-side ones, then the
            // lowest remaining written positions
            for (int pass = 0; pass < 3; ++pass)
                for (uint32_t q = 0; q < K && nl < lanes; ++q) {
                    const uint8_t b = by_pos[q];
                    if (lane[q]) continue;
                    const bool take = pass == 0 ? ld[b] < line_bits : (pass == 1 ? ls[b] < line_bits : true);
                    if (take) { lane[q] = true; ++nl; }
                }
            uint32_t k = 0;
            for (uint32_t q = 0; q < K; ++q)
                if (lane[q]) in_log[k++] = by_pos[q];
            uint8_t rest[16];
            uint32_t nr = 0;
            for (uint32_t q = 0; q < K; ++q)
                if (!lane[q]) rest[nr++] = by_pos[q];
            const uint32_t nw = tb > 6 ? tb - 6 : 0;
            for (uint32_t q = 0; q < nw; ++q) in_log[k++] = rest[nr - nw + q];
            for (uint32_t q = 0; q + nw < nr; ++q) in_log[k++] = rest[q];
        }
        for (uint32_t j = 0; j < ni; ++j) jpos[in_log[j]] = (uint8_t)j;
        // Tiles may be enumerated in any order: outer_order picks which
        // outside bits (by physical position in the written layout) vary
        // between tiles processed at the same time.
        std::sort(out_log, out_log + no, [&](uint8_t x, uint8_t y) {
            return outer_order == 1 ? ld[x] > ld[y] : ld[x] < ld[y];
        });
        TileArgs ta{};
        for (uint32_t b = 0; b < K; ++b) {
            ta.pos_src[b] = ls[in_log[b]];
            ta.pos_dst[b] = ld[in_log[b]];
            if (ta.pos_src[b] >= 32 || ta.pos_dst[b] >= 32)
                return fail(QSIM_ERR_INVALID, "layout put a tile bit above bit 31");
        }
        if (elem == 8 && (ta.pos_src[0] != 0 || ta.pos_dst[0] != 0))
            return fail(QSIM_ERR_INVALID, "layout moved address bit 0");
        for (uint32_t q = 0; q < no; ++q) ta.out_dst[q] = ld[out_log[q]];

        std::vector<TmStep> tm;
        std::vector<uint32_t> inner;
        bool sign = false;
        tm.reserve(p.steps.size());
        for (size_t q = p.steps.size(); q-- > 0;) {
            const uint32_t s = p.steps[q];
            const uint64_t T = 1ull << target[s];
            const bool ph = kind && kind[s] == kStepPhase;
            // A phase step is an inner step on the sign plane: its tile
            // bits select rows inside the tile, its outside bits the tiles.
            const uint64_t rmask = ph ? (cmask[s] | T) : cmask[s];
            TmStep d;
            d.cm = rmask & ~I;
            d.tbit = target[s];
            d.inner = (ph || (I & T)) ? 1u : 0u;
            tm.push_back(d);
            sign |= ph;
            if (d.inner) {
                uint32_t icm = 0;
                uint64_t ci = rmask & I;
                while (ci) {
                    const uint32_t b = (uint32_t)__builtin_ctzll(ci);
                    ci &= ci - 1;
                    icm |= 1u << jpos[b];
                }
                inner.push_back(pack_inner(ph ? kSignPlane : jpos[target[s]], icm));
            }
        }
        const uint32_t n_inner = (uint32_t)inner.size();
        const uint32_t rec_words = 2u + (n_inner + 31u) / 32u;
        const uint64_t n_tiles = 1ull << (M - K);
        if (n_tiles > 0x7FFFFFFFull)
            return fail(QSIM_ERR_INVALID, "more than 2^31 - 1 tiles in a pass: raise tile_bits");

        Launch lm;
        lm.kind = Launch::TILEMAP;
        lm.steps_off = blob_push(pr.blob, tm.data(), tm.size() * sizeof(TmStep));
        lm.n = (uint32_t)tm.size();
        lm.n_tiles = n_tiles;
        lm.tm.n_tiles = n_tiles;
        lm.tm.n_steps = (uint32_t)tm.size();
        lm.tm.rec_words = rec_words;
        lm.tm.n_out = no;
        std::memcpy(lm.tm.out_pos, out_log, sizeof(out_log));
        std::memcpy(lm.tm.lam_src, ls, 64);

        Launch lt;
        lt.kind = Launch::TILE;
        lt.inner_off = push_inner(pr.blob, inner);
        lt.n_tiles = n_tiles;
        lt.ta = ta;
        lt.ta.n_inner = n_inner;
        lt.ta.rec_words = rec_words;
        lt.ta.tb = K - eb;
        lt.ta.eb = eb;
        lt.ta.n_out = no;
        lt.ta.sign = sign ? 1u : 0u;
        // One-tile-per-workgroup launches: workgroups go to the 8 XCDs in
        // turn, so 2^6 consecutive tiles (about one XCD's resident
        // workgroups) are mapped to one XCD; tiles next to each other in
        // this order write interleaved parts of the same lines, which then
        // meet in one L2 (measured about 2% faster at M = 32).
        if (xcd_swizzle) lt.ta.xcd = std::min<uint32_t>(6u, M - K >= 3 ? M - K - 3 : 0u);
        const uint32_t vpt = (1u << eb) >> LO;
        for (uint32_t r = 0; r < 32; ++r) {
            const uint64_t j = (uint64_t)r << (LO + lt.ta.tb);
            lt.ta.off_r_src[r] = r < vpt ? (uint32_t)pdep(j, ta.pos_src, K) : 0u;
            lt.ta.off_r_dst[r] = r < vpt ? (uint32_t)pdep(j, ta.pos_dst, K) : 0u;
        }
        pr.launches.push_back(lm);
        pr.launches.push_back(lt);
        pr.rec_bytes = std::max<size_t>(pr.rec_bytes, (size_t)n_tiles * rec_words * 4);
    }
    return QSIM_OK;
}

int prepare(qsim_state *s, const qsim_step *steps, uint64_t L, Prepared &pr) {
    const uint32_t M = s->M;
    if (M <= 4) {
        prepare_direct(steps, L, pr);
        return QSIM_OK;
    }
    if ((int)M <= s->tune.small_bits) {
        prepare_small(M, s->elem, steps, L, pr);
        return QSIM_OK;
    }
    const StepLists sl = split_steps(steps, L);
    std::vector<Pass> passes;
    try {
        passes = plan_passes(M, sl.tg.data(), sl.cm.data(), sl.kd.data(), L, plan_config(s->tune, s->elem));
    } catch (const std::logic_error &e) {   // (host memory and threads: host_exception)
        return fail(QSIM_ERR_INVALID, std::string("planner: ") + e.what());
    }
    return prepare_passes(M, s->elem, passes, sl.tg.data(), sl.cm.data(), sl.kd.data(), s->tune.outer_order,
                          s->tune.remap, s->tune.rows_eb, pr, s->tune.xcd_swizzle);
}

// Timing helpers: a launch of `kind` (0 tile, 1 map, 2 other) is bracketed
// by two events from the state's pool when profiling is on.
hipError_t prof_event(qsim_state *s, hipEvent_t *ev) {
    if (!s->ev_pool.empty()) {
        *ev = s->ev_pool.back();
        s->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

hipError_t prof_begin(qsim_state *s, hipStream_t st, hipEvent_t *a) {
    if (!s->profiling) return hipSuccess;
    hipError_t e = prof_event(s, a);
    if (e == hipSuccess) e = hipEventRecord(*a, st);
    return e;
}

hipError_t prof_end(qsim_state *s, hipStream_t st, int kind, hipEvent_t a, uint64_t bytes) {
    if (!s->profiling) return hipSuccess;
    hipEvent_t b;
    hipError_t e = prof_event(s, &b);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) s->timed.push_back({kind, a, b, bytes});
    return e;
}

// Fold finished timings into the totals (waits for them).
hipError_t prof_collect(qsim_state *s) {
    for (auto &t : s->timed) {
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, t.a, t.b)) != hipSuccess) return e;
        if (t.kind == 0) { s->prof.tile_launches++; s->prof.tile_ms += ms; s->prof.tile_bytes += t.bytes; }
        else if (t.kind == 1) { s->prof.map_launches++; s->prof.map_ms += ms; }
        else { s->prof.other_launches++; s->prof.other_ms += ms; }
        s->ev_pool.push_back(t.a);
        s->ev_pool.push_back(t.b);
    }
    s->timed.clear();
    return hipSuccess;
}

// Enqueue the launches of `pr` on `st`, with the plan blob already on the
// device at `dev` (or enqueued ahead of them on `st`) and `rec` holding
// room for the tile records of one pass.  With `timed` the launches are
// bracketed by profiling events when the state's profiling is on.
int enqueue_launches(qsim_state *s, Prepared &pr, hipStream_t st, uint8_t *dev, uint32_t *rec, bool timed) {
    // An exception from here on (a timing record that cannot be stored)
    // leaves some of the launches enqueued: the state is poisoned.
    struct PoisonOnThrow {
        qsim_state *s;
        int before = std::uncaught_exceptions();
        ~PoisonOnThrow() {
            if (std::uncaught_exceptions() > before) s->poisoned = true;
        }
    } poison_on_throw{s};
    hipError_t e;
    const bool prof = timed && s->profiling;
    const uint64_t n = 1ull << s->M;
    s->last_stream = st;   // set first: a failure part-way still leaves launched work to wait for
    const uint64_t pass_bytes = 2ull * n * s->elem;
    for (Launch &l : pr.launches) {
        const void *src = s->buf[s->cur];
        void *dst = s->buf[s->cur ^ 1];
        hipEvent_t ev_a = nullptr;
        if (prof && (e = prof_begin(s, st, &ev_a)) != hipSuccess) return device_fail(s, e, "profiling event");
        // The product-input pass counts as "other": it writes the state and
        // reads nothing, unlike the tile passes whose bytes are summed.
        const int kind = l.kind == Launch::TILE && !l.product ? 0 : (l.kind == Launch::TILEMAP ? 1 : 2);
        switch (l.kind) {
            case Launch::DIRECT:
                e = launch_direct(s->elem, src, dst, n, reinterpret_cast<const TmStep *>(dev + l.steps_off), l.n, st);
                s->cur ^= 1;
                break;
            case Launch::SMALL:
                l.ta.inner = reinterpret_cast<const uint32_t *>(dev + l.inner_off);
                l.ta.rec = nullptr;
                e = launch_small(s->elem, src, dst, s->M, l.ta, st);
                s->cur ^= 1;
                break;
            case Launch::TILEMAP:
                l.tm.steps = reinterpret_cast<const TmStep *>(dev + l.steps_off);
                l.tm.rec = rec;
                e = launch_tilemap(l.tm, st);
                break;
            case Launch::TILE:
                l.ta.inner = reinterpret_cast<const uint32_t *>(dev + l.inner_off);
                l.ta.rec = rec;
                if (l.product) {
                    l.pa.q = dev + l.q_off;
                    e = launch_tile_product(s->elem, dst, l.n_tiles, l.ta, l.pa, st);
                } else {
                    e = launch_tile(s->elem, src, dst, l.n_tiles, l.ta, s->tune.variant, s->tune.wg_per_cu, st);
                }
                s->cur ^= 1;
                break;
        }
        if (e == hipSuccess) e = injected("launch");
        if (e != hipSuccess) return device_fail(s, e, "kernel launch");
        injected_throw("host-launch");
        if (prof && (e = prof_end(s, st, kind, ev_a, kind == 1 ? 0 : pass_bytes)) != hipSuccess)
            return device_fail(s, e, "profiling event");
    }
    s->last_stream = st;
    return QSIM_OK;
}

// Upload the plan through the state's pinned staging buffer into its own
// plan buffer, then enqueue the launches (the state's buffers grow as
// needed).
int enqueue(qsim_state *s, Prepared &pr, hipStream_t st) {
    hipError_t e;
    if ((e = s->stage.ensure(pr.blob.size())) != hipSuccess) return device_fail(s, e, "host staging");
    if ((e = s->plan.ensure(pr.blob.size())) != hipSuccess) return device_fail(s, e, "plan buffer");
    if (pr.rec_bytes && (e = s->rec.ensure(pr.rec_bytes)) != hipSuccess) return device_fail(s, e, "tile records");
    std::memcpy(s->stage.p, pr.blob.data(), pr.blob.size());
    s->last_stream = st;
    e = hipMemcpyAsync(s->plan.p, s->stage.p, pr.blob.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = injected("upload");
    if (e != hipSuccess) return device_fail(s, e, "plan upload");
    if ((e = hipEventRecord(s->stage.ev, st)) != hipSuccess) return device_fail(s, e, "event record");
    s->stage.pending = true;
    return enqueue_launches(s, pr, st, static_cast<uint8_t *>(s->plan.p), static_cast<uint32_t *>(s->rec.p), true);
}

int check_state(const qsim_state *s) {
    if (!s) return fail(QSIM_ERR_INVALID, "state is NULL");
    if (s->poisoned) return fail(QSIM_ERR_DEVICE, "state is poisoned by an earlier device error");
    return QSIM_OK;
}

}  // namespace

int qsim::host_exception(qsim_state *s) noexcept {
    int code = QSIM_ERR_INVALID;
    char what[160] = "unknown exception";
    try {
        throw;
    } catch (const std::bad_alloc &) {
        code = QSIM_ERR_NOMEM;
        std::snprintf(what, sizeof what, "host memory allocation failed");
    } catch (const std::system_error &e) {   // a thread or a lock that could not be had
        code = QSIM_ERR_NOMEM;
        std::snprintf(what, sizeof what, "host resource: %s", e.what());
    } catch (const std::exception &e) {
        std::snprintf(what, sizeof what, "host: %s", e.what());
    } catch (...) {
    }
    if (s && s->poisoned) code = QSIM_ERR_DEVICE;   // poisoned during this call (checked on entry)
    try {
        g_err = what;
    } catch (...) {
    }
    return code;
}

// ------------------------------------------------------------ allocation-free apply

// Device scratch of qsim_apply_steps_noalloc: the plan blob at the start,
// the tile records of the current pass after it.  Each device that runs the
// library holds its own copy until the process ends.  Host code never uses
// the array's name as an address: the address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) uint8_t scratch[QSIM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

// Address of `scratch` on device `dev` (the current device).
hipError_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

namespace {

// ------------------------------------------------------------ batched mode

// Launch parameters of batched mode for one dtype (qsim_batch_tuning).
struct BatchTune {
    uint32_t tiles_per_item = 32;
    uint32_t tile_bits = 0;        // 0: 13 for 8-byte entries, 12 for 16-byte ones
    // measured per 4096-circuit batch (kernel): whole circuits up to 64
    // tiles per pass 15.29 ms (32: 15.46, 16: 15.57, 8: 15.67); with the
    // mask climb 14.94 ms (81.2 instead of 83.4 GB; host enqueue 11.5
    // instead of 7.5 ms on 16 threads, still under the kernel)
    uint32_t circuit_tiles = 64;
    uint32_t plan_search = 2;      // 1 greedy scan, 2 with the mask climb
    uint32_t order = 2;            // 1 level by level, 2 critical path first
};

uint32_t batch_tile_bits(const BatchTune &t, uint32_t elem) { return t.tile_bits ? t.tile_bits : (elem == 8 ? 13u : 12u); }

void export_batch_tune(const BatchTune &t, uint32_t elem, qsim_batch_tuning *out) {
    std::memset(out, 0, sizeof(*out));
    out->tiles_per_item = t.tiles_per_item;
    out->tile_bits = batch_tile_bits(t, elem);
    out->circuit_tiles = t.circuit_tiles;
    out->plan_search = t.plan_search;
    out->order = t.order;
}

int batch_tune_from(const qsim_batch_tuning *in, BatchTune *out) {
    BatchTune t;
    if (in) {
        if (in->tiles_per_item) t.tiles_per_item = in->tiles_per_item;
        if (in->tile_bits) t.tile_bits = in->tile_bits;
        if (in->circuit_tiles) t.circuit_tiles = in->circuit_tiles;
        if (in->plan_search) t.plan_search = in->plan_search;
        if (in->order) t.order = in->order;
    }
    if (t.tiles_per_item > kBatchTilesMax) return fail(QSIM_ERR_INVALID, "tiles_per_item above 256");
    if (t.tile_bits && (t.tile_bits < 10 || t.tile_bits > 13)) return fail(QSIM_ERR_INVALID, "batch tile_bits out of 10..13");
    if (t.circuit_tiles > kBatchTilesMax) return fail(QSIM_ERR_INVALID, "circuit_tiles above 256");
    if (t.plan_search < 1 || t.plan_search > 2) return fail(QSIM_ERR_INVALID, "batch plan_search must be 1 or 2");
    if (t.order < 1 || t.order > 2) return fail(QSIM_ERR_INVALID, "batch order must be 1 or 2");
    *out = t;
    return QSIM_OK;
}

// Process-wide workspace of the batched launch, in two slots used in turn:
// while one batch's kernel runs, the next batch's plan is uploaded into the
// other slot on a side stream, ordered by events (the upload waits until
// the slot's previous kernel is done; the kernel waits for its upload).
struct BatchSlot {
    DevBuf ws;          // counters, items, pass and circuit descriptors, step arrays
    HostStage stage;    // pinned staging of the upload
    uint32_t *hdr = nullptr;          // pinned copy of the counter header, written after the kernel
    hipEvent_t uploaded = nullptr;    // upload finished
    hipEvent_t done = nullptr;        // kernel and header copy finished
    hipEvent_t k0 = nullptr, k1 = nullptr;   // around the kernel (timing)
    bool pending = false;
    bool timed = false;
    qsim_batch_info info{};
};

struct BatchWorkspace {
    std::mutex mu;
    BatchTune tune[2];                // per dtype (qsim_batch_set_tuning / qsim_batch_autotune)
    BatchSlot slot[2];
    int next = 0;                     // slot of the next batch
    int last = -1;                    // slot of the last batch launched
    hipStream_t upload = nullptr;     // side stream for plan uploads (default priority)
    int device = -1;                  // device the streams and buffers belong to
    int status = QSIM_OK;             // first failure since the last status query
};

BatchWorkspace &batch_ws() {
    static BatchWorkspace w;
    return w;
}

// Wait for a slot's launch, fold its error flag into the sticky status and
// read its kernel time.
void batch_collect(BatchWorkspace &w, BatchSlot &b) {
    if (!b.pending) return;
    b.pending = false;
    hipError_t e = hipEventSynchronize(b.done);
    int rc = QSIM_OK;
    if (e != hipSuccess) rc = fail(QSIM_ERR_DEVICE, std::string("batch: ") + hipGetErrorString(e));
    else if (b.hdr[2]) rc = fail(QSIM_ERR_DEVICE, "batch: a dependency wait timed out; results are invalid");
    if (rc == QSIM_OK && b.timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b.k0, b.k1) == hipSuccess) b.info.kernel_ms = ms;
    }
    if (rc != QSIM_OK && w.status == QSIM_OK) w.status = rc;
}

// Wait for every batch in flight; report (and clear) the first failure.
int batch_status() {
    BatchWorkspace &w = batch_ws();
    std::lock_guard<std::mutex> lk(w.mu);
    batch_collect(w, w.slot[w.next ^ 1]);
    batch_collect(w, w.slot[w.next]);
    const int rc = w.status;
    w.status = QSIM_OK;
    return rc;
}

// Per-circuit host preparation (run in parallel over circuits).
struct BatchCircuitPlan {
    Prepared pr;                 // blob of this circuit + its launches
    bool small = false, direct = false;
    int rc = QSIM_OK;
    std::string err;
};

// Queue order of batched mode by list scheduling: the resident workgroups
// are simulated taking items in turn, each item ready once the previous
// pass of its circuit has finished (plus a little slack, so that the real
// workgroup rarely arrives before its predecessor's last tile is done),
// and among the ready items the one with the longest remaining chain (its
// own time plus that of the later passes of its circuit) goes first.
// Times are estimates in units of one tile (a tile item: its tiles; a
// whole circuit: all of its tiles; a small circuit: its share of a tile)
// plus a fixed cost per item.  The GPU takes items in the resulting order;
// an item whose predecessor has not finished after all only waits longer,
// so an estimate error costs time, never correctness (every item's
// predecessors come earlier in the order).
struct SimItem {
    uint64_t word;          // queue entry
    float dur;              // estimated duration
    float prio;             // remaining chain, itself included
    uint32_t next_pass;     // first item of the next pass of its circuit (~0u: none)
    uint32_t pass_id;       // pass of the item (~0u: independent item)
};

std::vector<uint64_t> order_critical_path(const std::vector<SimItem> &items, const std::vector<uint32_t> &pass_items,
                                          const std::vector<uint32_t> &pass_first, uint64_t workers, float slack) {
    // pass_items[p] = items of pass p, pass_first[p] = index of its first item
    // (the items of a pass are consecutive and share their priority)
    std::vector<uint32_t> left(pass_items);
    // Heap keys: non-negative floats order like their bit patterns.  The
    // ready heap holds runs of consecutive items of equal priority (a pass,
    // or one independent item) as (prio bits, ~first index): highest
    // priority first, then the lowest index, the order of taking the items
    // one by one.  A run stays on top while it hands out its items.  The
    // event heap holds (time bits, id), earliest first.
    auto fbits = [](float f) { uint32_t u; std::memcpy(&u, &f, 4); return (uint64_t)u; };
    auto ready_key = [&](uint32_t i) { return fbits(items[i].prio) << 32 | (uint64_t)(~i); };
    std::vector<uint64_t> ready;
    std::vector<uint32_t> run_end(items.size(), 0);   // for the first item of a run: one past its last
    ready.reserve(items.size());
    std::vector<uint8_t> has_pred(items.size(), 0);
    for (const SimItem &it : items)
        if (it.next_pass != ~0u) has_pred[it.next_pass] = 1;
    for (uint32_t i = 0; i < items.size();) {
        const uint32_t p = items[i].pass_id;
        const uint32_t n = p == ~0u ? 1u : pass_items[p];
        for (uint32_t j = i; j < i + n; ++j) run_end[j] = i + n;
        // ready at the start: independent items and the first pass of each chain
        if (p == ~0u || !has_pred[pass_first[p]]) ready.push_back(ready_key(i));
        i += n;
    }
    std::make_heap(ready.begin(), ready.end());
    std::vector<uint64_t> events;
    events.reserve(2 * std::max<uint64_t>(workers, 1) + pass_items.size());
    auto later = std::greater<uint64_t>();
    std::vector<uint64_t> order;
    order.reserve(items.size());
    float now = 0;
    uint64_t free_w = std::max<uint64_t>(workers, 1);
    while (order.size() < items.size()) {
        while (free_w > 0 && !ready.empty()) {
            const uint32_t i = ~(uint32_t)ready.front();
            if (i + 1 < run_end[i]) {
                ready.front() = ready_key(i + 1);   // still the largest key
            } else {
                std::pop_heap(ready.begin(), ready.end());
                ready.pop_back();
            }
            order.push_back(items[i].word);
            events.push_back(fbits(now + items[i].dur) << 32 | i);
            std::push_heap(events.begin(), events.end(), later);
            --free_w;
        }
        if (events.empty()) break;   // cannot happen: every pass follows one that finishes
        std::pop_heap(events.begin(), events.end(), later);
        const uint64_t ev = events.back();
        events.pop_back();
        const uint32_t id = (uint32_t)ev;
        const uint32_t tbits = (uint32_t)(ev >> 32);
        std::memcpy(&now, &tbits, 4);
        if (id & 0x80000000u) {   // the next pass of a chain becomes ready
            ready.push_back(ready_key(id & 0x7FFFFFFFu));
            std::push_heap(ready.begin(), ready.end());
            continue;
        }
        ++free_w;
        const SimItem &it = items[id];
        if (it.pass_id != ~0u && --left[it.pass_id] == 0 && it.next_pass != ~0u) {
            events.push_back(fbits(now + slack) << 32 | (it.next_pass | 0x80000000u));
            std::push_heap(events.begin(), events.end(), later);
        }
    }
    return order;
}

// fn(i) for i < n on up to 16 host threads, indices handed out one at a
// time (n / grain threads at most).
template <typename F>
void host_parallel(uint32_t n, uint32_t grain, F &&fn) {
    const uint32_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const uint32_t nt = std::min<uint32_t>(hw, (n + grain - 1) / grain);
    parallel_for(n, (int)nt, [&](size_t i) { fn((uint32_t)i); });
}

// Host-side buffers of batch_enqueue, kept per calling thread from one
// batch to the next: a batch of thousands of circuits fills megabytes of
// plans and descriptors, and fresh allocations of that size would be
// page-faulted in again on every call.
struct BatchHostScratch {
    std::vector<BatchCircuitPlan> plans;
    std::vector<BatchPass> bpass;
    std::vector<BatchSmall> bsmall;
    std::vector<size_t> small_blob_off, pass_blob_off, circuit_blob_off;
    std::vector<uint32_t> small_circuit;
    std::vector<std::pair<uint32_t, uint32_t>> circuit_first_pass;
    std::vector<SimItem> sim;
    std::vector<uint32_t> pass_items, pass_first;
    std::vector<uint32_t> circ_pass0, circ_small;   // per circuit: its first pass / its small entry
};

int batch_enqueue(qsim_state *const *states, const qsim_step *const *steps, const uint64_t *Ls, uint32_t n,
                  hipStream_t st) {
    const uint32_t elem = states[0]->elem;
    BatchWorkspace &w = batch_ws();
    BatchTune tune;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        tune = w.tune[elem == 8 ? 0 : 1];
    }
    const uint32_t Kb = batch_tile_bits(tune, elem);
    const uint32_t tb = Kb - 5;
    if ((size_t)elem << Kb > 128 * 1024) return fail(QSIM_ERR_INVALID, "batch tiles above 128 KiB of LDS");

    // Phase timings on stderr when QSIM_TRACE_BATCH is set.
    const bool trace = std::getenv("QSIM_TRACE_BATCH") != nullptr;
    auto t_prev = std::chrono::steady_clock::now();
    auto lap = [&](const char *what) {
        if (!trace) return;
        const auto t = std::chrono::steady_clock::now();
        std::fprintf(stderr, "qsim batch: %-10s %8.3f ms\n", what,
                     std::chrono::duration<double, std::milli>(t - t_prev).count());
        t_prev = t;
    };

    // 1. validate and plan every circuit (host threads); nothing is
    // enqueued unless every circuit passes
    static thread_local BatchHostScratch hs;
    std::vector<BatchCircuitPlan> &plans = hs.plans;
    if (plans.size() < n) plans.resize(n);
    auto plan_one = [&](uint32_t c) {
        qsim_state *s = states[c];
        const uint64_t L = Ls[c];
        BatchCircuitPlan &bp = plans[c];
        bp.pr.blob.clear();
        bp.pr.launches.clear();
        bp.pr.rec_bytes = 0;
        bp.small = bp.direct = false;
        bp.rc = QSIM_OK;
        bp.err.clear();
        if ((bp.rc = validate_steps(s->M, steps[c], L))) {
            bp.err = g_err;
            return;
        }
        if (L == 0) return;
        if (s->M <= 4) {
            bp.direct = true;
            prepare_direct(steps[c], L, bp.pr);
        } else if (s->M <= Kb) {
            bp.small = true;
            prepare_small(s->M, elem, steps[c], L, bp.pr);
        } else {
            const StepLists sl = split_steps(steps[c], L);
            PlanConfig pc = plan_config(s->tune, elem);
            pc.tile_bits = (int)Kb;
            pc.low_bits = std::min(pc.low_bits, (int)Kb);
            pc.mid_low_bits = std::min(pc.mid_low_bits, pc.low_bits);
            pc.threads = 1;   // circuits are already planned on several threads
            pc.search = (tune.plan_search == 2 || s->M >= 30) ? 1 : 0;   // never the beam search here
            try {
                std::vector<Pass> passes = plan_passes(s->M, sl.tg.data(), sl.cm.data(), sl.kd.data(), L, pc);
                bp.rc = prepare_passes(s->M, elem, passes, sl.tg.data(), sl.cm.data(), sl.kd.data(),
                                       s->tune.outer_order, s->tune.remap, 5u, bp.pr);
                if (bp.rc) bp.err = g_err;
            } catch (const std::logic_error &e) {
                bp.rc = QSIM_ERR_INVALID;
                bp.err = std::string("planner: ") + e.what();
            }
        }
    };
    host_parallel(n, 64, plan_one);
    for (uint32_t c = 0; c < n; ++c)
        if (plans[c].rc) return fail(plans[c].rc, "circuit " + std::to_string(c) + ": " + plans[c].err);
    lap("plan");

    // 2. descriptors: passes of the tiled circuits, the small circuits,
    // and where each circuit's blob goes
    std::vector<BatchPass> &bpass = hs.bpass;
    std::vector<BatchSmall> &bsmall = hs.bsmall;
    std::vector<size_t> &small_blob_off = hs.small_blob_off;   // per entry: offset of its circuit blob
    std::vector<size_t> &pass_blob_off = hs.pass_blob_off;
    std::vector<uint32_t> &small_circuit = hs.small_circuit;
    std::vector<std::pair<uint32_t, uint32_t>> &circuit_first_pass = hs.circuit_first_pass;   // (circuit, its first pass)
    std::vector<size_t> &circuit_blob_off = hs.circuit_blob_off;
    circuit_blob_off.assign(n, 0);
    size_t blob_size = 0;
    uint32_t rec_stride = 2;
    uint64_t max_tiles = 0;
    bool any_sign = false;   // some tile or small item has phase steps
    uint64_t alg_bytes = 0;
    uint32_t n_passes = 0;
    // Where each circuit's entries go, and the checks (a few fields of each
    // launch); then the descriptors themselves, circuits in parallel.
    std::vector<uint32_t> &circ_pass0 = hs.circ_pass0, &circ_small = hs.circ_small;
    circ_pass0.assign(n, ~0u);
    circ_small.assign(n, ~0u);
    circuit_first_pass.clear();
    uint32_t n_bpass = 0, n_bsmall = 0;
    for (uint32_t c = 0; c < n; ++c) {
        const BatchCircuitPlan &bp = plans[c];
        circuit_blob_off[c] = blob_size;
        blob_size += (bp.pr.blob.size() + 255) & ~size_t(255);
        if (bp.pr.launches.empty()) continue;
        const uint64_t state_bytes = (uint64_t)elem << states[c]->M;
        if (bp.direct || bp.small) {
            circ_small[c] = n_bsmall++;
            any_sign |= bp.pr.launches[0].ta.sign != 0;
            alg_bytes += 2 * state_bytes;
            ++n_passes;
            continue;
        }
        const uint64_t n_tiles = 1ull << (states[c]->M - Kb);
        uint32_t level = 0;
        for (size_t i = 0; i + 1 < bp.pr.launches.size(); i += 2, ++level) {
            const Launch &lt = bp.pr.launches[i + 1];
            // every pass of a circuit has 2^(M - tile bits) tiles of one shape
            if (lt.n_tiles != n_tiles || lt.ta.tb != tb || lt.ta.eb != 5)
                return fail(QSIM_ERR_INVALID, "circuit " + std::to_string(c) + ": a pass has another tile shape");
            any_sign |= lt.ta.sign != 0;
            rec_stride = std::max(rec_stride, lt.ta.rec_words);
        }
        // the per-circuit counter counts every finished tile of the circuit
        if ((uint64_t)level * n_tiles > 0xFFFFFFFFull)
            return fail(QSIM_ERR_INVALID, "circuit " + std::to_string(c) + ": passes x tiles beyond 2^32 - 1");
        circ_pass0[c] = n_bpass;
        circuit_first_pass.push_back({c, n_bpass});
        n_bpass += level;
        alg_bytes += 2 * state_bytes * level;
        n_passes += level;
        max_tiles = std::max(max_tiles, n_tiles);
    }
    // (every entry is overwritten below: no clearing of the kept capacity)
    bpass.resize(n_bpass);
    pass_blob_off.resize(n_bpass);
    bsmall.resize(n_bsmall);
    small_blob_off.resize(n_bsmall);
    small_circuit.resize(n_bsmall);
    host_parallel(n, 256, [&](uint32_t c) {
        const BatchCircuitPlan &bp = plans[c];
        const qsim_state *s = states[c];
        if (circ_small[c] != ~0u) {
            const uint32_t k = circ_small[c];
            const Launch &l = bp.pr.launches[0];
            BatchSmall sm{};
            sm.ta = l.ta;
            sm.src = s->buf[s->cur];
            sm.dst = s->buf[s->cur ^ 1];
            sm.L = l.n;
            sm.M = s->M;
            sm.direct = bp.direct ? 1u : 0u;
            bsmall[k] = sm;
            small_blob_off[k] = circuit_blob_off[c] + (bp.direct ? l.steps_off : l.inner_off);
            small_circuit[k] = c;
            return;
        }
        if (circ_pass0[c] == ~0u) return;
        uint32_t g = circ_pass0[c], level = 0;
        for (size_t i = 0; i + 1 < bp.pr.launches.size(); i += 2, ++level, ++g) {
            const Launch &lm = bp.pr.launches[i], &lt = bp.pr.launches[i + 1];
            BatchPass &p = bpass[g];
            p = BatchPass{};
            p.ta = lt.ta;
            p.tm = lm.tm;
            p.src = s->buf[s->cur ^ (level & 1u)];
            p.dst = s->buf[s->cur ^ ((level + 1) & 1u)];
            p.n_tiles = lt.n_tiles;
            p.circuit = c;
            p.level = level;
            // remember both step-array offsets inside the circuit blob
            p.ta.inner = reinterpret_cast<const uint32_t *>(lt.inner_off);
            p.ta.rec = nullptr;
            p.tm.steps = reinterpret_cast<const TmStep *>(lm.steps_off);
            p.tm.rec = nullptr;
            pass_blob_off[g] = circuit_blob_off[c];
        }
    });

    lap("describe");

    // 3. the items: one per small circuit, one per mid-size circuit (every
    // pass in one workgroup: no waits between its passes), and blocks of
    // tiles_per_item tiles of each pass of the others
    const uint32_t tpi = std::max<uint32_t>(1, tune.tiles_per_item);
    std::vector<uint8_t> whole_circ(circuit_first_pass.size(), 0);
    for (size_t k = 0; k < circuit_first_pass.size(); ++k)
        whole_circ[k] = bpass[circuit_first_pass[k].second].n_tiles <= tune.circuit_tiles;
    uint64_t rec_tiles = 0;   // tiles whose records one item holds in LDS at once
    for (size_t k = 0; k < circuit_first_pass.size(); ++k) {
        const uint64_t nt = bpass[circuit_first_pass[k].second].n_tiles;
        rec_tiles = std::max<uint64_t>(rec_tiles, whole_circ[k] ? nt : std::min<uint64_t>(nt, tpi));
    }
    const size_t lds = ((size_t)elem << Kb) + (size_t)rec_tiles * rec_stride * 4;
    if (lds > 160 * 1024) return fail(QSIM_ERR_INVALID, "batch: tile and records need more LDS than a workgroup has");
    uint64_t workers = 0;
    hipError_t e = batch_grid(elem, tb, any_sign, lds, &workers);
    if (e != hipSuccess) return fail(QSIM_ERR_DEVICE, std::string("batch occupancy: ") + hipGetErrorString(e));

    lap("occupancy");

    std::vector<uint64_t> items;
    const size_t n_small = bsmall.size();
    if (tune.order == 2) {
        std::vector<SimItem> &sim = hs.sim;
        std::vector<uint32_t> &pass_items = hs.pass_items, &pass_first = hs.pass_first;
        sim.clear();
        pass_items.clear();
        pass_first.clear();
        const float kItemCost = 0.25f;   // per-item cost in tiles (wait, drain, first load)
        const float kSlack = 2.0f;       // a pass's successors become ready this many tiles after it ends
        for (size_t k = 0; k < n_small; ++k) {
            const float d = std::ldexp(1.0f, (int)bsmall[k].M - (int)Kb) + kItemCost;
            sim.push_back({batch_item(kItemSmall, (uint32_t)k, 0), d, d, ~0u, ~0u});
        }
        for (size_t k = 0; k < circuit_first_pass.size(); ++k) {
            const uint32_t g0 = circuit_first_pass[k].second;
            const uint32_t g1 = k + 1 < circuit_first_pass.size() ? circuit_first_pass[k + 1].second
                                                                    : (uint32_t)bpass.size();
            const uint64_t nt = bpass[g0].n_tiles;
            if (whole_circ[k]) {
                const float d = (float)(g1 - g0) * ((float)nt + kItemCost);
                sim.push_back({batch_item(kItemCircuit, g0, g1 - g0), d, d, ~0u, ~0u});
                continue;
            }
            const float pass_d = (float)std::min<uint64_t>(nt, tpi) + kItemCost + kSlack;
            uint32_t prev_first = ~0u;
            for (uint32_t g = g0; g < g1; ++g) {
                const uint32_t first = (uint32_t)sim.size(), pid = (uint32_t)pass_items.size();
                const float remaining = (float)(g1 - g) * pass_d;
                for (uint64_t t = 0; t * tpi < nt; ++t) {
                    const float d = (float)std::min<uint64_t>(tpi, nt - t * tpi) + kItemCost;
                    sim.push_back({batch_item(kItemTile, g, (uint32_t)t), d, remaining, ~0u, pid});
                }
                pass_items.push_back((uint32_t)sim.size() - first);
                pass_first.push_back(first);
                if (prev_first != ~0u)
                    for (uint32_t j = prev_first; j < first; ++j) sim[j].next_pass = first;
                prev_first = first;
            }
        }
        lap("items");
        items = order_critical_path(sim, pass_items, pass_first, workers, kSlack);
        if (items.size() != sim.size()) return fail(QSIM_ERR_INVALID, "batch: queue ordering failed");
    } else {
        // level by level, with the small circuits spread between the levels
        // and the mid-size ones over the first half of them
        uint32_t max_level = 0;
        for (const BatchPass &p : bpass) max_level = std::max(max_level, p.level + 1);
        std::vector<uint64_t> whole;
        std::vector<uint8_t> in_whole(bpass.size(), 0);
        for (size_t k = 0; k < circuit_first_pass.size(); ++k) {
            if (!whole_circ[k]) continue;
            const uint32_t g0 = circuit_first_pass[k].second;
            const uint32_t g1 = k + 1 < circuit_first_pass.size() ? circuit_first_pass[k + 1].second
                                                                    : (uint32_t)bpass.size();
            whole.push_back(batch_item(kItemCircuit, g0, g1 - g0));
            for (uint32_t g = g0; g < g1; ++g) in_whole[g] = 1;
        }
        std::vector<std::vector<uint32_t>> by_level(max_level);
        for (size_t g = 0; g < bpass.size(); ++g)
            if (!in_whole[g]) by_level[bpass[g].level].push_back((uint32_t)g);
        size_t small_next = 0, whole_next = 0;
        const size_t levels = std::max<size_t>(max_level, 1), whole_levels = (levels + 1) / 2;
        for (size_t lv = 0; lv < levels; ++lv) {
            if (lv < by_level.size())
                for (uint32_t g : by_level[lv])
                    for (uint64_t t = 0; t * tpi < bpass[g].n_tiles; ++t)
                        items.push_back(batch_item(kItemTile, g, (uint32_t)t));
            const size_t wupto = whole.size() * std::min(lv + 1, whole_levels) / whole_levels;
            for (; whole_next < wupto; ++whole_next) items.push_back(whole[whole_next]);
            const size_t upto = n_small * (lv + 1) / levels;
            for (; small_next < upto; ++small_next) items.push_back(batch_item(kItemSmall, (uint32_t)small_next, 0));
        }
        for (; whole_next < whole.size(); ++whole_next) items.push_back(whole[whole_next]);
        for (; small_next < n_small; ++small_next) items.push_back(batch_item(kItemSmall, (uint32_t)small_next, 0));
    }
    if (items.size() > 0xFFFFFFF0ull) return fail(QSIM_ERR_INVALID, "batch too large");
    lap("queue");

    const size_t ctr_bytes = ((kBatchCtrHeader + n) * 4 + 255) & ~size_t(255);
    const size_t items_off = ctr_bytes;
    const size_t pass_off = (items_off + items.size() * 8 + 255) & ~size_t(255);
    const size_t small_off = (pass_off + bpass.size() * sizeof(BatchPass) + 255) & ~size_t(255);
    const size_t blob_off = (small_off + bsmall.size() * sizeof(BatchSmall) + 255) & ~size_t(255);
    const size_t total = blob_off + blob_size;

    std::lock_guard<std::mutex> lk(w.mu);
    if (w.device != states[0]->device) {
        // the workspace moves to this device: finish and free what it held
        for (BatchSlot &b : w.slot) {
            batch_collect(w, b);
            b.ws.release();
            b.stage.release();
            if (b.hdr) (void)hipHostFree(b.hdr);
            for (hipEvent_t ev : {b.uploaded, b.done, b.k0, b.k1})
                if (ev) (void)hipEventDestroy(ev);
            b = BatchSlot{};
        }
        if (w.upload) (void)hipStreamDestroy(w.upload);
        w.upload = nullptr;
        w.last = -1;
        w.device = states[0]->device;
    }
    if (!w.upload && (e = hipStreamCreateWithFlags(&w.upload, hipStreamNonBlocking)) != hipSuccess)
        return fail(QSIM_ERR_DEVICE, "batch upload stream");
    BatchSlot &b = w.slot[w.next];
    // The slot's previous batch (two launches ago) must be done with its
    // buffers: its status is read, its device buffers are then reused.
    batch_collect(w, b);
    if (!b.hdr && (e = hipHostMalloc((void **)&b.hdr, kBatchCtrHeader * 4, hipHostMallocDefault)) != hipSuccess)
        return fail(QSIM_ERR_DEVICE, "batch status buffer");
    if (!b.uploaded && (e = hipEventCreateWithFlags(&b.uploaded, hipEventDisableTiming)) != hipSuccess)
        return fail(QSIM_ERR_DEVICE, "batch event");
    if (!b.done && (e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming)) != hipSuccess)
        return fail(QSIM_ERR_DEVICE, "batch event");
    if (!b.k0 && (e = hipEventCreate(&b.k0)) != hipSuccess) return fail(QSIM_ERR_DEVICE, "batch event");
    if (!b.k1 && (e = hipEventCreate(&b.k1)) != hipSuccess) return fail(QSIM_ERR_DEVICE, "batch event");
    if ((e = b.ws.ensure(total)) != hipSuccess) return fail(QSIM_ERR_NOMEM, "batch workspace");
    if ((e = b.stage.ensure(total)) != hipSuccess) return fail(QSIM_ERR_DEVICE, "batch staging");
    // passes per circuit (odd: the result is in the other buffer), counted
    // before anything is enqueued so nothing after the launch can fail
    std::vector<uint32_t> flips(n, 0);
    for (size_t k = 0; k < bsmall.size(); ++k) flips[small_circuit[k]] = 1;
    for (const BatchPass &p : bpass) flips[p.circuit] = p.level + 1;
    uint8_t *dev = static_cast<uint8_t *>(b.ws.p);
    // device pointers inside the descriptors
    for (size_t g = 0; g < bpass.size(); ++g) {
        const size_t cb = blob_off + pass_blob_off[g];
        bpass[g].ta.inner = reinterpret_cast<const uint32_t *>(dev + cb + reinterpret_cast<size_t>(bpass[g].ta.inner));
        bpass[g].tm.steps = reinterpret_cast<const TmStep *>(dev + cb + reinterpret_cast<size_t>(bpass[g].tm.steps));
    }
    for (size_t k = 0; k < bsmall.size(); ++k) {
        const uint8_t *p = dev + blob_off + small_blob_off[k];
        if (bsmall[k].direct) bsmall[k].steps_rev = reinterpret_cast<const TmStep *>(p);
        else bsmall[k].ta.inner = reinterpret_cast<const uint32_t *>(p);
    }
    uint8_t *h = static_cast<uint8_t *>(b.stage.p);
    {
        // the copies into the pinned staging buffer, in pieces of at most
        // 1 MiB shared among a few host threads
        struct Piece { uint8_t *dst; const void *src; size_t n; };
        std::vector<Piece> pieces;
        auto add = [&](uint8_t *dst, const void *src, size_t bytes) {
            for (size_t o = 0; o < bytes; o += (1u << 20))
                pieces.push_back({dst + o, static_cast<const uint8_t *>(src) + o, std::min<size_t>(1u << 20, bytes - o)});
        };
        std::memset(h, 0, ctr_bytes);
        add(h + items_off, items.data(), items.size() * 8);
        add(h + pass_off, bpass.data(), bpass.size() * sizeof(BatchPass));
        add(h + small_off, bsmall.data(), bsmall.size() * sizeof(BatchSmall));
        for (uint32_t c = 0; c < n; ++c) add(h + blob_off + circuit_blob_off[c], plans[c].pr.blob.data(), plans[c].pr.blob.size());
        const size_t nt = std::min<size_t>(8, std::max<size_t>(1, total >> 22));   // a thread per 4 MiB, at most 8
        parallel_for((pieces.size() + 63) / 64, (int)nt, [&](size_t k) {
            for (size_t q = 64 * k; q < std::min(64 * k + 64, pieces.size()); ++q)
                std::memcpy(pieces[q].dst, pieces[q].src, pieces[q].n);
        });
    }
    lap("stage");
    // Upload on the side stream (after the slot's previous kernel, which
    // the collect above has already waited for), then the kernel on the
    // caller's stream after the upload; the counter header is copied back
    // behind the kernel so the status can be read without another copy.
    if ((e = hipMemcpyAsync(dev, h, total, hipMemcpyHostToDevice, w.upload)) != hipSuccess)
        return fail(QSIM_ERR_DEVICE, std::string("batch upload: ") + hipGetErrorString(e));
    if ((e = hipEventRecord(b.stage.ev, w.upload)) != hipSuccess) return fail(QSIM_ERR_DEVICE, "batch event");
    b.stage.pending = true;
    if ((e = hipEventRecord(b.uploaded, w.upload)) != hipSuccess) return fail(QSIM_ERR_DEVICE, "batch event");
    if ((e = hipStreamWaitEvent(st, b.uploaded, 0)) != hipSuccess) return fail(QSIM_ERR_DEVICE, "batch event");
    uint32_t *ctr_dev = reinterpret_cast<uint32_t *>(dev);
    // From the launch on, a failure leaves the states part-way: they are
    // poisoned, after whatever did launch has finished (so the slot can be
    // reused).
    auto launched_fail = [&](const char *what, hipError_t err) {
        (void)hipStreamSynchronize(st);
        for (uint32_t c = 0; c < n; ++c) states[c]->poisoned = true;
        return fail(QSIM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(err));
    };
    b.timed = false;
    if (!items.empty()) {
        b.timed = hipEventRecord(b.k0, st) == hipSuccess;
        e = launch_batch(elem, tb, any_sign, reinterpret_cast<const BatchPass *>(dev + pass_off),
                         reinterpret_cast<const BatchSmall *>(dev + small_off),
                         reinterpret_cast<const uint64_t *>(dev + items_off), (uint32_t)items.size(), ctr_dev,
                         1u << 24, tpi, rec_stride, lds, st);
        if (e == hipSuccess) e = injected("batch");
        if (e != hipSuccess) return launched_fail("batch launch", e);
        b.timed = b.timed && hipEventRecord(b.k1, st) == hipSuccess;
    }
    if ((e = hipMemcpyAsync(b.hdr, ctr_dev, kBatchCtrHeader * 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return launched_fail("batch status copy", e);
    if ((e = hipEventRecord(b.done, st)) != hipSuccess) return launched_fail("batch event", e);
    b.pending = true;
    b.info = qsim_batch_info{};
    b.info.circuits = n;
    b.info.items = (uint32_t)items.size();
    b.info.passes = n_passes;
    b.info.workgroups = (uint32_t)std::min<uint64_t>(workers, items.size());
    b.info.algorithmic_bytes = alg_bytes;
    export_batch_tune(tune, elem, &b.info.tuning);
    w.last = w.next;
    w.next ^= 1;
    lap("launch");
    // every circuit's result sits in the buffer its last pass wrote
    for (uint32_t c = 0; c < n; ++c) {
        states[c]->cur ^= (int)(flips[c] & 1u);
        states[c]->last_stream = st;
    }
    return QSIM_OK;
}

}  // namespace

int qsim::state_rebind(qsim_state *s, uint32_t M, int dtype, void *buf0, void *buf1) {
    if (!s || s->owned) return fail(QSIM_ERR_INVALID, "state_rebind needs a wrapped state");
    const uint32_t elem = elem_of((qsim_dtype)dtype);
    if (!elem || M < 1 || M > QSIM_MAX_M || !buf0 || !buf1) return fail(QSIM_ERR_INVALID, "state_rebind arguments");
    DeviceGuard g(s->device);
    hipError_t e = hipStreamSynchronize(s->last_stream);
    if (e != hipSuccess) return device_fail(s, e, "synchronize");
    if (s->elem != elem) s->tune = default_tuning(elem);
    s->M = M;
    s->dtype = (qsim_dtype)dtype;
    s->elem = elem;
    s->buf[0] = buf0;
    s->buf[1] = buf1;
    s->cur = 0;
    s->poisoned = false;
    return QSIM_OK;
}

extern "C" {

qsim_state *qsim_state_create(uint32_t M, qsim_dtype dtype) try {
    const uint32_t elem = elem_of(dtype);
    if (elem == 0) { fail(QSIM_ERR_INVALID, "dtype must be QSIM_C64 or QSIM_C128"); return nullptr; }
    if (M < 1 || M > QSIM_MAX_M) { fail(QSIM_ERR_INVALID, "M out of range [1, 36]"); return nullptr; }
    const uint64_t bytes = (uint64_t)elem << M;
    const uint64_t cap = budget_bytes();
    if (cap && g_allocated.load() + 2 * bytes > cap) {
        fail(QSIM_ERR_NOMEM, "state would exceed QSIM_HBM_BUDGET_BYTES");
        return nullptr;
    }
    qsim_state *s = new (std::nothrow) qsim_state();
    if (!s) { fail(QSIM_ERR_NOMEM, "host allocation failed"); return nullptr; }
    s->M = M;
    s->dtype = dtype;
    s->elem = elem;
    s->tune = default_tuning(elem);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        fail(QSIM_ERR_DEVICE, "no HIP device");
        return nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipMalloc(&s->buf[i], bytes);
        if (e != hipSuccess) {
            if (i == 1) (void)hipFree(s->buf[0]);
            (void)hipGetLastError();
            delete s;
            fail(QSIM_ERR_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
            return nullptr;
        }
    }
    s->owned = true;
    g_allocated += 2 * bytes;
    return s;
} catch (...) {
    (void)host_exception(nullptr);
    return nullptr;
}

qsim_state *qsim_state_wrap(uint32_t M, qsim_dtype dtype, void *buf0, void *buf1) try {
    const uint32_t elem = elem_of(dtype);
    if (elem == 0) { fail(QSIM_ERR_INVALID, "dtype must be QSIM_C64 or QSIM_C128"); return nullptr; }
    if (M < 1 || M > QSIM_MAX_M) { fail(QSIM_ERR_INVALID, "M out of range [1, 36]"); return nullptr; }
    if (!buf0 || !buf1) { fail(QSIM_ERR_INVALID, "buffer is NULL"); return nullptr; }
    if (((uintptr_t)buf0 | (uintptr_t)buf1) & 15u) { fail(QSIM_ERR_INVALID, "buffers must be 16-byte aligned"); return nullptr; }
    const uint64_t bytes = (uint64_t)elem << M;
    const uintptr_t a = (uintptr_t)buf0, b = (uintptr_t)buf1;
    if (a < b + bytes && b < a + bytes) { fail(QSIM_ERR_INVALID, "buffers overlap"); return nullptr; }
    qsim_state *s = new (std::nothrow) qsim_state();
    if (!s) { fail(QSIM_ERR_NOMEM, "host allocation failed"); return nullptr; }
    s->M = M;
    s->dtype = dtype;
    s->elem = elem;
    s->tune = default_tuning(elem);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        fail(QSIM_ERR_DEVICE, "no HIP device");
        return nullptr;
    }
    s->buf[0] = buf0;
    s->buf[1] = buf1;
    s->owned = false;
    return s;
} catch (...) {
    (void)host_exception(nullptr);
    return nullptr;
}

void qsim_state_destroy(qsim_state *s) try {
    if (!s) return;
    DeviceGuard g(s->device);
    (void)hipStreamSynchronize(s->last_stream);
    (void)prof_collect(s);
    for (hipEvent_t ev : s->ev_pool) (void)hipEventDestroy(ev);
    s->ev_pool.clear();
    s->stage.release();
    s->plan.release();
    s->rec.release();
    if (s->owned) {
        (void)hipFree(s->buf[0]);
        (void)hipFree(s->buf[1]);
        g_allocated -= 2 * ((uint64_t)s->elem << s->M);
    }
    delete s;
} catch (...) {
    (void)host_exception(nullptr);
}

uint32_t qsim_state_qubits(const qsim_state *s) { return s ? s->M : 0; }
uint32_t qsim_state_elem_bytes(const qsim_state *s) { return s ? s->elem : 0; }

const void *qsim_state_current(const qsim_state *s) { return s ? s->buf[s->cur] : nullptr; }

int qsim_write_portion(qsim_state *s, uint64_t offset, uint64_t count, const void *host_src) try {
    int rc = check_state(s);
    if (rc) return rc;
    const uint64_t n = 1ull << s->M;
    if (offset > n || count > n - offset) return fail(QSIM_ERR_RANGE, "portion beyond 2^M rows");
    if (count == 0) return QSIM_OK;
    if (!host_src) return fail(QSIM_ERR_INVALID, "host_src is NULL");
    DeviceGuard g(s->device);
    hipError_t e = hipStreamSynchronize(s->last_stream);
    if (e != hipSuccess) return device_fail(s, e, "synchronize");
    e = hipMemcpy(static_cast<uint8_t *>(s->buf[s->cur]) + offset * s->elem, host_src, count * s->elem,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(s, e, "write portion");
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_state_set_product(qsim_state *s, const void *qubits, void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if (!qubits) return fail(QSIM_ERR_INVALID, "qubits is NULL");
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = launch_product(s->elem, s->buf[s->cur], s->M, qubits, st);
    if (e != hipSuccess) return device_fail(s, e, "product-state launch");
    s->last_stream = st;
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_rowmap_build(uint32_t M, const qsim_step *steps, uint64_t L, uint32_t *x_dev, void *hip_stream) try {
    if (M < 1 || M > 32) return fail(QSIM_ERR_INVALID, "qsim_rowmap_build needs 1 <= M <= 32");
    if (!x_dev) return fail(QSIM_ERR_INVALID, "x_dev is NULL");
    int rc = validate_steps(M, steps, L);
    if (rc) return rc;
    for (uint64_t i = 0; i < L; ++i)
        if (steps[i].kind == QSIM_STEP_PHASE)
            return fail(QSIM_ERR_INVALID, "step " + std::to_string(i) + ": a row array holds no signs (phase step)");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    qsim_state *tmp = qsim_state_create(M, QSIM_C64);
    if (!tmp) return QSIM_ERR_NOMEM;
    std::unique_ptr<qsim_state, void (*)(qsim_state *)> hold(tmp, qsim_state_destroy);
    const uint64_t n = 1ull << M;
    hipError_t e = launch_iota(static_cast<uint64_t *>(tmp->buf[0]), n, st);
    if (e != hipSuccess) rc = device_fail(tmp, e, "rowmap iota");
    if (!rc) rc = qsim_apply_steps(tmp, steps, L, st);
    if (!rc) {
        e = launch_narrow(static_cast<const uint64_t *>(tmp->buf[tmp->cur]), x_dev, n, st);
        if (e != hipSuccess) rc = device_fail(tmp, e, "rowmap narrow");
    }
    if (!rc && (e = hipStreamSynchronize(st)) != hipSuccess) rc = device_fail(tmp, e, "rowmap synchronize");
    if (rc) {
        const std::string msg = g_err;   // (kept across the destroy)
        hold.reset();
        g_err = msg;
    }
    return rc;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_rowmap_apply(qsim_state *s, const uint32_t *x_dev, void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if (!x_dev) return fail(QSIM_ERR_INVALID, "x_dev is NULL");
    if (s->M > 32) return fail(QSIM_ERR_INVALID, "row arrays hold 32-bit rows");
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = launch_gather(s->elem, s->buf[s->cur], s->buf[s->cur ^ 1], x_dev, 1ull << s->M, st);
    if (e != hipSuccess) return device_fail(s, e, "rowmap gather");
    s->cur ^= 1;
    s->last_stream = st;
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_apply_steps(qsim_state *s, const qsim_step *steps, uint64_t L, void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if ((rc = validate_steps(s->M, steps, L))) return rc;
    if (L == 0) return QSIM_OK;
    Prepared pr;
    if ((rc = prepare(s, steps, L, pr))) return rc;
    DeviceGuard g(s->device);
    if (!g.ok) return device_fail(s, hipErrorInvalidDevice, "set device");
    return enqueue(s, pr, static_cast<hipStream_t>(hip_stream));
} catch (...) {
    return host_exception(s);
}

int qsim_apply_steps_noalloc(qsim_state *s, const qsim_step *steps, uint64_t L, void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if ((rc = validate_steps(s->M, steps, L))) return rc;
    if (L == 0) return QSIM_OK;
    Prepared pr;
    if ((rc = prepare(s, steps, L, pr))) return rc;
    // the records start on a 256-byte boundary after the blob
    pr.blob.resize((pr.blob.size() + 255) & ~size_t(255), 0);
    const uint64_t need = (uint64_t)pr.blob.size() + pr.rec_bytes;
    if (need > QSIM_NOALLOC_SCRATCH_BYTES)
        return fail(QSIM_ERR_NOMEM, "qsim_apply_steps_noalloc: the plan and one pass's tile records need " +
                                        std::to_string(need) + " bytes, above the scratch of " +
                                        std::to_string((uint64_t)QSIM_NOALLOC_SCRATCH_BYTES) + " bytes");
    DeviceGuard g(s->device);
    if (!g.ok) return device_fail(s, hipErrorInvalidDevice, "set device");
    void *base = nullptr;
    hipError_t e = scratch_address(s->device, &base);
    if (e != hipSuccess) return device_fail(s, e, "scratch address");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    s->last_stream = st;
    if ((e = launch_put(base, pr.blob.data(), pr.blob.size(), st)) != hipSuccess)
        return device_fail(s, e, "plan upload");
    uint8_t *dev = static_cast<uint8_t *>(base);
    return enqueue_launches(s, pr, st, dev, reinterpret_cast<uint32_t *>(dev + pr.blob.size()), false);
} catch (...) {
    return host_exception(s);
}

namespace {

// Turn the first tile pass of `pr` into one that forms its source tile from
// the qubits.  That pass reads the natural layout, so tile-index bit k is
// logical address bit pos_src[k].  Returns false if the plan does not start
// with a tile pass the product kernel runs (one tile per workgroup, 32 rows
// per thread, at most 512 threads).
bool make_product_pass(Prepared &pr, uint32_t M, uint32_t elem, const void *qubits, uint32_t cut) {
    if (pr.launches.size() < 2 || pr.launches[0].kind != Launch::TILEMAP || pr.launches[1].kind != Launch::TILE)
        return false;
    Launch &l = pr.launches[1];
    const uint32_t tb = l.ta.tb, K = tb + l.ta.eb;
    if (l.ta.eb != 5 || tb > 9 || K > 16) return false;
    ProductTileArgs pa{};
    pa.M = M;
    uint32_t k_of[64];
    uint64_t I = 0;
    for (uint32_t k = 0; k < K; ++k) {
        I |= 1ull << l.ta.pos_src[k];
        k_of[l.ta.pos_src[k]] = k;
    }
    for (uint32_t b = 0, i = 0; b < M; ++b)
        if ((I >> b) & 1ull) {
            pa.bit[i] = (uint8_t)b;
            pa.tix[i] = (uint8_t)k_of[b];
            ++i;
        }
    // Stage the partials down to just above address bit cut - 1 and fold
    // bits cut - 1 .. 0 in at the store when the tile holds those bits (the
    // first pass keeps the lowest bits in its tile); otherwise stage the
    // whole tile.
    pa.cut = std::min<uint32_t>(cut, K - 1);
    while (pa.cut > 0) {
        bool low = true;
        for (uint32_t i = 0; i < pa.cut; ++i) low = low && pa.bit[i] == i;
        if (low) break;
        --pa.cut;
    }
    // The kernel folds the factors above the fifth lowest tile bit before
    // splitting at the five: the top address bit must lie above it (not so
    // only for a 2^5-entry tile that holds bit M - 1).
    if (pa.bit[4] + 1u >= M) return false;
    l.pa = pa;
    l.product = true;
    l.q_off = blob_push(pr.blob, qubits, (size_t)4 * M * (elem / 2));
    return true;
}

}  // namespace

int qsim_apply_steps_product(qsim_state *s, const void *qubits, const qsim_step *steps, uint64_t L,
                             void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if (!qubits) return fail(QSIM_ERR_INVALID, "qubits is NULL");
    if ((rc = validate_steps(s->M, steps, L))) return rc;
    Prepared pr;
    if (L > 0 && (rc = prepare(s, steps, L, pr))) return rc;
    DeviceGuard g(s->device);
    if (!g.ok) return device_fail(s, hipErrorInvalidDevice, "set device");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (L > 0 && make_product_pass(pr, s->M, s->elem, qubits, s->tune.product_cut)) return enqueue(s, pr, st);
    // Small states and plans that start otherwise: the product kernel, then the diagram.
    if ((rc = qsim_state_set_product(s, qubits, hip_stream))) return rc;
    return L > 0 ? enqueue(s, pr, st) : QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_apply_tile_pass(qsim_state *s, uint64_t tile_mask, const qsim_step *steps, uint64_t L, void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if ((rc = validate_steps(s->M, steps, L))) return rc;
    const uint64_t all = (1ull << s->M) - 1ull;
    const int K = __builtin_popcountll(tile_mask);
    const int kmax = s->elem == 8 ? kMaxTileBits : kMaxTileBits - 1;
    if ((tile_mask & ~all) || (tile_mask >> 32) || K < 5 || K > kmax || (s->elem == 8 && !(tile_mask & 1ull)))
        return fail(QSIM_ERR_INVALID, "tile_mask: 5..14 bits (13 for complex128) below min(M, 32), bit 0 for complex64");
    const StepLists sl = split_steps(steps, L);
    Pass p;
    p.tile_mask = tile_mask;
    for (uint64_t i = 0; i < L; ++i) {
        if (sl.kd[i] == kStepNot && !((tile_mask >> sl.tg[i]) & 1ull) && (sl.cm[i] & tile_mask))
            return fail(QSIM_ERR_INVALID, "step " + std::to_string(i) + " has a control in the tile but its target outside");
        p.steps.push_back((uint32_t)i);
    }
    Prepared pr;
    if ((rc = prepare_passes(s->M, s->elem, std::vector<Pass>{p}, sl.tg.data(), sl.cm.data(), sl.kd.data(),
                             s->tune.outer_order, false, s->tune.rows_eb, pr, s->tune.xcd_swizzle)))
        return rc;
    DeviceGuard g(s->device);
    if (!g.ok) return device_fail(s, hipErrorInvalidDevice, "set device");
    return enqueue(s, pr, static_cast<hipStream_t>(hip_stream));
} catch (...) {
    return host_exception(s);
}

int qsim_apply_steps_plain(qsim_state *s, const qsim_step *steps, uint64_t L, void *hip_stream) try {
    int rc = check_state(s);
    if (rc) return rc;
    if ((rc = validate_steps(s->M, steps, L))) return rc;
    if (L == 0) return QSIM_OK;
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    s->last_stream = st;
    for (uint64_t i = 0; i < L;) {
        // consecutive NOT steps on one target run as one launch (toggle parity)
        uint64_t j = i + 1;
        if (steps[i].kind == QSIM_STEP_NOT)
            while (j < L && j - i < kPlainRunMax && steps[j].kind == QSIM_STEP_NOT && steps[j].target == steps[i].target)
                ++j;
        hipEvent_t ev_a = nullptr;
        hipError_t e = prof_begin(s, st, &ev_a);
        if (e == hipSuccess) {
            if (steps[i].kind == QSIM_STEP_PHASE) {
                e = launch_plain_phase(s->elem, s->buf[s->cur], s->M, phase_mask(steps[i]), st);
            } else if (j - i == 1) {
                e = launch_plain_step(s->elem, s->buf[s->cur], s->M, steps[i].target, steps[i].control_mask, st);
            } else {
                uint64_t cms[kPlainRunMax];
                for (uint64_t q = i; q < j; ++q) cms[q - i] = steps[q].control_mask;
                e = launch_plain_run(s->elem, s->buf[s->cur], s->M, steps[i].target, cms, (uint32_t)(j - i), st);
            }
        }
        if (e == hipSuccess) e = prof_end(s, st, 2, ev_a, 0);
        if (e != hipSuccess) return device_fail(s, e, "plain step launch");
        i = j;
    }
    s->last_stream = st;
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_read_portion(const qsim_state *cs, uint64_t offset, uint64_t count, void *host_dst) try {
    qsim_state *s = const_cast<qsim_state *>(cs);
    int rc = check_state(s);
    if (rc) return rc;
    const uint64_t n = 1ull << s->M;
    if (offset > n || count > n - offset) return fail(QSIM_ERR_RANGE, "portion beyond 2^M rows");
    if (count == 0) return QSIM_OK;
    if (!host_dst) return fail(QSIM_ERR_INVALID, "host_dst is NULL");
    DeviceGuard g(s->device);
    hipError_t e = hipStreamSynchronize(s->last_stream);
    if (e != hipSuccess) return device_fail(s, e, "synchronize");
    e = hipMemcpy(host_dst, static_cast<const uint8_t *>(s->buf[s->cur]) + offset * s->elem, count * s->elem,
                  hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = injected("read");
    if (e != hipSuccess) return device_fail(s, e, "read portion");
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_read_portion_async(const qsim_state *cs, uint64_t offset, uint64_t count, void *host_dst,
                            void *hip_stream) try {
    qsim_state *s = const_cast<qsim_state *>(cs);
    int rc = check_state(s);
    if (rc) return rc;
    const uint64_t n = 1ull << s->M;
    if (offset > n || count > n - offset) return fail(QSIM_ERR_RANGE, "portion beyond 2^M rows");
    if (count == 0) return QSIM_OK;
    if (!host_dst) return fail(QSIM_ERR_INVALID, "host_dst is NULL");
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemcpyAsync(host_dst, static_cast<const uint8_t *>(s->buf[s->cur]) + offset * s->elem,
                                  count * s->elem, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return device_fail(s, e, "read portion");
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_apply_batch(qsim_state *const *states, const qsim_step *const *steps, const uint64_t *Ls, uint32_t n,
                     void *hip_stream) try {
    if (n == 0) return QSIM_OK;
    if (!states || !steps || !Ls) return fail(QSIM_ERR_INVALID, "NULL array");
    std::unordered_set<const qsim_state *> seen;
    seen.reserve(2 * (size_t)n);
    for (uint32_t c = 0; c < n; ++c) {
        int rc = check_state(states[c]);
        if (rc) return rc;
        if (states[c]->dtype != states[0]->dtype) return fail(QSIM_ERR_INVALID, "states differ in dtype");
        if (states[c]->device != states[0]->device) return fail(QSIM_ERR_INVALID, "states differ in device");
        if (Ls[c] > 0 && !steps[c]) return fail(QSIM_ERR_INVALID, "circuit " + std::to_string(c) + ": steps is NULL");
        if (!seen.insert(states[c]).second) return fail(QSIM_ERR_INVALID, "a state appears twice in the batch");
    }
    // (the steps themselves are validated by the planning threads)
    DeviceGuard g(states[0]->device);
    if (!g.ok) return fail(QSIM_ERR_DEVICE, "set device");
    return batch_enqueue(states, steps, Ls, n, static_cast<hipStream_t>(hip_stream));
} catch (...) {
    return host_exception(nullptr);
}

int qsim_batch_last_status(void) try {
    return batch_status();
} catch (...) {
    return host_exception(nullptr);
}

int qsim_batch_set_tuning(qsim_dtype dtype, const qsim_batch_tuning *t) try {
    const uint32_t elem = elem_of(dtype);
    if (!elem) return fail(QSIM_ERR_INVALID, "dtype must be QSIM_C64 or QSIM_C128");
    BatchTune bt;
    int rc = batch_tune_from(t, &bt);
    if (rc) return rc;
    if (((size_t)elem << batch_tile_bits(bt, elem)) > 128 * 1024)
        return fail(QSIM_ERR_INVALID, "batch tiles above 128 KiB of LDS");
    BatchWorkspace &w = batch_ws();
    std::lock_guard<std::mutex> lk(w.mu);
    w.tune[elem == 8 ? 0 : 1] = bt;
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_batch_get_tuning(qsim_dtype dtype, qsim_batch_tuning *out) try {
    const uint32_t elem = elem_of(dtype);
    if (!elem) return fail(QSIM_ERR_INVALID, "dtype must be QSIM_C64 or QSIM_C128");
    if (!out) return fail(QSIM_ERR_INVALID, "out is NULL");
    BatchWorkspace &w = batch_ws();
    std::lock_guard<std::mutex> lk(w.mu);
    export_batch_tune(w.tune[elem == 8 ? 0 : 1], elem, out);
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_batch_set_tiles_per_item(uint32_t tiles) try {
    if (tiles == 0) tiles = BatchTune{}.tiles_per_item;
    if (tiles > kBatchTilesMax) return fail(QSIM_ERR_INVALID, "tiles_per_item above 256");
    BatchWorkspace &w = batch_ws();
    std::lock_guard<std::mutex> lk(w.mu);
    for (BatchTune &t : w.tune) t.tiles_per_item = tiles;
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

uint32_t qsim_batch_tiles_per_item(void) {
    BatchWorkspace &w = batch_ws();
    std::lock_guard<std::mutex> lk(w.mu);
    return w.tune[0].tiles_per_item;
}

int qsim_batch_last_info(qsim_batch_info *out) try {
    if (!out) return fail(QSIM_ERR_INVALID, "out is NULL");
    BatchWorkspace &w = batch_ws();
    std::lock_guard<std::mutex> lk(w.mu);
    if (w.last < 0) return fail(QSIM_ERR_INVALID, "no batch has run");
    batch_collect(w, w.slot[w.last]);
    *out = w.slot[w.last].info;
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

}  // extern "C"

namespace {

// ---- tuning cache of qsim_autotune and qsim_batch_autotune
// (QSIM_TUNING_CACHE): a JSON object {"<section>": {"<key>": {"<field>":
// <number>, ...}, ...}, ...} that this library writes and reads back, with
// the sections "qsim_tuning" (one state) and "qsim_batch_tuning".

using CacheMap = std::map<std::string, std::map<std::string, double>>;
using CacheFile = std::map<std::string, CacheMap>;

struct JsonIn {
    const char *p, *end;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(char c) {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string &out) {
        if (!lit('"')) return false;
        out.clear();
        while (p < end && *p != '"') {
            if (*p == '\\') return false;   // keys and fields this library writes need no escapes
            out.push_back(*p++);
        }
        return lit('"');
    }
    bool num(double &out) {
        ws();
        char *e = nullptr;
        out = std::strtod(p, &e);
        if (e == p || e > end) return false;
        p = e;
        return true;
    }
};

bool parse_cache(const std::string &text, CacheFile &out) {
    JsonIn in{text.data(), text.data() + text.size()};
    std::string top, key, field;
    if (!in.lit('{')) return false;
    if (in.lit('}')) return true;
    do {
        if (!in.str(top) || !in.lit(':') || !in.lit('{')) return false;
        CacheMap &section = out[top];
        if (in.lit('}')) continue;
        do {
            if (!in.str(key) || !in.lit(':') || !in.lit('{')) return false;
            auto &entry = section[key];
            if (in.lit('}')) continue;
            do {
                double v = 0;
                if (!in.str(field) || !in.lit(':') || !in.num(v)) return false;
                entry[field] = v;
            } while (in.lit(','));
            if (!in.lit('}')) return false;
        } while (in.lit(','));
        if (!in.lit('}')) return false;
    } while (in.lit(','));
    return in.lit('}');
}

std::string write_cache(const CacheFile &file) {
    std::string o = "{";
    char buf[64];
    bool first_section = true;
    for (const auto &sec : file) {
        o += (first_section ? "\n  \"" : ",\n  \"") + sec.first + "\": {";
        first_section = false;
        bool first = true;
        for (const auto &kv : sec.second) {
            o += first ? "\n    \"" : ",\n    \"";
            first = false;
            o += kv.first + "\": {";
            bool f2 = true;
            for (const auto &fv : kv.second) {
                std::snprintf(buf, sizeof buf, "%.6g", fv.second);
                o += (f2 ? "\"" : ", \"") + fv.first + "\": " + buf;
                f2 = false;
            }
            o += "}";
        }
        o += "\n  }";
    }
    return o + "\n}\n";
}

bool read_file(const char *path, std::string &out) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t k;
    out.clear();
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, k);
    std::fclose(f);
    return true;
}

bool write_file(const char *path, const std::string &text) {
    // written beside it under a name of this process, then renamed over it:
    // readers see the old file or the new one, never a part of either
    const std::string tmp = std::string(path) + "." + std::to_string((long)getpid()) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok) return false;
    return std::rename(tmp.c_str(), path) == 0;
}

// The cache file named by QSIM_TUNING_CACHE, if any: false (and nothing
// read) when it is set but unreadable as a cache; a missing file is an
// empty cache, to be written.
bool load_cache(const char *path, CacheFile &out) {
    std::string text;
    return !read_file(path, text) || parse_cache(text, out);
}

std::string device_arch(int device) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    return arch;
}

// Powers of two around [lo, hi]: "L<p>-<q>" with p <= lo (0 for lo = 0) and q >= hi.
std::string l_band(uint64_t lo, uint64_t hi) {
    uint64_t plo = 0, phi = 1;
    if (lo > 0) for (plo = 1; plo * 2 <= lo; plo *= 2) {}
    while (phi < hi) phi *= 2;
    return "L" + std::to_string(plo) + "-" + std::to_string(phi);
}

// Cache key of a batch: device architecture, dtype, range of M and range
// of L rounded out to powers of two.
std::string batch_cache_key(int device, uint32_t elem, qsim_state *const *states, const uint64_t *Ls, uint32_t n) {
    uint32_t mlo = 64, mhi = 0;
    uint64_t llo = ~0ull, lhi = 0;
    for (uint32_t c = 0; c < n; ++c) {
        mlo = std::min(mlo, states[c]->M);
        mhi = std::max(mhi, states[c]->M);
        llo = std::min(llo, Ls[c]);
        lhi = std::max(lhi, Ls[c]);
    }
    return device_arch(device) + ":" + (elem == 8 ? "c64" : "c128") + ":M" + std::to_string(mlo) + "-" +
           std::to_string(mhi) + ":" + l_band(llo, lhi);
}

}  // namespace

extern "C" {

int qsim_batch_autotune(qsim_state *const *states, const qsim_step *const *steps, const uint64_t *Ls, uint32_t n,
                        void *hip_stream, qsim_batch_tuning *out) try {
    if (n == 0) return out ? qsim_batch_get_tuning(QSIM_C64, out) : QSIM_OK;
    if (!states || !steps || !Ls) return fail(QSIM_ERR_INVALID, "NULL array");
    for (uint32_t c = 0; c < n; ++c) {
        int rc = check_state(states[c]);
        if (rc) return rc;
        if (Ls[c] > 0 && !steps[c]) return fail(QSIM_ERR_INVALID, "circuit " + std::to_string(c) + ": steps is NULL");
    }
    const uint32_t elem = states[0]->elem;
    const int di = elem == 8 ? 0 : 1;
    BatchWorkspace &w = batch_ws();
    auto set = [&](const BatchTune &t) {
        std::lock_guard<std::mutex> lk(w.mu);
        w.tune[di] = t;
    };
    const char *cache_path = std::getenv("QSIM_TUNING_CACHE");
    const std::string key = batch_cache_key(states[0]->device, elem, states, Ls, n);
    CacheFile cache_file;
    CacheMap &cache = cache_file["qsim_batch_tuning"];
    bool cache_ok = false;
    if (cache_path && *cache_path) {
        cache_ok = load_cache(cache_path, cache_file);
        auto it = cache.find(key);
        if (cache_ok && it != cache.end()) {
            qsim_batch_tuning in{};
            auto get = [&](const char *f) { auto x = it->second.find(f); return x == it->second.end() ? 0u : (uint32_t)x->second; };
            in.tiles_per_item = get("tiles_per_item");
            in.tile_bits = get("tile_bits");
            in.circuit_tiles = get("circuit_tiles");
            in.plan_search = get("plan_search");
            in.order = get("order");
            BatchTune bt;
            if (batch_tune_from(&in, &bt) == QSIM_OK) {
                set(bt);
                if (out) {
                    export_batch_tune(bt, elem, out);
                    out->from_cache = 1;
                }
                return QSIM_OK;
            }
        }
    }
    // Each trial applies the batch and then the batch of reversed diagrams,
    // which undoes it (every step is its own inverse), so the states end as
    // they began: one such pair to settle, then two timed back to back.
    std::vector<std::vector<qsim_step>> rev(n);
    std::vector<const qsim_step *> rev_ptr(n);
    for (uint32_t c = 0; c < n; ++c) {
        rev[c].assign(steps[c], steps[c] + Ls[c]);
        std::reverse(rev[c].begin(), rev[c].end());
        rev_ptr[c] = rev[c].data();
    }
    BatchTune keep;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        keep = w.tune[di];
    }
    // an exception part-way leaves the setting the call found
    struct RestoreOnThrow {
        BatchWorkspace &w;
        int di;
        BatchTune keep;
        int before = std::uncaught_exceptions();
        ~RestoreOnThrow() {
            if (std::uncaught_exceptions() > before) {
                std::lock_guard<std::mutex> lk(w.mu);
                w.tune[di] = keep;
            }
        }
    } restore_on_throw{w, di, keep};
    // A trial's cost is the time per batch of a long run of batches: the
    // host plans the next batch while the device runs the current one, so
    // it is the larger of the kernel's device time and the host's enqueue
    // time (each the mean over a batch and its reverse, after a settling
    // pair).
    auto trial = [&](const BatchTune &t, double *ms) {
        set(t);
        int rc = qsim_apply_batch(states, steps, Ls, n, hip_stream);
        if (!rc) rc = qsim_apply_batch(states, rev_ptr.data(), Ls, n, hip_stream);
        if (!rc) rc = batch_status();
        double host = 0;
        for (int k = 0; k < 2 && !rc; ++k) {
            const auto t0 = std::chrono::steady_clock::now();   // nothing in flight: enqueue time only
            rc = qsim_apply_batch(states, k ? rev_ptr.data() : steps, Ls, n, hip_stream);
            host += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (!rc) rc = batch_status();
        }
        double kern = 0;
        if (!rc) {
            std::lock_guard<std::mutex> lk(w.mu);
            kern = (w.slot[0].info.kernel_ms + w.slot[1].info.kernel_ms) / 2;
        }
        *ms = std::max(host / 2, kern);
        return rc;
    };
    BatchTune best;   // the defaults
    double best_ms = 0, default_ms = 0;
    int rc = trial(best, &best_ms);
    default_ms = best_ms;
    // one parameter at a time, each candidate against the best so far
    const uint32_t kb = batch_tile_bits(BatchTune{}, elem);
    const std::vector<std::pair<int, std::vector<uint32_t>>> space = {
        {0, {1}},                  // order: level by level
        {1, {kb - 1}},             // tile bits: one less
        {2, {1}},                  // planning with the greedy scan alone
        {3, {1, 8, 16, 32, 128}},  // whole-circuit cut-off (1 = none)
        {4, {8, 16, 64}},          // tiles per item
    };
    for (const auto &dim : space) {
        for (uint32_t v : dim.second) {
            if (rc) break;
            BatchTune t = best;
            uint32_t *f = dim.first == 0 ? &t.order : dim.first == 1 ? &t.tile_bits : dim.first == 2 ? &t.plan_search
                          : dim.first == 3 ? &t.circuit_tiles : &t.tiles_per_item;
            if (dim.first == 1 && !t.tile_bits) t.tile_bits = kb;
            if (*f == v) continue;
            *f = v;
            double ms = 0;
            if ((rc = trial(t, &ms))) break;
            if (ms < 0.995 * best_ms) {   // a clear gain only
                best = t;
                best_ms = ms;
            }
        }
    }
    set(rc ? keep : best);
    if (rc) return rc;
    if (cache_path && *cache_path && cache_ok) {
        auto &e = cache[key];
        e["tiles_per_item"] = best.tiles_per_item;
        e["tile_bits"] = batch_tile_bits(best, elem);
        e["circuit_tiles"] = best.circuit_tiles;
        e["plan_search"] = best.plan_search;
        e["order"] = best.order;
        e["best_ms"] = best_ms;
        e["default_ms"] = default_ms;
        (void)write_file(cache_path, write_cache(cache_file));   // a cache that cannot be written is skipped
    }
    if (out) {
        export_batch_tune(best, elem, out);
        out->best_ms = (float)best_ms;
        out->default_ms = (float)default_ms;
    }
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_autotune(qsim_state *s, const qsim_step *steps, uint64_t L, void *hip_stream, qsim_tuning *out) try {
    int rc = check_state(s);
    if (rc) return rc;
    if ((rc = validate_steps(s->M, steps, L))) return rc;
    const Tuning keep = s->tune;
    auto export_tuning = [&](const Tuning &t) {
        if (out) export_tuning_to(t, out);
    };
    if (L == 0 || (int)s->M <= s->tune.small_bits) {   // one launch: nothing to choose
        export_tuning(s->tune);
        return QSIM_OK;
    }
    // A choice stored for this architecture, dtype, M and band of L (the
    // fields the candidates below vary, on top of the state's tuning).
    const char *cache_path = std::getenv("QSIM_TUNING_CACHE");
    const std::string key = device_arch(s->device) + ":" + (s->elem == 8 ? "c64" : "c128") + ":M" +
                            std::to_string(s->M) + ":" + l_band(L, L);
    CacheFile cache_file;
    CacheMap &cache = cache_file["qsim_tuning"];
    const bool cache_ok = cache_path && *cache_path && load_cache(cache_path, cache_file);
    if (cache_ok) {
        auto it = cache.find(key);
        if (it != cache.end()) {
            qsim_tuning in{};
            export_tuning_to(keep, &in);
            auto get = [&](const char *f, uint32_t dflt) {
                auto x = it->second.find(f);
                return x == it->second.end() ? dflt : (uint32_t)x->second;
            };
            in.tile_bits = get("tile_bits", in.tile_bits);
            in.kernel_variant = get("kernel_variant", in.kernel_variant);
            in.mid_low_bits = get("mid_low_bits", in.mid_low_bits);
            in.plan_search = get("plan_search", in.plan_search);
            Tuning t;
            if (tuning_from(&in, s->elem, &t) == QSIM_OK) {   // (an entry out of range is measured again)
                s->tune = t;
                export_tuning(t);
                return QSIM_OK;
            }
        }
    }
    // Candidates around the measured defaults: tile size, kernel shape and
    // the low bits of the middle passes.
    // -1 for plan_search keeps the state's planner setting; 1 is the mask
    // climb, 2 the climb with the beam search over whole plans.
    struct Cand { int tile_bits; uint32_t variant; int mid_low; int search; };
    std::vector<Cand> cands;
    if (s->elem == 8)
        cands = {{13, 0, 2, -1}, {13, 0, 3, -1}, {13, 1, 2, -1}, {14, 1, 2, -1}, {14, 2, 2, -1}, {12, 0, 2, -1},
                 {13, 0, 2, 1}, {13, 0, 1, 2}};
    else
        cands = {{13, 1, 2, -1}, {13, 0, 2, -1}, {12, 0, 2, -1}, {12, 1, 2, -1}, {13, 1, 3, -1},
                 {12, 0, 1, 1}, {12, 0, 1, 2}, {12, 0, 2, 1}, {13, 1, 1, 1}};
    std::vector<qsim_step> rev(steps, steps + L);
    std::reverse(rev.begin(), rev.end());
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // the events are released however the function ends, and an exception
    // part-way leaves the state with the tuning it came with
    struct Scope {
        qsim_state *s;
        Tuning keep;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int before = std::uncaught_exceptions();
        ~Scope() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (std::uncaught_exceptions() > before) s->tune = keep;
        }
    } scope{s, keep};
    hipEvent_t &e0 = scope.e0, &e1 = scope.e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return device_fail(s, hipErrorOutOfMemory, "autotune events");
    // Each candidate applies the diagram (timed) and then its reverse, which
    // undoes it (every step is its own inverse), so the state is unchanged.
    float best_ms = 0.f, first_ms = 0.f;
    Tuning best = keep;
    bool first = true;
    for (const Cand &c : cands) {
        Tuning t = keep;
        t.tile_bits = std::min(c.tile_bits, s->elem == 8 ? kMaxTileBits : kMaxTileBits - 1);
        t.variant = c.variant;
        t.mid_low_bits = std::min(c.mid_low, t.low_bits);
        if (c.search >= 0) t.plan_search = c.search;
        if ((uint32_t)t.tile_bits < t.rows_eb || (uint32_t)t.tile_bits - t.rows_eb > 10) continue;
        s->tune = t;
        if ((rc = qsim_apply_steps(s, rev.data(), L, st)) || (rc = qsim_apply_steps(s, steps, L, st))) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = device_fail(s, hipErrorUnknown, "autotune"); break; }
        if ((rc = qsim_apply_steps(s, steps, L, st))) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = device_fail(s, hipErrorUnknown, "autotune");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // the state now holds U k1; applying the reversed list undoes it
        if ((rc = qsim_apply_steps(s, rev.data(), L, st))) break;
        if (first) first_ms = ms;
        if (first || ms < best_ms) {
            best_ms = ms;
            best = t;
            first = false;
        }
    }
    (void)hipStreamSynchronize(st);
    s->tune = rc ? keep : best;
    if (rc) return rc;
    if (cache_ok) {
        qsim_tuning ext{};
        export_tuning_to(best, &ext);
        auto &e = cache[key];
        e["tile_bits"] = ext.tile_bits;
        e["kernel_variant"] = ext.kernel_variant;
        e["mid_low_bits"] = ext.mid_low_bits;
        e["plan_search"] = ext.plan_search;
        e["best_ms"] = best_ms;
        e["default_ms"] = first_ms;
        (void)write_file(cache_path, write_cache(cache_file));   // a cache that cannot be written is skipped
    }
    export_tuning(best);
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_state_set_tuning(qsim_state *s, const qsim_tuning *tuning) try {
    int rc = check_state(s);
    if (rc) return rc;
    Tuning t;
    if ((rc = tuning_from(tuning, s->elem, &t))) return rc;
    s->tune = t;
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_plan_describe(uint32_t M, qsim_dtype dtype, const qsim_step *steps, uint64_t L,
                       const qsim_tuning *tuning, uint32_t *n_passes, uint64_t *pass_mask, uint32_t *pass_len,
                       uint32_t cap, uint32_t *order) try {
    const uint32_t elem = elem_of(dtype);
    if (elem == 0) return fail(QSIM_ERR_INVALID, "dtype must be QSIM_C64 or QSIM_C128");
    if (M < 1 || M > QSIM_MAX_M) return fail(QSIM_ERR_INVALID, "M out of range [1, 36]");
    int rc = validate_steps(M, steps, L);
    if (rc) return rc;
    Tuning t;
    if ((rc = tuning_from(tuning, elem, &t))) return rc;
    const StepLists sl = split_steps(steps, L);
    std::vector<Pass> passes;
    try {
        passes = plan_passes(M, sl.tg.data(), sl.cm.data(), sl.kd.data(), L, plan_config(t, elem));
    } catch (const std::logic_error &e) {   // (host memory and threads: host_exception)
        return fail(QSIM_ERR_INVALID, std::string("planner: ") + e.what());
    }
    if (n_passes) *n_passes = (uint32_t)passes.size();
    size_t k = 0;
    for (size_t p = 0; p < passes.size(); ++p) {
        if (p < cap) {
            if (pass_mask) pass_mask[p] = passes[p].tile_mask;
            if (pass_len) pass_len[p] = (uint32_t)passes[p].steps.size();
        }
        for (uint32_t s : passes[p].steps)
            if (order) order[k++] = s;
    }
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

int qsim_state_profile(qsim_state *s, int enable) try {
    int rc = check_state(s);
    if (rc) return rc;
    DeviceGuard g(s->device);
    hipError_t e = prof_collect(s);
    if (e != hipSuccess) return device_fail(s, e, "profiling");
    s->profiling = enable != 0;
    if (enable) s->prof = qsim_profile{};
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_state_profile_read(qsim_state *s, qsim_profile *out) try {
    int rc = check_state(s);
    if (rc) return rc;
    if (!out) return fail(QSIM_ERR_INVALID, "out is NULL");
    DeviceGuard g(s->device);
    hipError_t e = prof_collect(s);
    if (e != hipSuccess) return device_fail(s, e, "profiling");
    *out = s->prof;
    return QSIM_OK;
} catch (...) {
    return host_exception(s);
}

int qsim_copy_bytes(void *dst, const void *src, uint64_t bytes, void *hip_stream) try {
    if (!dst || !src) return fail(QSIM_ERR_INVALID, "NULL pointer");
    if ((bytes & 15u) || (((uintptr_t)dst | (uintptr_t)src) & 15u))
        return fail(QSIM_ERR_INVALID, "size and pointers must be multiples of 16");
    hipError_t e = launch_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QSIM_ERR_DEVICE, std::string("copy launch: ") + hipGetErrorString(e));
    return QSIM_OK;
} catch (...) {
    return host_exception(nullptr);
}

const char *qsim_last_error(void) { return g_err.c_str(); }

const char *qsim_version(void) { return "qsim 0.1 (gfx950)"; }

}  // extern "C"
