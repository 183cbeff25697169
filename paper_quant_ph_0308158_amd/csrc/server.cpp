// Serving runtime of libqsim (qsim_server_* in include/qsim.h).
//
// Requests (M, dtype, initial state, wiring diagram) are queued by
// qsim_server_submit.  A scheduler admits them, in arrival order with
// bounded overtaking, while both a slot (one HIP stream and one worker
// thread) and room in the HBM arena are free; admitted requests run
// concurrently on their own streams, so work that arrives while others are
// on the device overlaps with them (continuous batching).  Each worker
// enqueues the initial state, the fused apply and the read-back of the
// result in contiguous row ranges, first row to last (how the paper's
// Abstract and Conclusions hand the result on), into pinned buffers,
// digests every portion as it lands, then returns its memory to the arena.
// With fcfs set the server runs one request at a time in arrival order: the
// plain comparator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qsim.h"
#include "qsim_internal.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over one device arena, 2 MiB granules, with
// coalescing of neighbouring free ranges.
class Arena {
  public:
    static constexpr uint64_t kAlign = 2ull << 20;
    hipError_t init(uint64_t bytes) {
        bytes = (bytes / kAlign) * kAlign;
        if (bytes == 0) return hipErrorInvalidValue;
        hipError_t e = hipMalloc(&base_, bytes);
        if (e != hipSuccess) return e;
        size_ = bytes;
        free_[0] = bytes;
        return hipSuccess;
    }
    ~Arena() {
        if (base_) (void)hipFree(base_);
    }
    // Offset of a free range of `bytes`, or ~0 when none fits.
    uint64_t alloc(uint64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                return off;
            }
        }
        return ~0ull;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint8_t *ptr(uint64_t off) const { return static_cast<uint8_t *>(base_) + off; }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }

  private:
    void *base_ = nullptr;
    uint64_t size_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
};

// 64-bit digest of a result in row order: the sum (mod 2^64), over its
// 8-byte words w_j (j counted from the first byte of the result), of
// mix(w_j ^ mix(j + kKey)), finally mixed with the byte count.  Every word
// is keyed by its position, so portions fold in any order and a host can
// recompute the digest of a result with vector arithmetic.  mix is the
// 64-bit finaliser of the SplitMix64 generator (Steele, Lea and Flood).
struct Digest {
    static constexpr uint64_t kKey = 0x9E3779B97F4A7C15ull;
    uint64_t sum = 0;
    uint64_t n = 0;   // bytes folded
    static uint64_t mix(uint64_t z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    void add(const void *p, size_t bytes) {
        const uint64_t *w = static_cast<const uint64_t *>(p);
        const uint64_t j0 = n / 8;
        uint64_t acc = 0;
        for (size_t i = 0; i < bytes / 8; ++i) acc += mix(w[i] ^ mix(j0 + i + kKey));
        sum += acc;
        n += bytes;
    }
    uint64_t value() const { return mix(sum ^ mix(n)); }
};

struct Request {
    int64_t id = 0;
    uint32_t M = 0;
    qsim_dtype dtype = QSIM_C64;
    uint32_t elem = 8;
    std::vector<uint8_t> k1;        // empty: the alternating input
    std::vector<qsim_step> steps;
    qsim_request_info info{};
    uint64_t arena_off = ~0ull;
    uint64_t bytes = 0;             // two buffers
    uint32_t bypassed = 0;
};

}  // namespace

struct qsim_server {
    qsim_server_config cfg{};
    int device = 0;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work;   // workers wait for admitted requests
    std::condition_variable cv_done;   // drain waits for completions
    std::deque<std::shared_ptr<Request>> queue;      // submitted, not admitted
    std::deque<std::shared_ptr<Request>> admitted;   // admitted, not yet taken by a worker
    std::map<int64_t, std::shared_ptr<Request>> all;
    int64_t next_id = 0;
    uint32_t busy_slots = 0;
    uint64_t outstanding = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::string error;

    // Admit queued requests while a slot and arena room are free.  The
    // queue is served in arrival order; a later request may overtake a head
    // that does not fit yet, but the head is overtaken at most max_bypass
    // times before admission waits for it (fcfs: never overtaken).
    void admit_locked() {
        const uint32_t slots = cfg.fcfs ? 1u : cfg.max_slots;
        if (queue.empty()) return;
        Request *head = queue.front().get();
        uint32_t overtook = 0;
        auto it = queue.begin();
        while (it != queue.end() && busy_slots + admitted.size() < slots) {
            Request &r = **it;
            const uint64_t off = arena.alloc(r.bytes);
            if (off != ~0ull) {
                r.arena_off = off;
                r.info.t_admit_ns = now_ns();
                if (&r != head) ++overtook;
                admitted.push_back(*it);
                it = queue.erase(it);
                cv_work.notify_one();
                continue;
            }
            if (cfg.fcfs || (&r == head && r.bypassed >= cfg.max_bypass)) break;
            ++it;
        }
        if (!queue.empty() && queue.front().get() == head) head->bypassed += overtook;
    }

    void worker_main(uint32_t slot);
};

namespace {

// Entry i of the alternating input: |S| (+1, -1, +1, ...) with |S| = 2^(-M/2)
// (the paper's example input, Sec. 2(b) and Sec. 4), written as raw words.
__global__ void k_fill_alternating(uint64_t *w, uint64_t n, uint32_t words_per_entry, uint64_t pos,
                                   uint64_t neg) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        w[i * words_per_entry] = (i & 1u) ? neg : pos;
        if (words_per_entry == 2) w[i * 2 + 1] = 0;
    }
}

void alternating_words(uint32_t M, uint32_t elem, uint64_t *pos, uint64_t *neg) {
    const double s = std::pow(2.0, -0.5 * (double)M);
    if (elem == 8) {
        const float f = (float)s, g = -(float)s;
        uint32_t a, b;
        std::memcpy(&a, &f, 4);
        std::memcpy(&b, &g, 4);
        *pos = a;   // imaginary half is zero
        *neg = b;
    } else {
        const double g = -s;
        std::memcpy(pos, &s, 8);
        std::memcpy(neg, &g, 8);
    }
}

}  // namespace

void qsim_server::worker_main(uint32_t slot) {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    void *pinned[2] = {nullptr, nullptr};
    const uint64_t portion_max = (uint64_t)cfg.portion_entries * 16u;
    bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; i < 2 && ok; ++i) {
        ok = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc(&pinned[i], portion_max, hipHostMallocDefault) == hipSuccess;
    }
    (void)slot;
    qsim_state *state = nullptr;   // one wrapped state per slot, re-pointed per request
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || !admitted.empty(); });
            if (admitted.empty()) break;  // stopping and nothing left
            r = admitted.front();
            admitted.pop_front();
            ++busy_slots;
        }
        int status = ok ? QSIM_OK : QSIM_ERR_DEVICE;
        Digest dg;
        // digest = 1: every request; k > 1: every k-th request by id
        const bool digest = cfg.digest == 1 || (cfg.digest > 1 && r->id % cfg.digest == 0);
        const uint64_t n = 1ull << r->M;
        const uint64_t half = r->bytes / 2;
        uint8_t *b0 = arena.ptr(r->arena_off), *b1 = b0 + half;
        if (ok && !state) state = qsim_state_wrap(r->M, r->dtype, b0, b1);
        qsim_state *s = state;
        if (!s || qsim::state_rebind(s, r->M, r->dtype, b0, b1) != QSIM_OK) {
            s = nullptr;
            status = QSIM_ERR_DEVICE;
        }
        if (status == QSIM_OK) {
            if (r->k1.empty()) {
                uint64_t pos, neg;
                alternating_words(r->M, r->elem, &pos, &neg);
                const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 1ull << 20);
                hipLaunchKernelGGL(k_fill_alternating, dim3((uint32_t)blocks), dim3(256), 0, st,
                                   reinterpret_cast<uint64_t *>(b0), n, r->elem / 8u, pos, neg);
                if (hipGetLastError() != hipSuccess) status = QSIM_ERR_DEVICE;
            } else if (hipMemcpyAsync(b0, r->k1.data(), r->k1.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
                status = QSIM_ERR_DEVICE;
            }
        }
        if (status == QSIM_OK)
            status = qsim_apply_steps(s, r->steps.data(), r->steps.size(), st);
        if (status == QSIM_OK) {
            // read back in portions, two in flight, digesting each as it lands
            const uint64_t per = cfg.portion_entries;
            const uint64_t nport = (n + per - 1) / per;
            uint64_t cnt[2] = {0, 0};
            auto issue = [&](uint64_t p) {
                const int k = (int)(p & 1);
                cnt[k] = std::min(per, n - p * per);
                int rc = qsim_read_portion_async(s, p * per, cnt[k], pinned[k], st);
                if (rc == QSIM_OK && hipEventRecord(ev[k], st) != hipSuccess) rc = QSIM_ERR_DEVICE;
                return rc;
            };
            status = issue(0);
            if (status == QSIM_OK && nport > 1) status = issue(1);
            for (uint64_t p = 0; p < nport && status == QSIM_OK; ++p) {
                const int k = (int)(p & 1);
                if (hipEventSynchronize(ev[k]) != hipSuccess) { status = QSIM_ERR_DEVICE; break; }
                if (digest) dg.add(pinned[k], cnt[k] * r->elem);
                else dg.n += cnt[k] * r->elem;
                if (p + 2 < nport) status = issue(p + 2);
            }
        }
        if (s && hipStreamSynchronize(st) != hipSuccess) status = QSIM_ERR_DEVICE;
        {
            std::lock_guard<std::mutex> lk(mu);
            r->info.status = status;
            r->info.digest = digest ? dg.value() : 0;
            r->info.bytes = dg.n;
            r->info.t_done_ns = now_ns();
            r->info.done = 1;
            arena.release(r->arena_off, r->bytes);
            r->k1.clear();
            r->k1.shrink_to_fit();
            --busy_slots;
            --outstanding;
            admit_locked();
        }
        cv_done.notify_all();
    }
    if (state) qsim_state_destroy(state);
    for (int i = 0; i < 2; ++i) {
        if (pinned[i]) (void)hipHostFree(pinned[i]);
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
    if (st) (void)hipStreamDestroy(st);
}

extern "C" {

qsim_server *qsim_server_create(const qsim_server_config *cfg) {
    qsim_server_config c{};
    if (cfg) c = *cfg;
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = 200ull * 1000 * 1000 * 1000;
    if (c.max_slots == 0) c.max_slots = 4;   // measured: 2, 3, 4, 6, 8, 16 slots; 4 best in p50, mean and capacity
    if (c.portion_entries == 0) c.portion_entries = 1u << 20;
    if (c.max_bypass == 0) c.max_bypass = 64;
    if (c.max_slots > 64) return nullptr;
    auto *s = new (std::nothrow) qsim_server();
    if (!s) return nullptr;
    s->cfg = c;
    if (hipGetDevice(&s->device) != hipSuccess || s->arena.init(c.hbm_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return nullptr;
    }
    const uint32_t nworkers = c.fcfs ? 1u : c.max_slots;
    try {
        s->workers.reserve(nworkers);
        for (uint32_t i = 0; i < nworkers; ++i) s->workers.emplace_back(&qsim_server::worker_main, s, i);
    } catch (...) {
        // a worker that cannot be started: stop the ones that did
        (void)qsim::host_exception(nullptr);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        delete s;
        return nullptr;
    }
    return s;
}

int64_t qsim_server_submit(qsim_server *srv, uint32_t M, qsim_dtype dtype, const void *host_k1,
                           const qsim_step *steps, uint64_t L) try {
    if (!srv) return QSIM_ERR_INVALID;
    const uint32_t elem = dtype == QSIM_C64 ? 8u : (dtype == QSIM_C128 ? 16u : 0u);
    if (!elem || M < 1 || M > QSIM_MAX_M) return QSIM_ERR_INVALID;
    if (L > 0 && !steps) return QSIM_ERR_INVALID;
    const uint64_t all = (1ull << M) - 1ull;
    for (uint64_t i = 0; i < L; ++i)
        if (steps[i].kind > QSIM_STEP_PHASE || steps[i].target >= M || (steps[i].control_mask & ~all) ||
            ((steps[i].control_mask >> steps[i].target) & 1ull))
            return QSIM_ERR_INVALID;
    auto r = std::make_shared<Request>();
    r->M = M;
    r->dtype = dtype;
    r->elem = elem;
    r->bytes = 2ull * ((uint64_t)elem << M);
    if (r->bytes > srv->arena.size()) return QSIM_ERR_NOMEM;
    if (host_k1) {
        r->k1.resize((uint64_t)elem << M);
        std::memcpy(r->k1.data(), host_k1, r->k1.size());
    }
    r->steps.assign(steps, steps + L);
    r->info.t_submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    r->id = srv->next_id;
    srv->queue.push_back(r);
    try {
        srv->all[r->id] = r;
    } catch (...) {
        srv->queue.pop_back();   // (a request that cannot be recorded is not queued)
        throw;
    }
    ++srv->next_id;
    ++srv->outstanding;
    srv->admit_locked();
    return r->id;
} catch (...) {
    return qsim::host_exception(nullptr);
}

int qsim_server_drain(qsim_server *srv) try {
    if (!srv) return QSIM_ERR_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
    return QSIM_OK;
} catch (...) {
    return qsim::host_exception(nullptr);
}

int qsim_server_request_info(qsim_server *srv, int64_t id, qsim_request_info *out) try {
    if (!srv || !out) return QSIM_ERR_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return QSIM_ERR_RANGE;
    *out = it->second->info;
    return QSIM_OK;
} catch (...) {
    return qsim::host_exception(nullptr);
}

int qsim_server_stats(qsim_server *srv, uint64_t *arena_bytes, uint64_t *arena_used, uint32_t *queued,
                      uint32_t *running) try {
    if (!srv) return QSIM_ERR_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (arena_bytes) *arena_bytes = srv->arena.size();
    if (arena_used) *arena_used = srv->arena.used();
    if (queued) *queued = (uint32_t)srv->queue.size();
    if (running) *running = srv->busy_slots + (uint32_t)srv->admitted.size();
    return QSIM_OK;
} catch (...) {
    return qsim::host_exception(nullptr);
}

void qsim_server_destroy(qsim_server *srv) try {
    if (!srv) return;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    delete srv;
} catch (...) {
    (void)qsim::host_exception(nullptr);
}

}  // extern "C"
