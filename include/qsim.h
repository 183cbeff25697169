/*
 * qsim.h - C ABI of libqsim: applying a wiring diagram of controlled-NOT
 * steps to a 2^M-entry complex state vector on an AMD Instinct MI355X
 * (gfx950), after J. R. Burger, "New approaches to quantum computer
 * simulation in a classical supercomputer" (quant-ph/0308158).
 *
 * The operation (Sec. 2(a), 2(h), 2(i) Summary of Method):
 *     k2 = U_L ... U_2 U_1 k1
 * where U_s is the matrix of wiring-diagram step s: a NOT on one target
 * address bit that fires when all of its controlling bits are 1.  Each U_s
 * is a symmetric permutation matrix with a single 1 per row (Sec. 2(a)), so
 * entries of the state are only moved, never combined: every result is
 * exact to the bit.
 *
 * Conventions used throughout:
 *  - Address bit b (0-based) is the paper's a(b+1); bit 0 is the LSB
 *    (Sec. 2(b)).  Entry i of a state is row i counted from the top, for
 *    i = 0 .. 2^M - 1.
 *  - steps[0] is U_1 and acts first.
 *  - A step's control_mask holds one bit per controlling address bit.  All
 *    of them must be 1 for the NOT to fire (Sec. 2(g), generalised to any
 *    number of controls); control_mask == 0 is the unconditional NOT
 *    (Sec. 2(e)).
 *  - Beyond the wiring-diagram class, a step may instead be a controlled
 *    phase of -1 (kind QSIM_STEP_PHASE): the diagonal matrix that negates
 *    every row whose target bit and control bits are all 1.  Diagrams
 *    mixing both kinds give the signed permutation matrices, such as the
 *    paper's first example of a unitary matrix (Sec. 2(a)).  Negation flips
 *    the sign bit of both parts of an entry (IEEE 754 negate), so results
 *    stay exact to the bit.
 *  - Entries are opaque words of 8 bytes (QSIM_C64: two float32) or 16
 *    bytes (QSIM_C128: two float64), stored contiguously in row order.  The
 *    library never reads them as floating point: NaN payloads, -0.0 and
 *    subnormals are preserved.
 *
 * Memory: a state owns (or borrows) two device buffers of 2^M entries each
 * and ping-pongs between them; which one holds the current vector after an
 * apply is reported by qsim_state_current().
 *
 * Errors: functions returning int return QSIM_OK (0) or a negative
 * qsim_status; constructors return NULL.  A human-readable message for the
 * last failure on the calling thread is returned by qsim_last_error().
 * Arguments are validated completely before any device work is enqueued: on
 * QSIM_ERR_INVALID or QSIM_ERR_RANGE nothing has run and the state is
 * unchanged.  After QSIM_ERR_DEVICE the state is poisoned and every later
 * call on it returns QSIM_ERR_DEVICE.  No C++ exception leaves the
 * library: host memory, threads or locks that cannot be had give
 * QSIM_ERR_NOMEM (nothing enqueued, the state unchanged), or
 * QSIM_ERR_DEVICE with the state poisoned if part of the call's device
 * work had already been enqueued.
 *
 * Threads: one state must not be used from two threads at once; distinct
 * states are independent.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { QSIM_C64 = 0, QSIM_C128 = 1 } qsim_dtype;

typedef enum {
    QSIM_OK = 0,
    QSIM_ERR_INVALID = -1, /* bad argument: M, dtype, step, NULL pointer    */
    QSIM_ERR_NOMEM = -2,   /* device or host allocation failed, or budget   */
    QSIM_ERR_DEVICE = -3,  /* a HIP call failed; the state is poisoned      */
    QSIM_ERR_RANGE = -4    /* offset + count beyond 2^M                     */
} qsim_status;

/* Kinds of step. */
typedef enum {
    QSIM_STEP_NOT = 0,   /* controlled NOT: the wiring-diagram step          */
    QSIM_STEP_PHASE = 1  /* controlled phase -1 (signed steps, Sec. 2(a))    */
} qsim_step_kind;

/* One step (16 bytes).  QSIM_STEP_NOT: a NOT on address bit `target` (the
 * paper's 'goto' minus one) that fires when every bit set in `control_mask`
 * is 1 in the row address (the paper's 'from', any number of them),
 * Sec. 2(b)-(g).  QSIM_STEP_PHASE: every row whose bit `target` and
 * control bits are all 1 is negated.  Valid iff kind is one of the two,
 * target < M, control_mask < 2^M and bit `target` of control_mask is 0. */
typedef struct {
    uint32_t target;
    uint32_t kind;
    uint64_t control_mask;
} qsim_step;

typedef struct qsim_state qsim_state;

/* Largest M accepted (entries are addressed with 64-bit integers; the
 * allocation itself fails first on a 288 GB device beyond M = 34 for
 * QSIM_C64 and M = 33 for QSIM_C128). */
#define QSIM_MAX_M 36u

/* Create a state of 2^M entries of `dtype` on the current HIP device:
 * allocates two device buffers of 2^M * elem bytes.  The state is the
 * paper's vector k1 of 2^M rows, one per address of M bits (Sec. 2(b)),
 * holding complex amplitudes of arbitrary magnitude and phase (Sec. 1).  The contents are
 * undefined until written (qsim_write_portion or through the pointer of
 * qsim_state_current()).  Returns NULL on bad M / dtype (QSIM_ERR_INVALID)
 * or allocation failure (QSIM_ERR_NOMEM). */
qsim_state *qsim_state_create(uint32_t M, qsim_dtype dtype);

/* Wrap two caller-owned device buffers of 2^M * elem bytes each (for example
 * torch tensors): the same 2^M-row vector as qsim_state_create (Sec. 1,
 * Sec. 2(b)) in memory the caller provides.  buf0 holds k1; buf1 is scratch.  Both must be 16-byte
 * aligned, must not overlap and must outlive the state.  NULL on error. */
qsim_state *qsim_state_wrap(uint32_t M, qsim_dtype dtype, void *buf0, void *buf1);

/* Release the state (and its buffers if it allocated them).  Waits for work
 * enqueued on the state to finish.  NULL is ignored.  (Resource management;
 * no passage of the paper.) */
void qsim_state_destroy(qsim_state *state);

/* Number of address bits M (Sec. 2(b)) and entry size in bytes of a state
 * (0 on NULL). */
uint32_t qsim_state_qubits(const qsim_state *state);
uint32_t qsim_state_elem_bytes(const qsim_state *state);

/* Device pointer to the buffer that holds the current vector (k1 before any
 * apply, k2 = U k1 after, Sec. 2(a)).  Valid until the next apply on the
 * state.  (Which of the two buffers holds it is a property of this
 * library's out-of-place passes; the paper keeps k1 and k2 as separate
 * arrays, Sec. 4.) */
const void *qsim_state_current(const qsim_state *state);

/* Copy `count` entries from host memory into rows [offset, offset+count) of
 * the current vector (the arbitrary initial magnitude and phase of Sec. 1).
 * Synchronous.  QSIM_ERR_RANGE if offset + count > 2^M. */
int qsim_write_portion(qsim_state *state, uint64_t offset, uint64_t count,
                       const void *host_src);

/* Set the current vector to the Kronecker product q_M (x) ... (x) q_1 of M
 * qubit pairs, computed on the device (the input calculated on the fly of
 * Appendix 1): entry i = q_M(bit M-1 of i) * ... * q_1(bit 0 of i).  The
 * product is taken from q_M down to q_1 in the entries' precision (float
 * for QSIM_C64, double for QSIM_C128), each complex product formed as
 * (ac - bd) + (ad + bc)i with every operation rounded separately, so the
 * result does not depend on the device (except the payload and sign of a
 * NaN that a product makes, which IEEE 754 leaves to the implementation).  `qubits` (host memory, read
 * before the call returns) holds 2M complex numbers of the entry type:
 * q_b(v) at index 2(b-1) + v.  Enqueued on hip_stream; one write of the
 * state, no read. */
int qsim_state_set_product(qsim_state *state, const void *qubits, void *hip_stream);

/* Apply the wiring diagram to the product state q_M (x) ... (x) q_1
 * (Appendix 1: the input calculated on the fly): current <- U_L ... U_1 k1
 * with k1 the vector qsim_state_set_product would write, whatever the
 * current vector holds.  The result is bit-identical to
 * qsim_state_set_product followed by qsim_apply_steps.  When the plan
 * starts with a tile pass of the one-tile-per-workgroup kernel with 32 rows
 * per thread (states above the single-workgroup size with the default
 * rows_per_thread), that pass forms each source tile from the qubits in LDS
 * and never reads the state: the input is neither written nor read in HBM.
 * Otherwise the product kernel runs first.  `qubits` as for
 * qsim_state_set_product; steps, L, stream and errors as for
 * qsim_apply_steps (L == 0 sets the product state). */
int qsim_apply_steps_product(qsim_state *state, const void *qubits, const qsim_step *steps,
                             uint64_t L, void *hip_stream);

/* Apply the wiring diagram: current <- U_L ... U_1 current, with steps[0]
 * acting first (Sec. 2(a), 2(h)).  `steps` is caller-owned and is read
 * before the call returns.  Work is enqueued on `hip_stream` (a
 * hipStream_t; NULL = the default stream) and the call returns without
 * waiting for it.  L == 0 is a no-op.  QSIM_ERR_INVALID on any invalid step
 * (target >= M, control >= M, target among its controls, unknown kind) or
 * steps == NULL with L > 0. */
int qsim_apply_steps(qsim_state *state, const qsim_step *steps, uint64_t L,
                     void *hip_stream);

/* Bytes of device scratch that qsim_apply_steps_noalloc may use: one array
 * of this size on each device the library runs on, held until the process
 * ends. */
#define QSIM_NOALLOC_SCRATCH_BYTES (64u << 20)

/* qsim_apply_steps for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and errors as qsim_apply_steps, with
 * the same kernels; the uploaded plan and the per-tile records of the
 * current pass live in the library's per-device scratch array of
 * QSIM_NOALLOC_SCRATCH_BYTES instead of buffers the state grows.  The call
 * makes no hipMalloc, hipFree, pinned host allocation or other device
 * allocation: the plan travels to the device in kernel arguments, so
 * `steps` may be freed on return and the call does not wait for the
 * device.  Every call on one device shares that device's scratch, whose
 * contents are whatever the last call left: calls on one stream are
 * ordered, but calls whose work may overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.
 * QSIM_ERR_NOMEM, with nothing enqueued, if the plan and one pass's tile
 * records need more than QSIM_NOALLOC_SCRATCH_BYTES (the largest states
 * with small tiles or very long passes).  Launches are not timed by
 * qsim_state_profile. */
int qsim_apply_steps_noalloc(qsim_state *state, const qsim_step *steps, uint64_t L,
                             void *hip_stream);

/* The row array x of a whole diagram of QSIM_STEP_NOT steps (a row array
 * holds no signs: phase steps are rejected with QSIM_ERR_INVALID)
 * (Sec. 2(h), Summary of Method): x(i)
 * is the row of k1 that lands in row i of k2 = U_L ... U_1 k1, so that
 * k2(i) = k1(x(i)) for every input (the information about the unitary
 * matrix that the Conclusions propose to keep).  Built on the device by
 * applying the diagram to the index vector (entry i = i) with the fused
 * path; x_dev (device memory, 2^M uint32) receives it.  1 <= M <= 32.
 * Allocates and frees a temporary state of 2 * 2^M * 8 bytes; returns when
 * x_dev is written. */
int qsim_rowmap_build(uint32_t M, const qsim_step *steps, uint64_t L,
                      uint32_t *x_dev, void *hip_stream);

/* current <- k1(x(i)) for the row array x_dev of qsim_rowmap_build (the
 * gather form k2(i) = k1(x(i)) of Sec. 2(b), end): the same result as
 * applying the diagram again, as one gather (a read of x, a read of the
 * state at the rows x names, a write of the state).  x_dev: 2^M uint32 on
 * the state's device, caller-owned; asynchronous on hip_stream.
 * QSIM_ERR_INVALID for a NULL x_dev or a state above M = 32, QSIM_ERR_DEVICE
 * (state poisoned) on a HIP error. */
int qsim_rowmap_apply(qsim_state *state, const uint32_t *x_dev, void *hip_stream);

/* Same result as qsim_apply_steps, computed the plain way: one in-place
 * kernel launch per step that interchanges every pair of rows the step
 * toggles, or negates the rows a phase step selects (the state is
 * recalculated after each step, Sec. 2(h)).  Consecutive NOT steps on one
 * target (up to 16) share one launch that interchanges a pair when an odd
 * number of their control conditions hold (the toggle parity of the
 * same-target shortcut, Sec. 2(i)).  A comparator for the fused path; not
 * faster. */
int qsim_apply_steps_plain(qsim_state *state, const qsim_step *steps,
                           uint64_t L, void *hip_stream);

/* Copy rows [offset, offset+count) of the current vector to host memory:
 * the contiguous row ranges, first row to last, in which the result is
 * handed on to post-processing (Abstract, Conclusions).  Waits for the work last enqueued on the state.
 * QSIM_ERR_RANGE if offset + count > 2^M. */
int qsim_read_portion(const qsim_state *state, uint64_t offset, uint64_t count,
                      void *host_dst);

/* Stream-ordered variant of qsim_read_portion (the same contiguous
 * portions, Abstract and Conclusions): enqueues the device-to-host copy on
 * `hip_stream` after the work already enqueued on it.  `host_dst` should be pinned
 * (hipHostMalloc) memory and must stay valid until the stream reaches the
 * copy. */
int qsim_read_portion_async(const qsim_state *state, uint64_t offset,
                            uint64_t count, void *host_dst, void *hip_stream);

/* Apply n independent wiring diagrams to n distinct states in one
 * persistent kernel launch (batched mode).  Each circuit is the operation
 * of qsim_apply_steps (Sec. 2(a), 2(h)); running many at once is this
 * library's use of the parts that may run simultaneously (Sec. 2(i),
 * Parallelism) across circuits, which the paper does not treat.  Circuit c applies
 * steps[c][0 .. Ls[c]-1] to states[c] exactly as qsim_apply_steps would;
 * the results are bit-identical to n separate calls.  The states may differ
 * in M but must share one dtype.  All circuits are validated before any
 * work is enqueued. */
int qsim_apply_batch(qsim_state *const *states, const qsim_step *const *steps,
                     const uint64_t *Ls, uint32_t n, void *hip_stream);

/* (No passage of the paper: status of the batched launches.)  Wait for
 * every qsim_apply_batch launch of the process still in flight and report whether all launches since the previous call completed
 * cleanly: QSIM_OK, or QSIM_ERR_DEVICE if a HIP error occurred or a tile's
 * wait for the previous pass of its circuit ran out in one of them (the
 * results of that batch are then invalid).  Batches may be enqueued back to
 * back without calling this in between: the library keeps two workspaces
 * and uploads one batch's plan while the previous batch runs. */
int qsim_batch_last_status(void);

/* Launch parameters of batched mode (no passage of the paper: how the
 * circuits of one launch are cut into queue items).  Zero in any field
 * selects the default. */
typedef struct {
    uint32_t tiles_per_item; /* tiles of one pass per queue item (1..256;
                                default 32): larger items mean fewer
                                completion handshakes, smaller ones more
                                workgroups on each pass                   */
    uint32_t tile_bits;      /* log2 entries per tile of the tiled circuits
                                (10..13; default 13 for QSIM_C64, 12 for
                                QSIM_C128); circuits with M <= tile_bits run
                                whole in one workgroup's LDS              */
    uint32_t circuit_tiles;  /* circuits whose passes have at most this many
                                tiles run every pass in one workgroup (one
                                queue item, no waits between passes);
                                default 64; 1 = none                      */
    uint32_t plan_search;    /* pass planning of each circuit: 1 = greedy
                                scan, 2 = with the mask climb (default:
                                fewer passes, more host time)             */
    uint32_t order;          /* queue order: 1 = pass level by pass level,
                                2 = critical path first (default): the host
                                simulates the resident workgroups taking
                                items and queues first the ready item with
                                the longest remaining chain of passes     */
    uint32_t from_cache;     /* output of qsim_batch_autotune: 1 when the
                                setting came from the tuning cache        */
    float best_ms;           /* output of qsim_batch_autotune: measured time
                                per batch of the chosen setting in a long
                                run of batches, the larger of the kernel's
                                device time and the host's enqueue time
                                (0 when taken from the cache)             */
    float default_ms;        /* the same for the defaults                  */
} qsim_batch_tuning;

/* Set (t != NULL) or reset (NULL) the batched-mode parameters used by
 * later qsim_apply_batch calls on states of `dtype`, or read them back.
 * Process-wide.  QSIM_ERR_INVALID on out-of-range values.  (Launch
 * parameters; no passage of the paper.) */
int qsim_batch_set_tuning(qsim_dtype dtype, const qsim_batch_tuning *t);
int qsim_batch_get_tuning(qsim_dtype dtype, qsim_batch_tuning *out);

/* Shorthands for the tiles_per_item field, for both dtypes (0 restores the
 * default).  QSIM_ERR_INVALID above 256.  (Launch parameters; no passage
 * of the paper.) */
int qsim_batch_set_tiles_per_item(uint32_t tiles);
uint32_t qsim_batch_tiles_per_item(void);

/* Choose the batched-mode parameters for a batch by measurement (Sec. 2(a):
 * each trial applies the batch and then the batch of reversed diagrams,
 * which undoes it, since every step matrix is its own inverse; the states'
 * contents are unchanged on return).  Starting from the defaults, one
 * parameter at a time takes each of its candidate values (queue order,
 * tile size, planning, whole-circuit cut-off, tiles per item) and keeps
 * the fastest, by the time per batch of a long run of batches (the host
 * plans each batch while the device runs the one before, so the larger of
 * the two); the result becomes the setting for the batch's dtype and is
 * copied to *out (may be NULL).  When the environment variable
 * QSIM_TUNING_CACHE names a file, the choice is looked up there first under
 * the key (device architecture, dtype, range of M, range of L rounded out
 * to powers of two) and, when measured, stored there (a JSON object).
 * Arguments as for qsim_apply_batch.  Synchronous. */
int qsim_batch_autotune(qsim_state *const *states, const qsim_step *const *steps,
                        const uint64_t *Ls, uint32_t n, void *hip_stream,
                        qsim_batch_tuning *out);

/* What the last qsim_apply_batch launch did (waits for it): circuits,
 * queue items, tiled passes (whole-in-LDS circuits count one pass each),
 * the algorithmic bytes (one read and one write of a circuit's state per
 * pass, summed), the kernel's device time from HIP events recorded on its
 * stream, and the parameters it ran with.  QSIM_ERR_INVALID if no batch
 * has run.  (Measurement; no passage of the paper.) */
typedef struct {
    uint32_t circuits;
    uint32_t items;
    uint32_t passes;
    uint32_t workgroups;       /* workgroups of the launch                  */
    uint64_t algorithmic_bytes;
    double kernel_ms;
    qsim_batch_tuning tuning;
} qsim_batch_info;

int qsim_batch_last_info(qsim_batch_info *out);

/* ---------------------------------------------------------------- serving */

/* A request server: wiring diagrams submitted over time run on one device
 * with their states kept in an HBM arena.  Requests are admitted in arrival
 * order (a later request may overtake one that does not fit yet, a bounded
 * number of times) whenever a slot and arena room are free, and admitted
 * requests run concurrently, each on its own stream: requests that arrive
 * while others are on the device join them (continuous batching).  Each
 * result is read back in contiguous ranges of portion_entries rows, first
 * row to last (Abstract, Conclusions), and folded into a 64-bit digest as it lands.  With fcfs = 1
 * one request runs at a time in arrival order (the plain comparator). */
typedef struct qsim_server qsim_server;

typedef struct {
    uint64_t hbm_budget_bytes; /* arena size (0 = 200e9 bytes)               */
    uint32_t max_slots;        /* requests on the device at once (0 = 4)      */
    uint32_t portion_entries;  /* rows per read-back portion (0 = 2^20)       */
    uint32_t fcfs;             /* 1 = one request at a time, arrival order    */
    uint32_t max_bypass;       /* times the queue head may be overtaken (0 = 64) */
    uint32_t digest;           /* 1 = fold every portion into the request's
                                  digest; k > 1 = only for requests whose id
                                  is a multiple of k; 0 = none              */
    uint32_t reserved;
} qsim_server_config;

typedef struct {
    int32_t status;       /* QSIM_OK or the error the request ended with    */
    int32_t done;         /* 1 once the last portion has been read back      */
    uint64_t t_submit_ns; /* steady-clock times of submission, admission    */
    uint64_t t_admit_ns;  /* and completion (last portion digested)          */
    uint64_t t_done_ns;
    uint64_t digest;      /* digest of the result's bytes in row order (0
                             unless the server digests this request): the
                             sum mod 2^64 over its 8-byte words w_j, j = 0,
                             1, ... from the first row, of
                             mix(w_j ^ mix(j + 0x9E3779B97F4A7C15)), then
                             mix(sum ^ mix(byte count)); mix is SplitMix64's
                             finaliser                                      */
    uint64_t bytes;       /* bytes read back                                 */
} qsim_request_info;

/* Create a server on the current device; allocates the arena.  (Serving
 * runtime around qsim_apply_steps; the paper's counterpart is only the
 * hand-off of results in portions, Abstract and Conclusions.)  cfg may be
 * NULL (defaults).  NULL on failure (no device, arena allocation failed,
 * max_slots > 64). */
qsim_server *qsim_server_create(const qsim_server_config *cfg);

/* Queue a request: M address bits, entry type, initial state host_k1 (2^M
 * entries, copied before the call returns; NULL = the alternating input
 * |S|(1, -1, 1, -1, ...) of Sec. 2(b) and Sec. 4) and the wiring diagram
 * steps[0..L-1] (copied).  Returns the request id (>= 0), QSIM_ERR_INVALID
 * for an invalid request, QSIM_ERR_NOMEM if its two buffers exceed the
 * whole arena.  Never blocks on the device. */
int64_t qsim_server_submit(qsim_server *server, uint32_t M, qsim_dtype dtype,
                           const void *host_k1, const qsim_step *steps,
                           uint64_t L);

/* Wait until every submitted request is done.  (No passage of the paper.) */
int qsim_server_drain(qsim_server *server);

/* (No passage of the paper.)  Status, timestamps and digest of request
 * `id` (QSIM_ERR_RANGE for an unknown id). */
int qsim_server_request_info(qsim_server *server, int64_t id,
                             qsim_request_info *out);

/* (No passage of the paper.)  Arena size and use, queued and running
 * request counts (any pointer may be NULL). */
int qsim_server_stats(qsim_server *server, uint64_t *arena_bytes,
                      uint64_t *arena_used, uint32_t *queued,
                      uint32_t *running);

/* Drain, stop the workers and free the arena.  NULL is ignored.  (No
 * passage of the paper.) */
void qsim_server_destroy(qsim_server *server);

/* ---------------------------------------------------------------- tuning */

/* Launch parameters of the fused path.  Zero in any field selects the
 * default for the state's dtype. */
typedef struct {
    uint32_t tile_bits;    /* log2 entries per LDS tile (12..14)           */
    uint32_t low_bits;     /* lowest address bits inside the tiles of the
                              first and the last pass (natural layout)      */
    uint32_t max_seg_steps;/* cap on steps per pass                         */
    uint32_t reorder;      /* 1 = exact reordering of commuting steps, 2 = off */
    uint32_t small_bits;   /* largest M run whole inside one workgroup      */
    uint32_t kernel_variant; /* tile kernel: 1 = one tile per workgroup,
                                2 = persistent workgroups with the next
                                tile's loads in flight, 3 = persistent with
                                loads two tiles ahead                       */
    uint32_t wg_per_cu;    /* persistent variant: workgroups per CU
                              (0 = as many as fit)                          */
    uint32_t outer_order;  /* order in which tiles are enumerated: 1 = the
                              lowest outside address bit varies fastest,
                              2 = the highest one does                      */
    uint32_t remap;        /* 1 = between passes, store the state with its
                              address bits permuted so that each pass's tile
                              bits are low physical bits; 2 = keep the
                              natural order throughout                      */
    uint32_t mid_low_bits; /* low address bits forced into the tiles of the
                              passes between the first and the last one    */
    uint32_t min_overlap;  /* tile bits each middle pass shares with the
                              previous pass (with remap: the length, as a
                              power of two, of the runs written between
                              passes)                                       */
    uint32_t rows_per_thread; /* tile rows per thread of the fused pass:
                              8, 16 or 32 (threads per tile = 2^tile_bits /
                              rows_per_thread, at most 1024)               */
    uint32_t plan_search;  /* 1 = off, 2 = climb: after the greedy scan
                              builds a pass, swap single tile bits for
                              outside bits while that admits more pending
                              steps (fewer passes, more host time); 3 =
                              climb + beam search over whole plans (several
                              candidate masks per pass, the plan with the
                              fewest passes, then the fewest tile pairs that
                              share less than a 128-byte line; tens of ms of
                              host time on up to 16 threads at M = 32,
                              L = 1000; diagrams with L x passes above 4e6
                              keep the climb's plan);
                              0 = by size: climb + beam from M = 30; below
                              it the greedy scan for QSIM_C64 and the climb
                              for QSIM_C128                                */
    uint32_t xcd_swizzle;  /* 1 = off, 2 = on (default): the one-tile-per-
                              workgroup kernel maps 64 consecutive tiles to
                              one XCD (workgroups are dealt to the 8 XCDs in
                              turn), so neighbouring tiles share an L2    */
    uint32_t product_stage;/* first pass of qsim_apply_steps_product: what
                              a workgroup forms in LDS.  1 = the whole
                              source tile; 2 = the partial products down to
                              address bit 1, each entry finished with one
                              complex product as it is stored; 3 = down to
                              bit 2, two products per entry (default: a
                              quarter of the LDS, so more workgroups share
                              a CU).  Same values whichever (Appendix 1). */
} qsim_tuning;

/* Set (tuning != NULL) or reset to defaults (NULL) the parameters used by
 * later applies on `state`.  QSIM_ERR_INVALID on out-of-range values.
 * (Launch parameters; the paper's only counterpart is the user-controlled
 * trade-off between processors and memory of the Conclusions.) */
int qsim_state_set_tuning(qsim_state *state, const qsim_tuning *tuning);

/* Apply the steps, in the order given, as a single fused pass through
 * tiles whose address bits are `tile_mask` (for callers that plan passes
 * themselves, and for measuring one pass).  Every NOT step must target a
 * bit of tile_mask or have no control in it (Sec. 2(i): steps processed
 * together; phase steps always qualify);
 * tile_mask must have 5..14 bits set (5..13 for QSIM_C128), all below bit
 * 32 and below M, and must contain bit 0 for QSIM_C64.  L may be 0: the pass
 * then moves every entry back to its own row.  QSIM_ERR_INVALID otherwise;
 * nothing runs on error. */
int qsim_apply_tile_pass(qsim_state *state, uint64_t tile_mask,
                         const qsim_step *steps, uint64_t L, void *hip_stream);

/* Choose the launch parameters of the fused path for this state and
 * diagram by measurement: every candidate (tile size, kernel shape, forced
 * low bits of the middle passes, planner search) applies the diagram once
 * on the device,
 * timed with events, then its reverse, which undoes it (each step matrix is
 * its own inverse, Sec. 2(a)); the state's contents are unchanged on
 * return.  The fastest candidate becomes the state's tuning and is copied
 * to *out (may be NULL).  States small enough for one workgroup have
 * nothing to choose.  When the environment variable QSIM_TUNING_CACHE
 * names a file, the choice is looked up there first under (device
 * architecture, dtype, M, band of L between powers of two) and, if found
 * and valid, taken without measuring; a measured choice is stored there
 * (the file is shared with qsim_batch_autotune).  Synchronous. */
int qsim_autotune(qsim_state *state, const qsim_step *steps, uint64_t L,
                  void *hip_stream, qsim_tuning *out);

/* ---------------------------------------------------------------- planning */

/* Describe the pass plan the fused path would use for a diagram (host
 * only; no device work).  The steps are split into passes; each pass reads
 * and writes the whole state once through tiles of 2^tile_bits entries whose
 * address bits are the pass's tile mask.  Within a pass a step either
 * targets a tile bit or has no control among the tile bits (Sec. 2(i):
 * which steps may be processed together).  Steps may be reordered, but only
 * past steps they commute with (neither target is a control of the other).
 *
 * Outputs: *n_passes; pass_mask[p] and pass_len[p] for p < min(n_passes,
 * cap) (tile mask and number of steps of pass p); order[0..L-1] = the
 * original indices in execution order (passes back to back).  Any output
 * pointer may be NULL.  tuning may be NULL (defaults). */
int qsim_plan_describe(uint32_t M, qsim_dtype dtype, const qsim_step *steps,
                       uint64_t L, const qsim_tuning *tuning,
                       uint32_t *n_passes, uint64_t *pass_mask,
                       uint32_t *pass_len, uint32_t cap, uint32_t *order);

/* ---------------------------------------------------------------- timing */

/* (Measurement; no passage of the paper.)  Per-kernel device time of the
 * applies on one state, taken with HIP events
 * recorded on the stream of each launch (a few microseconds of gap per
 * launch while enabled). */
typedef struct {
    uint64_t tile_launches;   /* fused tile passes                          */
    double tile_ms;           /* summed device time of those launches       */
    uint64_t tile_bytes;      /* algorithmic HBM bytes: 2 * 2^M * elem each */
    uint64_t map_launches;    /* tile-map launches                          */
    double map_ms;
    uint64_t other_launches;  /* small-state, direct and plain-step launches */
    double other_ms;
} qsim_profile;

/* enable = 1: clear the counters and time every later launch on `state`;
 * enable = 0: stop timing.  (Measurement; no passage of the paper.) */
int qsim_state_profile(qsim_state *state, int enable);

/* Wait for the timed launches to finish and report their totals.
 * (Measurement; no passage of the paper.) */
int qsim_state_profile_read(qsim_state *state, qsim_profile *out);

/* ---------------------------------------------------------------- misc */

/* Stream copy of `bytes` bytes (a multiple of 16) from src to dst, device
 * pointers, 16-byte aligned: the achievable-bandwidth reference that the
 * fused path's traffic is compared against.  (Measurement; no passage of
 * the paper.) */
int qsim_copy_bytes(void *dst, const void *src, uint64_t bytes, void *hip_stream);

/* Message describing the last failure on the calling thread ("" if none).
 * (Error reporting; no passage of the paper.) */
const char *qsim_last_error(void);

/* Library version string.  (No passage of the paper.) */
const char *qsim_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QSIM_H */
