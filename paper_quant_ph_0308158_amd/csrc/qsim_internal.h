// Internal declarations shared by the host side (planner, C ABI) and the HIP
// kernels of libqsim.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "planner.h"

namespace qsim {

// Entries per LDS tile are 2^(tb + eb): every thread of a tile workgroup owns
// 2^eb entries (eb <= 5: one bit lane of each 32-bit bit-plane word per
// entry), so a workgroup of 2^tb threads covers one tile.
constexpr int kPlanes = 16;        // bit-plane registers per thread (tile bits <= 15)
constexpr int kMaxTileBits = 14;   // 2^14 entries * 8 B = 128 KiB of LDS
constexpr int kMaxOuterBits = 48;
constexpr uint32_t kMaxQubits = 36;    // largest M of a state

// Bit-plane that carries the sign of each row during the inner walk: tile
// indices have at most kMaxTileBits bits, so plane 15 is free.  A phase
// step is an inner step that targets it.
constexpr uint32_t kSignPlane = 15;

// A step as the tile-map kernel sees it (16 bytes).  `cm` is the part of the
// control mask outside the tile; `tbit` is the address bit of the target;
// `inner` is 1 when the target is a tile bit (the step moves entries inside
// a tile and the tile-map only records whether its outside controls hold)
// and for every phase step (outside part of its mask, target included).
// In the direct per-row walk `inner` = 1 marks a phase step and `cm` is
// its whole mask.
struct TmStep {
    uint64_t cm;
    uint32_t tbit;
    uint32_t inner;
};

// Inner steps are packed into 32 bits: tile-index bit of the target in bits
// 0..3, tile-index control mask in bits 16..31.
__host__ __device__ inline uint32_t pack_inner(uint32_t tj, uint32_t icm) {
    return (tj & 15u) | (icm << 16);
}

// Arguments of one pass of the fused tile kernel (passed by value).
//
// Between passes the state may be stored with its address bits permuted (a
// layout): logical bit b of a row address lives at physical bit lam(b).  A
// pass reads its source tiles in one layout and writes its output tiles in
// the next, so each side has its own physical positions for the tile-index
// bits (pos_src / pos_dst) and its own offset tables.  The walk itself works
// on logical tile indices and does not see layouts.
struct TileArgs {
    const uint32_t *inner;  // packed inner steps in reverse execution order
    const uint32_t *rec;    // per-tile records from the tile-map kernel (or null)
    uint32_t n_inner;
    uint32_t rec_words;     // 2 + ceil(n_inner / 32)
    uint32_t tb;            // log2(threads per workgroup); tile bits = tb + eb
    uint32_t n_out;         // outer bits (M - tile bits)
    uint32_t eb;            // log2(tile rows per thread): 3, 4 or 5
    uint32_t sign;          // 1 when the pass has phase steps (sign plane in use)
    uint32_t xcd;           // log2 of the consecutive tiles run on one XCD (0: none)
    uint32_t pad;
    uint32_t off_r_src[32]; // element offset of the tile-index bits above the thread bits, per r (read)
    uint32_t off_r_dst[32]; // same for the write layout
    uint8_t pos_src[16];    // physical bit of tile-index bit b in the read layout
    uint8_t pos_dst[16];    // physical bit of tile-index bit b in the write layout
    uint8_t out_dst[kMaxOuterBits];  // physical bit (write layout) of outer-index bit q
};

// First pass of a diagram applied to a product state (Appendix 1): the
// source tile is formed from the qubits in LDS instead of read from HBM.
struct ProductTileArgs {
    const void *q;          // q_b(v) at complex index 2(b-1) + v, in the entries' precision
    uint32_t M;
    uint32_t cut;           // partials staged down to just above address bit cut - 1 (0: whole tile)
    uint8_t bit[16];        // logical address bits of the tile, lowest first
    uint8_t tix[16];        // tile-index bit of bit[i]
};

struct TileMapArgs {
    const TmStep *steps;    // all steps of the pass in reverse execution order
    uint32_t *rec;
    uint64_t n_tiles;
    uint32_t n_steps;
    uint32_t rec_words;
    uint32_t n_out;
    uint32_t pad;
    uint8_t out_pos[kMaxOuterBits];  // logical bit of outer-index bit q
    uint8_t lam_src[64];             // physical bit of logical bit b in the read layout
};

// Batched mode: many circuits in one persistent launch.  Work items are
// read from a queue in order; each names a whole small circuit, a whole
// mid-size circuit (all its passes in one workgroup) or a block of tiles of
// one pass.  A tile of pass p of a circuit waits until every tile of pass
// p-1 of that circuit is done.  Tile records are formed in LDS by the item
// that uses them.
struct BatchPass {
    TileArgs ta;            // inner pointer filled in (rec unused)
    TileMapArgs tm;         // steps pointer filled in (rec unused)
    const void *src;
    void *dst;
    uint64_t n_tiles;
    uint32_t circuit;       // index of the circuit's completion counter
    uint32_t level;         // pass index within its circuit
};

struct BatchSmall {
    TileArgs ta;            // whole state as one tile (identity positions)
    const void *src;
    void *dst;
    const TmStep *steps_rev; // direct walk for states of fewer than 32 rows
    uint32_t L;
    uint32_t M;
    uint32_t direct;
    uint32_t pad;
};

enum : uint32_t { kItemSmall = 1, kItemTile = 2, kItemCircuit = 3 };

__host__ __device__ inline uint64_t batch_item(uint32_t kind, uint32_t index, uint32_t sub) {
    return ((uint64_t)kind << 62) | ((uint64_t)(index & 0x3FFFFFFFu) << 32) | sub;
}

// Counter words of a batched launch: [0] queue head, [1] reserved, [2]
// error flag (a dependency wait ran out), [3] reserved, [4 + c] finished
// tiles of circuit c.
constexpr uint32_t kBatchCtrHeader = 4;
constexpr uint32_t kBatchTilesMax = 256;

}  // namespace qsim

struct qsim_state;

namespace qsim {

// Point an existing wrapped state at new buffers (another M or dtype),
// keeping its plan, record and staging buffers.  Waits for the state's
// earlier work.  For the serving workers, which reuse one state per slot.
int state_rebind(qsim_state *s, uint32_t M, int dtype, void *buf0, void *buf1);

// Called in a catch (...) of an exported function: the error code for the
// exception being handled (QSIM_ERR_NOMEM for host memory, threads or
// locks that could not be had, QSIM_ERR_INVALID for any other, and
// QSIM_ERR_DEVICE if `s` was poisoned part-way through the call), with its
// message stored for qsim_last_error.  No exception crosses the C boundary.
int host_exception(qsim_state *s) noexcept;

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_direct(uint32_t elem, const void *src, void *dst, uint64_t n,
                         const TmStep *steps_rev, uint32_t L, hipStream_t st);
hipError_t launch_small(uint32_t elem, const void *src, void *dst, uint32_t M,
                        const TileArgs &a, hipStream_t st);
hipError_t launch_tilemap(const TileMapArgs &a, hipStream_t st);
hipError_t launch_tile(uint32_t elem, const void *src, void *dst, uint64_t n_tiles, const TileArgs &a,
                       uint32_t variant, uint32_t wg_per_cu, hipStream_t st);
hipError_t launch_plain_step(uint32_t elem, void *buf, uint32_t M, uint32_t target,
                             uint64_t cmask, hipStream_t st);
hipError_t launch_plain_phase(uint32_t elem, void *buf, uint32_t M, uint64_t mask, hipStream_t st);
// A run of k (2..kPlainRunMax) NOT steps on one target as one in-place launch.
constexpr uint32_t kPlainRunMax = 16;
hipError_t launch_plain_run(uint32_t elem, void *buf, uint32_t M, uint32_t target, const uint64_t *cmasks,
                            uint32_t k, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t st);
// Copy `bytes` (a multiple of 4) of host memory to device memory `dst` in
// stream order, carried in kernel arguments of kPutChunkBytes each: no
// staging buffer, and `src` may be reused as soon as the call returns.
constexpr uint32_t kPutChunkBytes = 2048;
hipError_t launch_put(void *dst, const void *src, size_t bytes, hipStream_t st);

hipError_t launch_product(uint32_t elem, void *out, uint32_t M, const void *qubits, hipStream_t st);
// One tile per workgroup, 32 rows per thread (a.eb = 5), natural read layout.
hipError_t launch_tile_product(uint32_t elem, void *dst, uint64_t n_tiles, const TileArgs &a,
                               const ProductTileArgs &pa, hipStream_t st);
hipError_t launch_iota(uint64_t *out, uint64_t n, hipStream_t st);
hipError_t launch_narrow(const uint64_t *in, uint32_t *out, uint64_t n, hipStream_t st);
hipError_t launch_gather(uint32_t elem, const void *src, void *dst, const uint32_t *x, uint64_t n, hipStream_t st);
// Workgroups of a batched launch (those resident at once): the workers the
// host's queue ordering plans for.  lds = dynamic LDS bytes per workgroup.
hipError_t batch_grid(uint32_t elem, uint32_t tb, bool sign, size_t lds, uint64_t *grid);
hipError_t launch_batch(uint32_t elem, uint32_t tb, bool sign, const BatchPass *passes, const BatchSmall *smalls,
                        const uint64_t *items, uint32_t n_items, uint32_t *counters, uint32_t spin_limit,
                        uint32_t tiles_per_item, uint32_t rec_stride, size_t lds, hipStream_t st);

}  // namespace qsim
