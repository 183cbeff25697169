// HIP kernels of libqsim for gfx950 (MI355X).
//
// The state is a vector of 2^M opaque entries (8 or 16 bytes).  A wiring
// diagram step s (target bit t, control mask C) is the symmetric
// permutation y_s(i) = i XOR 2^t when all bits of C are set in i, else i
// (Sec. 2(b)-(g)); k2 = U_L ... U_1 k1 gives k2(i) = k1(x(i)) with
// x = y_1 o y_2 o ... o y_L (the row array x(i) of Sec. 2(h), formed here per
// output row instead of as a 2^M-entry array).  Every kernel below moves
// entries only as integers.
//
// Fused tile pass (k_tile): a pass owns a set I of tile address bits.  Every
// step of the pass either targets a bit of I (inner step) or has no control
// in I (outer step), so the entries of one output tile (fixed outer bits)
// all come from one source tile.  Per tile:
//   * the tile-map kernel (k_tilemap) walks the pass's steps backwards on the
//     tile's outer address: outer steps flip it, inner steps record whether
//     their outside controls hold (one bit each);
//   * the source tile is read from HBM with coalesced 16-byte loads and
//     staged in LDS;
//   * each thread walks the inner steps backwards for its 32 tile rows at
//     once: the rows' tile indices are held as 16 bit-planes (plane b holds
//     bit b of 32 indices), so a step is planes[t] ^= AND of planes[c]; the
//     plane index is uniform, so it is a register-indexed move, not memory;
//   * the planes are transposed back to 16-bit indices, entries are gathered
//     from LDS and stored to the output tile with coalesced 16-byte stores.
// One pass therefore costs one read and one write of the state.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "qsim_internal.h"

namespace qsim {
namespace {

typedef uint4 vec16;

__device__ __forceinline__ vec16 ld_nt(const vec16 *p) {
    vec16 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    v.z = __builtin_nontemporal_load(&p->z);
    v.w = __builtin_nontemporal_load(&p->w);
    return v;
}

__device__ __forceinline__ void st_nt(vec16 *p, const vec16 &v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
}

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Bit q of the 32 lane positions p = 0..31 of a plane word.
__device__ __forceinline__ uint32_t lane_pattern(uint32_t q) {
    switch (q) {
        case 0: return 0xAAAAAAAAu;
        case 1: return 0xCCCCCCCCu;
        case 2: return 0xF0F0F0F0u;
        case 3: return 0xFF00FF00u;
        default: return 0xFFFF0000u;
    }
}

// Two interleaved 16x16 bit-matrix transposes: afterwards the low half of
// w[q] holds, in bit b, what bit q of w[b] held, and the high half of w[q]
// holds in bit 16+b what bit 16+q of w[b] held.
__device__ __forceinline__ void transpose_planes(uint32_t (&w)[kPlanes]) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (!(r & 8)) { uint32_t t = ((w[r] >> 8) ^ w[r + 8]) & 0x00FF00FFu; w[r + 8] ^= t; w[r] ^= t << 8; }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (!(r & 4)) { uint32_t t = ((w[r] >> 4) ^ w[r + 4]) & 0x0F0F0F0Fu; w[r + 4] ^= t; w[r] ^= t << 4; }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (!(r & 2)) { uint32_t t = ((w[r] >> 2) ^ w[r + 2]) & 0x33333333u; w[r + 2] ^= t; w[r] ^= t << 2; }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (!(r & 1)) { uint32_t t = ((w[r] >> 1) ^ w[r + 1]) & 0x55555555u; w[r + 1] ^= t; w[r] ^= t << 1; }
}

// A thread owns E = 2^EB tile rows (EB = 3, 4 or 5), held in
// VPT = E / (16 / ELEM) 16-byte vectors.  Tile index of lane position
// p < E of the calling thread (for 8-byte entries vector r holds positions
// p = 2r, 2r+1, adjacent rows; for 16-byte entries vector r holds p = r):
//   8 B : j = (p & 1) | tid << 1 | (p >> 1) << (1 + tb)
//   16 B: j = tid | p << tb
// where 2^tb is the number of threads; the tile has tb + EB bits.
template <int ELEM, int EB>
struct Shape {
    static constexpr uint32_t LO = (ELEM == 8) ? 1u : 0u;
    static constexpr uint32_t E = 1u << EB;
    static constexpr uint32_t VPT = E >> LO;   // 16-byte vectors per thread
    static constexpr uint32_t EPV = 16u / ELEM;
};

template <int ELEM, int EB>
using TileVecs = vec16[Shape<ELEM, EB>::VPT];

template <int ELEM, int EB>
__device__ __forceinline__ void init_planes(uint32_t (&w)[kPlanes], uint32_t tid, uint32_t tb) {
    constexpr uint32_t LO = Shape<ELEM, EB>::LO;
    const uint32_t K = tb + EB;
#pragma unroll
    for (uint32_t b = 0; b < (uint32_t)kPlanes; ++b) {
        uint32_t v;
        if (b < LO) v = lane_pattern(b);
        else if (b < LO + tb) v = ((tid >> (b - LO)) & 1u) ? 0xFFFFFFFFu : 0u;
        else if (b < K) v = lane_pattern(b - tb);
        else v = 0u;
        w[b] = v;
    }
}

// Walk the inner steps (reverse execution order) on the bit-planes.  With
// FLAGS the bit i of the tile record says whether inner step i's outside
// controls hold for this tile; without, every step's controls lie inside.
// Steps are fetched eight at a time with one scalar load (the step array is
// padded to a multiple of eight entries).
__device__ __forceinline__ void apply_inner(uint32_t (&w)[kPlanes], uint32_t d) {
    uint32_t m = d >> 16;
    uint32_t x = 0xFFFFFFFFu;
    while (m) {
        const uint32_t c = (uint32_t)__builtin_ctz(m);
        m &= m - 1u;
        x &= w[c];
    }
    w[d & 15u] ^= x;
}

template <bool FLAGS>
__device__ __forceinline__ void walk_inner(uint32_t (&w)[kPlanes], const uint32_t *__restrict__ inner,
                                           uint32_t n_inner, const uint32_t *__restrict__ flags) {
    for (uint32_t i0 = 0; i0 < n_inner; i0 += 8u) {
        uint32_t d[8];
#pragma unroll
        for (uint32_t j = 0; j < 8u; ++j) d[j] = uni(inner[i0 + j]);
        uint32_t fb;
        if (FLAGS) {
            fb = uni(flags[i0 >> 5]) >> (i0 & 31u);
        } else {
            const uint32_t rem = n_inner - i0;
            fb = rem >= 8u ? 0xFFu : ((1u << rem) - 1u);
        }
#pragma unroll
        for (uint32_t j = 0; j < 8u; ++j)
            if ((fb >> j) & 1u) apply_inner(w, d[j]);
    }
}

__device__ __forceinline__ uint32_t src_of(const uint32_t (&w)[kPlanes], uint32_t p) {
    return (w[p & 15u] >> ((p >> 4) * 16u)) & 0xFFFFu;
}

// Element offset of the thread bits of the tile index, for the physical
// positions `pos` of the tile-index bits.
template <int ELEM>
__device__ __forceinline__ uint32_t thread_offset(const uint8_t *pos, uint32_t tb, uint32_t tid) {
    constexpr uint32_t LO = (ELEM == 8) ? 1u : 0u;
    uint32_t off_t = 0;
    for (uint32_t b = 0; b < tb; ++b)
        if ((tid >> b) & 1u) off_t |= 1u << pos[LO + b];
    return off_t;
}

// Physical address (write layout) of the outer bits of output tile `tile`.
__device__ __forceinline__ uint64_t outer_address(const TileArgs &a, uint64_t tile) {
    uint64_t base = 0;
    for (uint32_t q = 0; q < a.n_out; ++q)
        if ((tile >> q) & 1u) base |= 1ull << a.out_dst[q];
    return base;
}

template <int ELEM, int EB>
__device__ __forceinline__ void load_tile(TileVecs<ELEM, EB> &v, const vec16 *__restrict__ src,
                                          uint64_t base, const TileArgs &a) {
#pragma unroll
    for (uint32_t r = 0; r < Shape<ELEM, EB>::VPT; ++r)
        v[r] = ld_nt(src + (base + a.off_r_src[r]) / Shape<ELEM, EB>::EPV);
}

// Source tile index of each of the calling thread's output positions, as
// bit-planes transposed to 16-bit indices (see src_of).
template <int ELEM, int EB, bool FLAGS>
__device__ __forceinline__ void tile_sources(uint32_t (&w)[kPlanes], const TileArgs &a,
                                             const uint32_t *__restrict__ flags) {
    init_planes<ELEM, EB>(w, threadIdx.x, a.tb);
    walk_inner<FLAGS>(w, a.inner, a.n_inner, flags);
    transpose_planes(w);
}

template <int ELEM, int EB>
__device__ __forceinline__ void tile_stage(const TileVecs<ELEM, EB> &v, uint32_t tb, vec16 *lds) {
#pragma unroll
    for (uint32_t r = 0; r < Shape<ELEM, EB>::VPT; ++r) lds[threadIdx.x | (r << tb)] = v[r];
}

// Sign of a transposed source index: bit kSignPlane (set by the phase
// steps of the pass) moved to bit 31, the sign bit of a float32 word and of
// the high word of a float64.
__device__ __forceinline__ uint32_t sign_word(uint32_t v) { return (v >> kSignPlane) << 31; }

// Gather the calling thread's output entries from the staged source tile
// and store them with 16-byte stores.  With phase steps in the pass, bit
// kSignPlane of each source index says whether the entry is negated: both
// its parts get their sign bit flipped.  SIGN is a template parameter so
// that passes without phase steps run code with no trace of it.
template <int ELEM, int EB, bool SIGN>
__device__ __forceinline__ void tile_emit(const uint32_t (&w)[kPlanes], vec16 *__restrict__ dst, uint64_t dst_base,
                                          const TileArgs &a, const vec16 *lds) {
    constexpr uint32_t VPT = Shape<ELEM, EB>::VPT;
    constexpr uint32_t EPV = Shape<ELEM, EB>::EPV;
    constexpr uint32_t kIndex = (1u << kSignPlane) - 1u;
    if constexpr (SIGN) {
        if (ELEM == 8) {
            const uint2 *l2 = reinterpret_cast<const uint2 *>(lds);
#pragma unroll
            for (uint32_t r = 0; r < VPT; ++r) {
                const uint32_t v0 = src_of(w, 2u * r), v1 = src_of(w, 2u * r + 1u);
                const uint2 e0 = l2[v0 & kIndex];
                const uint2 e1 = l2[v1 & kIndex];
                const uint32_t m0 = sign_word(v0), m1 = sign_word(v1);
                st_nt(dst + (dst_base + a.off_r_dst[r]) / EPV, make_uint4(e0.x ^ m0, e0.y ^ m0, e1.x ^ m1, e1.y ^ m1));
            }
        } else {
#pragma unroll
            for (uint32_t r = 0; r < VPT; ++r) {
                const uint32_t v0 = src_of(w, r);
                const vec16 e0 = lds[v0 & kIndex];
                const uint32_t m0 = sign_word(v0);
                st_nt(dst + (dst_base + a.off_r_dst[r]) / EPV, make_uint4(e0.x, e0.y ^ m0, e0.z, e0.w ^ m0));
            }
        }
        return;
    }
    if (ELEM == 8) {
        const uint2 *l2 = reinterpret_cast<const uint2 *>(lds);
#pragma unroll
        for (uint32_t r = 0; r < VPT; ++r) {
            const uint2 e0 = l2[src_of(w, 2u * r)];
            const uint2 e1 = l2[src_of(w, 2u * r + 1u)];
            st_nt(dst + (dst_base + a.off_r_dst[r]) / EPV, make_uint4(e0.x, e0.y, e1.x, e1.y));
        }
    } else {
#pragma unroll
        for (uint32_t r = 0; r < VPT; ++r) {
            const vec16 e0 = lds[src_of(w, r)];
            st_nt(dst + (dst_base + a.off_r_dst[r]) / EPV, e0);
        }
    }
}

// Walk, stage the loaded tile in LDS, gather and store one output tile.
// `v` holds the source tile's vectors on entry; when `next_base` is not
// ~0 the loads of the next source tile are issued into `v` as soon as the
// current one is in LDS, so they overlap the gather, the stores and the
// next tile's walk.
template <int ELEM, int EB, bool FLAGS, bool SIGN>
__device__ __forceinline__ void tile_step(TileVecs<ELEM, EB> &v, const vec16 *__restrict__ src,
                                          vec16 *__restrict__ dst, uint64_t dst_base, uint64_t next_base,
                                          const TileArgs &a, const uint32_t *__restrict__ flags, vec16 *lds) {
    uint32_t w[kPlanes];
    tile_sources<ELEM, EB, FLAGS>(w, a, flags);
    tile_stage<ELEM, EB>(v, a.tb, lds);
    __syncthreads();
    if (next_base != ~0ull) load_tile<ELEM, EB>(v, src, next_base, a);
    tile_emit<ELEM, EB, SIGN>(w, dst, dst_base, a, lds);
}

// Tile of workgroup b when consecutive workgroups go to the 8 XCDs in turn:
// 2^g consecutive tiles run on one XCD, so tiles that write parts of the
// same lines share that XCD's L2.  g = 0: tile b.
__device__ __forceinline__ uint64_t xcd_tile(uint64_t b, uint32_t g) {
    if (!g) return b;
    const uint64_t lo = (b >> 3) & ((1ull << g) - 1ull);
    return lo | ((b & 7ull) << g) | ((b >> (3 + g)) << (g + 3));
}

__device__ __forceinline__ uint64_t rec_base(const uint32_t *rec) {
    return (uint64_t)uni(rec[0]) | ((uint64_t)uni(rec[1]) << 32);
}

// Fused tile pass.  DEPTH = 0: one tile per workgroup.  DEPTH >= 1: a grid
// sized to the resident workgroups walks tiles blockIdx.x, blockIdx.x +
// gridDim.x, ...; the loads of each tile are issued DEPTH tiles ahead, into
// one of DEPTH register buffers, so they overlap the gathers, stores and
// walks of the tiles in between.
// Most threads a tile workgroup can have: tiles hold at most 2^14 8-byte or
// 2^13 16-byte entries, 2^EB per thread.  Bounding a kernel by its true
// workgroup size lets the compiler give each thread the registers that
// size leaves (a 256-thread workgroup of 16-byte entries has a whole SIMD's
// register file per wave).
template <int ELEM, int EB>
constexpr int tile_threads_max() {
    return std::min(1024, 1 << ((ELEM == 8 ? kMaxTileBits : kMaxTileBits - 1) - EB));
}

template <int ELEM, int DEPTH, int EB, bool SIGN>
__global__ void __launch_bounds__((tile_threads_max<ELEM, EB>())) k_tile(const vec16 *__restrict__ src,
                                                              vec16 *__restrict__ dst, TileArgs a,
                                                              uint64_t n_tiles) {
    extern __shared__ vec16 lds[];
    constexpr uint32_t VPT = Shape<ELEM, EB>::VPT;
    constexpr int NB = DEPTH > 0 ? DEPTH : 1;
    const uint32_t off_src = thread_offset<ELEM>(a.pos_src, a.tb, threadIdx.x);
    const uint32_t off_dst = thread_offset<ELEM>(a.pos_dst, a.tb, threadIdx.x);
    // Workgroup b takes sequence numbers q = b, b + stride, ...; tile
    // xcd_tile(q) is processed for q.  One tile per workgroup: runs of
    // 2^a.xcd consecutive tiles go to one XCD.  Persistent workgroups keep
    // tile q (the same mapping made them slower: 66.6 against 68.7 % of
    // peak per pass for 16-byte entries at M = 26).
    const uint64_t stride = DEPTH > 0 ? gridDim.x : n_tiles;
    const uint64_t q0 = blockIdx.x;
    const uint32_t g = DEPTH > 0 ? 0u : a.xcd;
    vec16 v[NB][VPT];
#pragma unroll
    for (int d = 0; d < NB; ++d) {
        const uint64_t q = q0 + (uint64_t)d * stride;
        if (q < n_tiles)
            load_tile<ELEM, EB>(v[d], src, rec_base(a.rec + xcd_tile(q, g) * a.rec_words) + off_src, a);
    }
    for (uint64_t first = q0;; first += (uint64_t)NB * stride) {
#pragma unroll
        for (int d = 0; d < NB; ++d) {
            const uint64_t q = first + (uint64_t)d * stride;
            if (q >= n_tiles) return;   // uniform over the workgroup
            const uint64_t tile = xcd_tile(q, g);
            const uint64_t next = q + (uint64_t)NB * stride;
            const uint64_t next_base =
                (DEPTH > 0 && next < n_tiles) ? rec_base(a.rec + next * a.rec_words) + off_src
                                              : ~0ull;
            tile_step<ELEM, EB, true, SIGN>(v[d], src, dst, outer_address(a, tile) + off_dst, next_base, a,
                                            a.rec + tile * a.rec_words + 2, lds);
            __syncthreads();
        }
    }
}

// Whole state in one workgroup's LDS: one tile, every step is inner.
template <int ELEM, bool SIGN>
__global__ void __launch_bounds__(512) k_small(const vec16 *__restrict__ src, vec16 *__restrict__ dst,
                                               TileArgs a) {
    extern __shared__ vec16 lds[];
    vec16 v[Shape<ELEM, 5>::VPT];
    load_tile<ELEM, 5>(v, src, thread_offset<ELEM>(a.pos_src, a.tb, threadIdx.x), a);
    tile_step<ELEM, 5, false, SIGN>(v, src, dst, thread_offset<ELEM>(a.pos_dst, a.tb, threadIdx.x), ~0ull, a,
                                    nullptr, lds);
}

// Per-tile record of a pass: source tile address and the outside-control
// flags of the inner steps, from a backward walk of the outer address.
// Written to `rec` (a.rec_words words).
__device__ __forceinline__ void tilemap_record(const TileMapArgs &a, uint64_t tile, uint32_t *rec) {
    uint64_t A = 0;
    for (uint32_t q = 0; q < a.n_out; ++q)
        if ((tile >> q) & 1u) A |= 1ull << a.out_pos[q];
    uint32_t word = 0, k = 0;
    // A is the logical outer address; the record holds its physical
    // address in the layout the pass reads.
    for (uint32_t s = 0; s < a.n_steps; ++s) {
        const uint64_t cm = ((uint64_t)uni((uint32_t)(a.steps[s].cm >> 32)) << 32) |
                            uni((uint32_t)a.steps[s].cm);
        const uint32_t tbit = uni(a.steps[s].tbit);
        const uint32_t inner = uni(a.steps[s].inner);
        const bool cond = (A & cm) == cm;
        if (inner) {
            word |= (cond ? 1u : 0u) << (k & 31u);
            ++k;
            if ((k & 31u) == 0u) { rec[2 + (k >> 5) - 1] = word; word = 0; }
        } else if (cond) {
            A ^= 1ull << tbit;
        }
    }
    if (k & 31u) rec[2 + (k >> 5)] = word;
    uint64_t P = 0;
    while (A) {
        const uint32_t b = (uint32_t)__builtin_ctzll(A);
        A &= A - 1;
        P |= 1ull << a.lam_src[b];
    }
    rec[0] = (uint32_t)P;
    rec[1] = (uint32_t)(P >> 32);
}

__device__ __forceinline__ void tilemap_one(const TileMapArgs &a, uint64_t tile) {
    tilemap_record(a, tile, a.rec + tile * a.rec_words);
}

__global__ void __launch_bounds__(256) k_tilemap(TileMapArgs a) {
    const uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile < a.n_tiles) tilemap_one(a, tile);
}

// One row of the direct gather: walk row i backwards through every step (a
// NOT step moves it, a phase step flips its sign when all its bits are 1
// at that point) and copy the entry it lands on, negated if the sign is
// odd.
template <int ELEM>
__device__ __forceinline__ void direct_row(const void *src, void *dst, uint64_t i,
                                           const TmStep *__restrict__ steps_rev, uint32_t L) {
    uint64_t x = i;
    uint32_t neg = 0;
    for (uint32_t s = 0; s < L; ++s) {
        const uint64_t cm = steps_rev[s].cm;
        const bool hit = (x & cm) == cm;
        if (steps_rev[s].inner) neg ^= hit ? 1u : 0u;
        else if (hit) x ^= 1ull << steps_rev[s].tbit;
    }
    const uint32_t m = neg << 31;
    if (ELEM == 8) {
        const uint2 e = reinterpret_cast<const uint2 *>(src)[x];
        reinterpret_cast<uint2 *>(dst)[i] = make_uint2(e.x ^ m, e.y ^ m);
    } else {
        const vec16 e = reinterpret_cast<const vec16 *>(src)[x];
        reinterpret_cast<vec16 *>(dst)[i] = make_uint4(e.x, e.y ^ m, e.z, e.w ^ m);
    }
}

// Direct gather: each thread walks its own row backwards through every step
// and copies the entry it lands on.  Used for states of fewer than 64 rows.
template <int ELEM>
__global__ void __launch_bounds__(256) k_direct(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                                uint64_t n, const TmStep *__restrict__ steps_rev, uint32_t L) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    direct_row<ELEM>(src, dst, i, steps_rev, L);
}

// Plain per-step update: one thread per row pair (i, i | 2^t) with bit t of
// i clear; the pair is interchanged when all control bits of i are 1.
template <int ELEM>
__global__ void __launch_bounds__(256) k_plain_step(uint8_t *__restrict__ buf, uint64_t half_n,
                                                    uint32_t t, uint64_t cm) {
    const uint64_t T = 1ull << t;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < half_n; q += stride) {
        const uint64_t lo = ((q >> t) << (t + 1)) | (q & (T - 1));
        if ((lo & cm) != cm) continue;
        if (ELEM == 8) {
            uint64_t *b = reinterpret_cast<uint64_t *>(buf);
            const uint64_t a0 = b[lo], a1 = b[lo | T];
            b[lo] = a1;
            b[lo | T] = a0;
        } else {
            vec16 *b = reinterpret_cast<vec16 *>(buf);
            const vec16 a0 = b[lo], a1 = b[lo | T];
            b[lo] = a1;
            b[lo | T] = a0;
        }
    }
}

// A run of NOT steps on one target t (controls never include t, so every
// step's condition reads the same bits in both rows of a pair): applied one
// after another they interchange the pair (i, i | 2^t) once per step whose
// controls hold, so the run interchanges it exactly when an odd number of
// them hold (the toggle parity of Sec. 2(i)).  One thread per pair.
struct PlainRun {
    uint64_t cm[kPlainRunMax];
    uint32_t k;
};

template <int ELEM>
__global__ void __launch_bounds__(256) k_plain_run(uint8_t *__restrict__ buf, uint64_t half_n, uint32_t t,
                                                   PlainRun r) {
    const uint64_t T = 1ull << t;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < half_n; q += stride) {
        const uint64_t lo = ((q >> t) << (t + 1)) | (q & (T - 1));
        uint32_t odd = 0;
        for (uint32_t j = 0; j < r.k; ++j) odd ^= (lo & r.cm[j]) == r.cm[j] ? 1u : 0u;
        if (!odd) continue;
        if (ELEM == 8) {
            uint64_t *b = reinterpret_cast<uint64_t *>(buf);
            const uint64_t a0 = b[lo], a1 = b[lo | T];
            b[lo] = a1;
            b[lo | T] = a0;
        } else {
            vec16 *b = reinterpret_cast<vec16 *>(buf);
            const vec16 a0 = b[lo], a1 = b[lo | T];
            b[lo] = a1;
            b[lo | T] = a0;
        }
    }
}

// Plain phase step: every row whose bits in `mask` are all 1 is negated in
// place (sign bits of both parts flipped).  One thread per row of the
// 2^(M - |mask|) selected rows: the row counter is spread into the free bits.
template <int ELEM>
__global__ void __launch_bounds__(256) k_plain_phase(uint8_t *__restrict__ buf, uint64_t n_rows, uint64_t mask,
                                                     uint32_t M) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_rows; q += stride) {
        uint64_t i = mask, c = q;
        for (uint32_t b = 0; b < M && c; ++b) {
            if ((mask >> b) & 1ull) continue;
            i |= (c & 1ull) << b;
            c >>= 1;
        }
        if (ELEM == 8) {
            uint2 *b = reinterpret_cast<uint2 *>(buf);
            const uint2 e = b[i];
            b[i] = make_uint2(e.x ^ 0x80000000u, e.y ^ 0x80000000u);
        } else {
            vec16 *b = reinterpret_cast<vec16 *>(buf);
            const vec16 e = b[i];
            b[i] = make_uint4(e.x, e.y ^ 0x80000000u, e.z, e.w ^ 0x80000000u);
        }
    }
}

// Plain streaming copy (the achievable-bandwidth reference): one 16-byte
// vector per thread and a grid covering the whole buffer, so each
// workgroup moves one 4 KiB block (the fastest copy shape measured on
// MI355X, ahead of grid-stride loops with several vectors per thread).
__global__ void __launch_bounds__(256) k_copy(const vec16 *__restrict__ src, vec16 *__restrict__ dst,
                                              uint64_t nvec) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;   // loops only past 2^31 vectors
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
        st_nt(dst + i, ld_nt(src + i));
}

// Upload of host bytes through a kernel's argument block: the runtime copies
// the arguments when the launch is enqueued, so the source may be freed at
// once and no staging memory is needed (the allocation-free entry point).
struct PutArgs {
    uint32_t words[kPutChunkBytes / 4];
};

__global__ void __launch_bounds__(256) k_put(uint32_t *__restrict__ dst, PutArgs a, uint32_t n_words) {
    for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) dst[i] = a.words[i];
}

// ------------------------------------------------------------ batched mode

// Publishing an item's results to workgroups on other XCDs (separate L2
// caches): every wave first waits until its own stores have reached its
// XCD's L2 (s_waitcnt 0 — a workgroup-scope fence alone does not wait for
// them), the workgroup barrier then orders them before thread 0's
// agent-scope release (one L2 writeback) and counter increment.
__device__ __forceinline__ void publish(uint32_t *counter, uint32_t count) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, count, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *p >= target (relaxed polls); a wait that runs past
// `limit` polls raises the error flag and gives up, so the launch always
// ends.  The caller follows with one agent-scope acquire and a barrier.
__device__ __forceinline__ void wait_at_least(uint32_t *p, uint32_t target, uint32_t *err, uint32_t limit) {
    uint32_t n = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++n > limit) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// Whole small circuit (2^M entries in LDS, every step inner) with the
// first 2^tb threads of the workgroup; states of fewer than 32 rows use a
// direct walk per row.
template <int ELEM, bool SIGN>
__device__ __forceinline__ void small_item(const BatchSmall &sm, vec16 *lds) {
    constexpr uint32_t VPT = Shape<ELEM, 5>::VPT;
    const uint32_t tid = threadIdx.x;
    if (sm.direct) {
        if (tid < (1u << sm.M)) direct_row<ELEM>(sm.src, sm.dst, tid, sm.steps_rev, sm.L);
        return;
    }
    const TileArgs &a = sm.ta;
    const bool active = tid < (1u << a.tb);
    const vec16 *src = static_cast<const vec16 *>(sm.src);
    vec16 *dst = static_cast<vec16 *>(sm.dst);
    uint32_t w[kPlanes];
    const uint32_t off = active ? thread_offset<ELEM>(a.pos_src, a.tb, tid) : 0u;
    if (active) {
        vec16 v[VPT];
        load_tile<ELEM, 5>(v, src, off, a);
        tile_sources<ELEM, 5, false>(w, a, nullptr);
        tile_stage<ELEM, 5>(v, a.tb, lds);
    }
    __syncthreads();
    if (active) tile_emit<ELEM, 5, SIGN>(w, dst, off, a, lds);
}

// Records of tiles t0 .. t0 + nt - 1 of a pass into LDS (rec_stride words
// apart), one tile per thread, then a barrier: the batched kernel forms
// its records where it uses them instead of in a separate phase.
__device__ __forceinline__ void batch_records(const TileMapArgs &tm, uint64_t t0, uint32_t nt, uint32_t *srec,
                                              uint32_t rec_stride) {
    for (uint32_t k = threadIdx.x; k < nt; k += blockDim.x) tilemap_record(tm, t0 + k, srec + k * rec_stride);
    __syncthreads();
}

// Tiles t0 .. t1 - 1 of one pass, each tile's loads issued while the one
// before it is gathered and stored; records from batch_records.
template <int ELEM, bool SIGN>
__device__ __forceinline__ void batch_tiles(const BatchPass &bp, uint64_t t0, uint64_t t1, const uint32_t *srec,
                                            uint32_t rec_stride, vec16 *lds) {
    constexpr uint32_t VPT = Shape<ELEM, 5>::VPT;
    const TileArgs &a = bp.ta;
    const vec16 *src = static_cast<const vec16 *>(bp.src);
    vec16 *dst = static_cast<vec16 *>(bp.dst);
    const uint32_t off_src = thread_offset<ELEM>(a.pos_src, a.tb, threadIdx.x);
    const uint32_t off_dst = thread_offset<ELEM>(a.pos_dst, a.tb, threadIdx.x);
    vec16 v[VPT];
    load_tile<ELEM, 5>(v, src, rec_base(srec) + off_src, a);
    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint32_t *r = srec + (tile - t0) * rec_stride;
        const uint64_t next_base = tile + 1 < t1 ? rec_base(r + rec_stride) + off_src : ~0ull;
        tile_step<ELEM, 5, true, SIGN>(v, src, dst, outer_address(a, tile) + off_dst, next_base, a, r + 2, lds);
        __syncthreads();
    }
}

// Persistent batched launch.  Items are taken from the queue one per
// atomic, in queue order; every item depends only on earlier items, so a
// workgroup that waits never blocks the items its wait depends on.  The
// dynamic LDS holds the tile, then the tile records of the current item
// (rec_stride words per tile).
template <int ELEM, bool SIGN>
__global__ void __launch_bounds__(256) k_batch(const BatchPass *__restrict__ passes,
                                               const BatchSmall *__restrict__ smalls,
                                               const uint64_t *__restrict__ items, uint32_t n_items,
                                               uint32_t *ctr, uint32_t spin_limit, uint32_t tiles_per_item,
                                               uint32_t rec_stride, uint32_t tile_entries) {
    extern __shared__ vec16 lds[];
    __shared__ uint32_t s_item;
    uint32_t *srec = reinterpret_cast<uint32_t *>(lds + tile_entries * ELEM / 16);
    const uint32_t tid = threadIdx.x;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = __hip_atomic_fetch_add(&ctr[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t it = s_item;
        if (it >= n_items) break;   // the same value for the whole workgroup
        const uint64_t e = items[it];
        const uint32_t kind = (uint32_t)(e >> 62);
        const uint32_t idx = (uint32_t)(e >> 32) & 0x3FFFFFFFu;
        const uint32_t sub = (uint32_t)e;
        if (kind == kItemSmall) {
            small_item<ELEM, SIGN>(smalls[idx], lds);
        } else if (kind == kItemCircuit) {
            // Every pass of one circuit (passes idx .. idx + sub - 1), all in
            // this workgroup: no other workgroup touches its buffers, so a
            // pass only has to see this workgroup's stores of the one before.
            for (uint32_t p = 0; p < sub; ++p) {
                const BatchPass &bp = passes[idx + p];
                batch_records(bp.tm, 0, (uint32_t)bp.n_tiles, srec, rec_stride);
                batch_tiles<ELEM, SIGN>(bp, 0, bp.n_tiles, srec, rec_stride, lds);
                // this pass's stores done, then the CU's L1 dropped before
                // the next pass reads what they wrote
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        } else {
            // a block of up to tiles_per_item tiles of one pass, after every
            // tile of the circuit's previous pass
            const BatchPass &bp = passes[idx];
            const uint64_t t0 = (uint64_t)sub * tiles_per_item;
            const uint64_t t1 = t0 + tiles_per_item < bp.n_tiles ? t0 + tiles_per_item : bp.n_tiles;
            batch_records(bp.tm, t0, (uint32_t)(t1 - t0), srec, rec_stride);
            if (tid == 0) {
                wait_at_least(&ctr[kBatchCtrHeader + bp.circuit], bp.level * (uint32_t)bp.n_tiles, &ctr[2],
                              spin_limit);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            batch_tiles<ELEM, SIGN>(bp, t0, t1, srec, rec_stride, lds);
            publish(&ctr[kBatchCtrHeader + bp.circuit], (uint32_t)(t1 - t0));
        }
    }
}

// ------------------------------------------------------------ product-state input

// Entry i of q_M (x) ... (x) q_1 (Appendix 1: the input from M qubit pairs,
// entry i the product of q_b(bit b-1 of i)), formed from q_M down to q_1 in
// the entries' precision; every complex product is (ac - bd) + (ad + bc)i
// with each operation rounded on its own (no contraction into fused
// multiply-adds), so the value is a fixed function of the qubits.
template <typename T>
struct ProductArgs {
    T q[2 * 2 * kMaxQubits];   // q_b(v) at 2 * (2(b-1) + v): (re, im)
    uint32_t M;
};

template <typename T>
__device__ __forceinline__ void cmul(T &re, T &im, T c, T d) {
#pragma clang fp contract(off)
    const T ac = re * c, bd = im * d, ad = re * d, bc = im * c;
    re = ac - bd;
    im = ad + bc;
}

// Fold q_b for b = hi down to lo (address bits hi-1 .. lo-1 of i) into acc.
template <typename T>
__device__ __forceinline__ void fold_bits(const ProductArgs<T> &a, uint64_t i, uint32_t hi, uint32_t lo, T &re,
                                          T &im) {
    for (uint32_t b = hi; b >= lo && b >= 1; --b) {
        const uint32_t v = (uint32_t)((i >> (b - 1)) & 1u);
        cmul(re, im, a.q[2 * (2 * (b - 1) + v)], a.q[2 * (2 * (b - 1) + v) + 1]);
    }
}

// States of M < 13 (or 12 for double) entries: one entry per thread.
template <typename T>
__global__ void __launch_bounds__(256) k_product_small(T *__restrict__ out, ProductArgs<T> a, uint64_t n) {
    const uint32_t M = a.M;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = (uint32_t)((i >> (M - 1)) & 1u);
    T re = a.q[2 * (2 * (M - 1) + v)], im = a.q[2 * (2 * (M - 1) + v) + 1];
    fold_bits(a, i, M - 1, 1, re, im);
    out[2 * i] = re;
    out[2 * i + 1] = im;
}

// Blocks of 2^(5 + tb) consecutive entries, 2^tb threads: thread t forms
// the 32 entries whose five lowest address bits run over all values and
// whose other bits are those of block index and t.  Their folds from q_M
// down share every factor above the fifth bit, so the thread folds those
// once and then splits its partial product at each of the five lowest
// bits (2 + 4 + ... + 32 products): about 3 complex products per entry
// instead of 10, every entry still folded q_M first with each product
// rounded on its own.  The entries are staged in LDS (entry j of the block
// at slot j ^ ((j >> 5) & 31), which spreads a wave's writes over the
// banks) and written out as consecutive 16-byte vectors.
template <typename T>
__global__ void __launch_bounds__(256) k_product(T *__restrict__ out, ProductArgs<T> a, uint64_t n_blocks,
                                                 uint32_t tb) {
    using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    extern __shared__ vec16 lds[];
    V2 *slot = reinterpret_cast<V2 *>(lds);
    const uint32_t M = a.M, t = threadIdx.x;
    const uint32_t entries = 32u << tb;
    constexpr uint32_t EPV = 16 / sizeof(V2);   // entries per 16-byte vector
    for (uint64_t blk = blockIdx.x; blk < n_blocks; blk += gridDim.x) {
        const uint64_t i0 = blk * entries + ((uint64_t)t << 5);
        const uint32_t vtop = (uint32_t)((i0 >> (M - 1)) & 1u);
        T re = a.q[2 * (2 * (M - 1) + vtop)], im = a.q[2 * (2 * (M - 1) + vtop) + 1];
        fold_bits(a, i0, M - 1, 6, re, im);    // q_{M-1} .. q_6: address bits M-2 .. 5
        T pr[32], pi[32];
        pr[0] = re;
        pi[0] = im;
#pragma unroll
        for (int b = 4; b >= 0; --b) {          // q_{b+1}: address bit b
            const int nk = 1 << (4 - b);
            const T c0 = a.q[2 * (2 * b)], d0 = a.q[2 * (2 * b) + 1];
            const T c1 = a.q[2 * (2 * b + 1)], d1 = a.q[2 * (2 * b + 1) + 1];
#pragma unroll
            for (int k = nk - 1; k >= 0; --k) {
                T r0 = pr[k], i0_ = pi[k], r1 = pr[k], i1 = pi[k];
                cmul(r0, i0_, c0, d0);
                cmul(r1, i1, c1, d1);
                pr[2 * k] = r0;
                pi[2 * k] = i0_;
                pr[2 * k + 1] = r1;
                pi[2 * k + 1] = i1;
            }
        }
        // partial e holds the entry whose five lowest bits are e, bit 0 the
        // last split
        __syncthreads();   // the previous block's slots have been read
#pragma unroll
        for (uint32_t e = 0; e < 32u; ++e) {
            const uint32_t j = (t << 5) | e;
            slot[j ^ ((j >> 5) & 31u)] = V2{pr[e], pi[e]};
        }
        __syncthreads();
        vec16 *dst = reinterpret_cast<vec16 *>(out + 2 * blk * entries);
        for (uint32_t v = t; v < entries / EPV; v += blockDim.x) {
            vec16 w;
            if constexpr (EPV == 2) {
                const uint32_t j0 = 2 * v, j1 = 2 * v + 1;
                const V2 e0 = slot[j0 ^ ((j0 >> 5) & 31u)], e1 = slot[j1 ^ ((j1 >> 5) & 31u)];
                w = make_uint4(__float_as_uint(e0.x), __float_as_uint(e0.y), __float_as_uint(e1.x),
                               __float_as_uint(e1.y));
            } else {
                const V2 e0 = slot[v ^ ((v >> 5) & 31u)];
                const uint64_t xr = __double_as_longlong(e0.x), xi = __double_as_longlong(e0.y);
                w = make_uint4((uint32_t)xr, (uint32_t)(xr >> 32), (uint32_t)xi, (uint32_t)(xi >> 32));
            }
            st_nt(dst + v, w);
        }
    }
}

// First pass of a diagram applied to q_M (x) ... (x) q_1.  No HBM read:
// each workgroup forms, from the qubits, the partial products of its source
// tile's entries, walks the pass's steps and stores the permuted entries.
// The fold of an entry runs q_M, ..., q_1 (address bits from the top down),
// so the entries of a tile that agree on every tile bit above bit[CUT - 1]
// share the fold down to just above that bit.  Those 2^(K - CUT) partials
// (the "table") are formed in LDS; at the store each output entry takes its
// partial and folds in the factors of tile bits bit[CUT - 1], ..., bit[0],
// which the first pass holds as address bits CUT - 1, ..., 0 (it keeps the
// lowest bits in its tile).  CUT = 0 stages the whole tile; CUT = 1, 2
// stage half or a quarter of it and finish each entry with one or two
// complex products, which lets more workgroups share a CU (so one
// workgroup's stores overlap the others' formation).  Every entry gets the
// same products in the same order as k_product writes, whatever CUT.
//
// Thread t forms the 2^(5 - CUT) partials whose tile bits bit[CUT .. 4] run
// over all values and whose other tile bits are the bits of t: their folds
// share every factor above bit[4], so a thread folds those once and then
// splits its partial product at each of bit[4], ..., bit[CUT]
// (2 + 4 + ... products), multiplying all partials by the factors of the
// outside bits in between, each product rounded as in k_product.
// pr/pi[e] is the partial whose tile bits bit[CUT + k] read bit k of e.
// The fold of the top address bits is shared by many threads: threads
// whose top h = min(tb, 6) thread bits (tile bits bit[5 + tb - h] and up)
// read u share it down to just above tile bit bit[4 + tb - h] (bit[4] when
// h = tb).  Thread u < 2^h of the workgroup folds that prefix into LDS
// slot u (one wave instead of all of them); every thread then continues
// from its slot through its lower thread bits.
__device__ __forceinline__ uint32_t prefix_bits(uint32_t tb) { return tb < 6u ? tb : 6u; }

template <typename T>
__device__ __forceinline__ void fold_down(T &re, T &im, const T *q, uint64_t addr, int hi, int lo) {
    // Factors are read at addresses that are the same for every lane (both
    // values of a bit, then a per-lane select): scalar loads, not a chain of
    // vector loads.
#pragma unroll 4
    for (int lv = hi; lv >= lo; --lv) {
        const T c0 = q[4 * lv], d0 = q[4 * lv + 1], c1 = q[4 * lv + 2], d1 = q[4 * lv + 3];
        const bool h = (addr >> lv) & 1u;
        cmul(re, im, h ? c1 : c0, h ? d1 : d0);
    }
}

template <typename T>
__device__ __forceinline__ void product_prefix(T *slots, uint64_t src_base, const ProductTileArgs &pa, uint32_t tb) {
    const uint32_t h = prefix_bits(tb), u = threadIdx.x;
    if (u >= (1u << h)) return;
    const T *q = static_cast<const T *>(pa.q);
    uint64_t addr = src_base;
    for (uint32_t i = 0; i < h; ++i) addr |= (uint64_t)((u >> i) & 1u) << pa.bit[5 + tb - h + i];
    const int top = (int)pa.M - 1;
    const int lo = (int)pa.bit[4 + tb - h] + 1;   // bit[4] when h = tb
    const bool b = (addr >> top) & 1u;
    T re = b ? q[4 * top + 2] : q[4 * top], im = b ? q[4 * top + 3] : q[4 * top + 1];
    fold_down(re, im, q, addr, top - 1, lo);
    slots[2 * u] = re;
    slots[2 * u + 1] = im;
}

template <typename T, int CUT>
__device__ __forceinline__ void product_form(T (&pr)[32 >> CUT], T (&pi)[32 >> CUT], const T *slots,
                                             uint64_t src_base, const ProductTileArgs &pa, uint32_t tb) {
    const T *q = static_cast<const T *>(pa.q);
    const uint32_t t = threadIdx.x, h = prefix_bits(tb);
    uint64_t addr = src_base;   // logical address with the five lowest tile bits clear
    for (uint32_t i = 0; i < tb; ++i) addr |= (uint64_t)((t >> i) & 1u) << pa.bit[5 + i];
    const uint32_t u = t >> (tb - h);
    T re = slots[2 * u], im = slots[2 * u + 1];
    // the thread bits below the shared ones, and the outside bits among them
    fold_down(re, im, q, addr, (int)pa.bit[4 + tb - h], (int)pa.bit[4] + 1);
    // Partial k covers the entries whose tile bits i..4 read k (bit 4 highest).
    pr[0] = re;
    pi[0] = im;
#pragma unroll
    for (int i = 4; i >= CUT; --i) {
        const int n = 1 << (4 - i);
        const uint32_t b = pa.bit[i];
        const T c0 = q[4 * b], d0 = q[4 * b + 1], c1 = q[4 * b + 2], d1 = q[4 * b + 3];
#pragma unroll
        for (int k = n - 1; k >= 0; --k) {
            T r0 = pr[k], i0 = pi[k], r1 = pr[k], i1 = pi[k];
            cmul(r0, i0, c0, d0);
            cmul(r1, i1, c1, d1);
            pr[2 * k] = r0;
            pi[2 * k] = i0;
            pr[2 * k + 1] = r1;
            pi[2 * k + 1] = i1;
        }
        const int lo = i > 0 ? (int)pa.bit[i - 1] + 1 : 0;
        for (int l = (int)b - 1; l >= lo; --l) {   // outside bits between tile bits (uniform)
            const bool h = (src_base >> l) & 1u;
            const T c = h ? q[4 * l + 2] : q[4 * l], d = h ? q[4 * l + 3] : q[4 * l + 1];
#pragma unroll
            for (int k = 0; k < 2 * n; ++k) cmul(pr[k], pi[k], c, d);
        }
    }
}

// Thread t's partial e goes to LDS slot t * 2^X + (e ^ (t mod 2^X)),
// X = 5 - CUT, so the lanes of a wave writing their e-th partials spread
// over the banks; product_slot_planes maps source tile indices to these
// slots.
template <typename T, int CUT>
__device__ __forceinline__ void product_stage(vec16 *lds, const T (&pr)[32 >> CUT], const T (&pi)[32 >> CUT]) {
    constexpr uint32_t X = 5 - CUT, N = 1u << X;
    const uint32_t t = threadIdx.x, row = t << X, x = t & (N - 1u);
#pragma unroll
    for (uint32_t e = 0; e < N; ++e) {
        const uint32_t slot = row | (e ^ x);
        if constexpr (sizeof(T) == 4)
            reinterpret_cast<float2 *>(lds)[slot] = make_float2(pr[e], pi[e]);
        else
            reinterpret_cast<double2 *>(lds)[slot] = make_double2(pr[e], pi[e]);
    }
}

// The walked source tile indices (plane b = tile-index bit b) turned into
// LDS slots of product_stage plus the bits folded in at the store.  With
// X = 5 - CUT: slot bit X + i = j[tix[5 + i]] (the bits of the thread that
// formed the partial), slot bit k < X = j[tix[CUT + k]] ^ j[tix[5 + k]] (a
// linear map over GF(2), applied to whole planes); plane 15 - CUT + i holds
// j[tix[i]] for i < CUT (address bit i, folded in at the store); the sign
// plane is kept.  Planes between the slot bits and those are zero.
template <int CUT>
__device__ __forceinline__ void product_slot_planes(uint32_t (&w)[kPlanes], const ProductTileArgs &pa, uint32_t tb) {
    constexpr uint32_t X = 5 - CUT;
    uint32_t s[kPlanes];
#pragma unroll
    for (int b = 0; b < kPlanes; ++b) s[b] = 0u;
    s[kSignPlane] = w[kSignPlane];
#pragma unroll
    for (uint32_t i = 0; i < 10u; ++i)
        if (i < tb) s[X + i] = w[pa.tix[5 + i]];
#pragma unroll
    for (uint32_t k = 0; k < X; ++k) s[k] = w[pa.tix[CUT + k]] ^ (k < tb ? s[X + k] : 0u);
#pragma unroll
    for (uint32_t i = 0; i < (uint32_t)CUT; ++i) s[kSignPlane - CUT + i] = w[pa.tix[i]];
#pragma unroll
    for (int b = 0; b < kPlanes; ++b) w[b] = s[b];
}

// The factors a CUT > 0 product pass folds in at the store, in LDS after
// the partials: for each value c of the CUT residual bits (bit i of c =
// address bit i), the CUT factors in fold order, q_CUT(bit CUT - 1) first.
// One lookup by c replaces a select per factor (the pass is bound by its
// vector instructions).
template <int ELEM, int CUT>
__device__ __forceinline__ size_t product_factor_offset(uint32_t tb) {
    return (size_t)ELEM << (tb + 5 - CUT);   // bytes of the partials before it
}

template <int ELEM, int CUT>
__device__ __forceinline__ void product_factors(vec16 *lds, const ProductTileArgs &pa, uint32_t tb) {
    using T = typename std::conditional<ELEM == 8, float, double>::type;
    const T *q = static_cast<const T *>(pa.q);
    using V2 = typename std::conditional<ELEM == 8, float2, double2>::type;
    V2 *fac = reinterpret_cast<V2 *>(reinterpret_cast<uint8_t *>(lds) + product_factor_offset<ELEM, CUT>(tb));
    for (uint32_t t = threadIdx.x; t < (CUT << CUT); t += blockDim.x) {   // tiles may have 2 threads
        const uint32_t c = t / CUT, j = t % CUT, bit = CUT - 1 - j, h = (c >> bit) & 1u;
        fac[t].x = q[4 * bit + 2 * h];
        fac[t].y = q[4 * bit + 2 * h + 1];
    }
}

// Store the calling thread's output entries of a CUT > 0 product pass: each
// takes its partial from the table and folds in the factors of address bits
// CUT - 1, ..., 0 that its source index carries, then gets the pass's sign.
template <int ELEM, bool SIGN, int CUT>
__device__ __forceinline__ void product_emit(const uint32_t (&w)[kPlanes], vec16 *__restrict__ dst, uint64_t dst_base,
                                             const TileArgs &a, const ProductTileArgs &pa, const vec16 *lds) {
    using T = typename std::conditional<ELEM == 8, float, double>::type;
    using V2 = typename std::conditional<ELEM == 8, float2, double2>::type;
    constexpr uint32_t VPT = Shape<ELEM, 5>::VPT;
    constexpr uint32_t EPV = Shape<ELEM, 5>::EPV;
    constexpr uint32_t kSlot = (1u << (kSignPlane - CUT)) - 1u;
    const V2 *tab = reinterpret_cast<const V2 *>(lds);
    const V2 *fac =
        reinterpret_cast<const V2 *>(reinterpret_cast<const uint8_t *>(lds) + product_factor_offset<ELEM, CUT>(a.tb));
    auto entry = [&](uint32_t v, T &re, T &im) {
        const V2 e = tab[v & kSlot];
        const V2 *g = fac + ((v >> (kSignPlane - CUT)) & ((1u << CUT) - 1u)) * CUT;
        re = e.x;
        im = e.y;
#pragma unroll
        for (int j = 0; j < CUT; ++j) cmul(re, im, g[j].x, g[j].y);
    };
#pragma unroll
    for (uint32_t r = 0; r < VPT; ++r) {
        if constexpr (ELEM == 8) {
            const uint32_t v0 = src_of(w, 2u * r), v1 = src_of(w, 2u * r + 1u);
            T r0, i0, r1, i1;
            entry(v0, r0, i0);
            entry(v1, r1, i1);
            const uint32_t m0 = SIGN ? sign_word(v0) : 0u, m1 = SIGN ? sign_word(v1) : 0u;
            st_nt(dst + (dst_base + a.off_r_dst[r]) / EPV,
                  make_uint4(__float_as_uint(r0) ^ m0, __float_as_uint(i0) ^ m0, __float_as_uint(r1) ^ m1,
                             __float_as_uint(i1) ^ m1));
        } else {
            const uint32_t v0 = src_of(w, r);
            T r0, i0;
            entry(v0, r0, i0);
            const uint32_t m0 = SIGN ? sign_word(v0) : 0u;
            const uint64_t xr = __double_as_longlong(r0), xi = __double_as_longlong(i0);
            st_nt(dst + (dst_base + a.off_r_dst[r]) / EPV,
                  make_uint4((uint32_t)xr, (uint32_t)(xr >> 32) ^ m0, (uint32_t)xi, (uint32_t)(xi >> 32) ^ m0));
        }
    }
}

// One source tile per workgroup: the first wave folds the shared prefixes
// while every wave walks the pass's steps; then the table (the whole tile
// for CUT = 0) is formed and the entries gathered and stored like k_tile.
// (Persistent workgroups that formed the next whole tile while the current
// one's stores drained were slower: 10.27 against 9.61 ms at M = 32.)  The
// pass is bound by its vector instructions: at M = 32 the factor lookup at
// the store and the shared prefixes took it from 6.67 to 6.25 ms, the rate
// of the product kernel's plain writes.
template <int ELEM, bool SIGN, int CUT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(CUT == 2 && !SIGN ? 6 : 1)))
k_tile_product(vec16 *__restrict__ dst, TileArgs a, ProductTileArgs pa, uint64_t n_tiles) {
    using T = typename std::conditional<ELEM == 8, float, double>::type;
    extern __shared__ vec16 lds[];
    const uint64_t tile = xcd_tile((uint64_t)blockIdx.x, a.xcd);
    if (tile >= n_tiles) return;   // uniform over the workgroup
    const uint32_t *rec = a.rec + tile * a.rec_words;
    const uint64_t src_base = rec_base(rec);
    // LDS: the partials, 256 bytes for the factor table, the prefix slots
    T *slots = reinterpret_cast<T *>(reinterpret_cast<uint8_t *>(lds) + product_factor_offset<ELEM, CUT>(a.tb) + 256);
    product_prefix<T>(slots, src_base, pa, a.tb);
    uint32_t w[kPlanes];
    init_planes<ELEM, 5>(w, threadIdx.x, a.tb);
    walk_inner<true>(w, a.inner, a.n_inner, rec + 2);   // while the first wave folds the prefixes
    __syncthreads();
    {
        T pr[32 >> CUT], pi[32 >> CUT];
        product_form<T, CUT>(pr, pi, slots, src_base, pa, a.tb);
        product_stage<T, CUT>(lds, pr, pi);
    }
    if constexpr (CUT > 0) product_factors<ELEM, CUT>(lds, pa, a.tb);
    product_slot_planes<CUT>(w, pa, a.tb);
    transpose_planes(w);
    __syncthreads();
    const uint64_t base = outer_address(a, tile) + thread_offset<ELEM>(a.pos_dst, a.tb, threadIdx.x);
    if constexpr (CUT == 0)
        tile_emit<ELEM, 5, SIGN>(w, dst, base, a, lds);
    else
        product_emit<ELEM, SIGN, CUT>(w, dst, base, a, pa, lds);
}

// ------------------------------------------------------------ materialised row array

// Index vector: entry i holds the integer i (8-byte entries).  Applying a
// diagram to it leaves in row i the row of k1 that lands there, the row
// array x(i) of the whole diagram.
// One-entry-per-thread kernels use grid-stride loops: a launch may not
// exceed 2^32 threads, and states reach 2^36 entries.
__global__ void __launch_bounds__(256) k_iota(uint64_t *__restrict__ out, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = i;
}

__global__ void __launch_bounds__(256) k_narrow(const uint64_t *__restrict__ in, uint32_t *__restrict__ out,
                                                uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (uint32_t)in[i];
}

// k2(i) = k1(x(i)) (Sec. 2(b) end, Summary of Method last bullet).  Every
// access is non-temporal: nothing is read twice (at M = 32 114.1 against
// 118.4 ms with ordinary accesses; the random reads fetch a whole 128-byte
// line per row either way).  Each thread takes two adjacent rows and the
// launch covers the rows once: a grid-stride loop keeps the workgroups in
// flight on regions gigabytes apart (110.0 against 114.0 ms at M = 32).
// n is a power of two of at least 2.
template <int ELEM>
__global__ void __launch_bounds__(256) k_gather(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                                const uint32_t *__restrict__ x, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; 2 * p < n; p += stride) {
        const uint64_t i = 2 * p;
        const uint64_t j0 = __builtin_nontemporal_load(x + i) & (n - 1);   // stays in the state
        const uint64_t j1 = __builtin_nontemporal_load(x + i + 1) & (n - 1);
        if (ELEM == 8) {
            const uint64_t *s = reinterpret_cast<const uint64_t *>(src);
            uint64_t *d = reinterpret_cast<uint64_t *>(dst);
            const uint64_t v0 = __builtin_nontemporal_load(s + j0), v1 = __builtin_nontemporal_load(s + j1);
            __builtin_nontemporal_store(v0, d + i);
            __builtin_nontemporal_store(v1, d + i + 1);
        } else {
            const vec16 *s = reinterpret_cast<const vec16 *>(src);
            vec16 *d = reinterpret_cast<vec16 *>(dst);
            const vec16 v0 = ld_nt(s + j0), v1 = ld_nt(s + j1);
            st_nt(d + i, v0);
            st_nt(d + i + 1, v1);
        }
    }
}

uint32_t stride_grid(uint64_t n) {
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g < (1ull << 20) ? g : (1ull << 20));
}

template <typename KernelT>
hipError_t allow_lds(KernelT kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_direct(uint32_t elem, const void *src, void *dst, uint64_t n,
                         const TmStep *steps_rev, uint32_t L, hipStream_t st) {
    const uint32_t bs = 256;
    const uint64_t grid = (n + bs - 1) / bs;
    if (elem == 8)
        hipLaunchKernelGGL(k_direct<8>, dim3((uint32_t)grid), dim3(bs), 0, st,
                           (const uint8_t *)src, (uint8_t *)dst, n, steps_rev, L);
    else
        hipLaunchKernelGGL(k_direct<16>, dim3((uint32_t)grid), dim3(bs), 0, st,
                           (const uint8_t *)src, (uint8_t *)dst, n, steps_rev, L);
    return hipGetLastError();
}

hipError_t launch_small(uint32_t elem, const void *src, void *dst, uint32_t M,
                        const TileArgs &a, hipStream_t st) {
    const size_t lds = (size_t)elem << M;
    const uint32_t threads = 1u << a.tb;
    auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(1), dim3(threads), lds, st, (const vec16 *)src, (vec16 *)dst, a);
        return hipGetLastError();
    };
    if (elem == 8) return a.sign ? go(k_small<8, true>) : go(k_small<8, false>);
    return a.sign ? go(k_small<16, true>) : go(k_small<16, false>);
}

hipError_t launch_tilemap(const TileMapArgs &a, hipStream_t st) {
    const uint32_t bs = 256;
    const uint64_t grid = (a.n_tiles + bs - 1) / bs;
    hipLaunchKernelGGL(k_tilemap, dim3((uint32_t)grid), dim3(bs), 0, st, a);
    return hipGetLastError();
}

// Resident workgroups of a kernel on the current device (for the persistent
// grid), from the runtime's occupancy query.
template <typename KernelT>
uint64_t resident_blocks(KernelT kernel, uint32_t threads, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel), (int)threads,
                                                     lds) != hipSuccess)
        return 0;
    return (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 1);
}

template <int ELEM, int DEPTH, int EB, bool SIGN>
hipError_t launch_tile_t(const void *src, void *dst, uint64_t n_tiles, const TileArgs &a, uint32_t wg_per_cu,
                         hipStream_t st) {
    const size_t lds = (size_t)ELEM << (a.tb + EB);
    const uint32_t threads = 1u << a.tb;
    if (threads > (uint32_t)tile_threads_max<ELEM, EB>()) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = allow_lds(k_tile<ELEM, DEPTH, EB, SIGN>, lds)) != hipSuccess) return e;
    uint64_t grid = n_tiles;
    if (DEPTH > 0) {
        uint64_t r = 0;
        if (wg_per_cu) {
            int dev = 0, cus = 0;
            if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
            if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
            r = (uint64_t)cus * wg_per_cu;
        } else {
            r = resident_blocks(k_tile<ELEM, DEPTH, EB, SIGN>, threads, lds);
        }
        if (r > 0 && r < grid) grid = r;
    }
    hipLaunchKernelGGL((k_tile<ELEM, DEPTH, EB, SIGN>), dim3((uint32_t)grid), dim3(threads), lds, st,
                       (const vec16 *)src, (vec16 *)dst, a, n_tiles);
    return hipGetLastError();
}

template <int ELEM, int EB, bool SIGN>
hipError_t launch_tile_s(const void *src, void *dst, uint64_t n_tiles, const TileArgs &a, uint32_t variant,
                         uint32_t wg_per_cu, hipStream_t st) {
    if (variant == 2) return launch_tile_t<ELEM, 2, EB, SIGN>(src, dst, n_tiles, a, wg_per_cu, st);
    if (variant >= 1) return launch_tile_t<ELEM, 1, EB, SIGN>(src, dst, n_tiles, a, wg_per_cu, st);
    return launch_tile_t<ELEM, 0, EB, SIGN>(src, dst, n_tiles, a, wg_per_cu, st);
}

template <int ELEM, int EB>
hipError_t launch_tile_e(const void *src, void *dst, uint64_t n_tiles, const TileArgs &a, uint32_t variant,
                         uint32_t wg_per_cu, hipStream_t st) {
    if (a.sign) return launch_tile_s<ELEM, EB, true>(src, dst, n_tiles, a, variant, wg_per_cu, st);
    return launch_tile_s<ELEM, EB, false>(src, dst, n_tiles, a, variant, wg_per_cu, st);
}

// variant 0: one tile per workgroup; 1: persistent, loads one tile ahead;
// 2: persistent, loads two tiles ahead.  a.eb = log2 of the rows per
// thread (3, 4 or 5).
hipError_t launch_tile(uint32_t elem, const void *src, void *dst, uint64_t n_tiles, const TileArgs &a,
                       uint32_t variant, uint32_t wg_per_cu, hipStream_t st) {
    if (elem == 8) {
        if (a.eb == 3) return launch_tile_e<8, 3>(src, dst, n_tiles, a, variant, wg_per_cu, st);
        if (a.eb == 4) return launch_tile_e<8, 4>(src, dst, n_tiles, a, variant, wg_per_cu, st);
        return launch_tile_e<8, 5>(src, dst, n_tiles, a, variant, wg_per_cu, st);
    }
    if (a.eb == 3) return launch_tile_e<16, 3>(src, dst, n_tiles, a, variant, wg_per_cu, st);
    if (a.eb == 4) return launch_tile_e<16, 4>(src, dst, n_tiles, a, variant, wg_per_cu, st);
    return launch_tile_e<16, 5>(src, dst, n_tiles, a, variant, wg_per_cu, st);
}

hipError_t launch_plain_step(uint32_t elem, void *buf, uint32_t M, uint32_t target,
                             uint64_t cmask, hipStream_t st) {
    const uint64_t half_n = 1ull << (M - 1);
    const uint32_t bs = 256;
    const uint64_t grid = std::min<uint64_t>((half_n + bs - 1) / bs, 1ull << 22);
    if (elem == 8)
        hipLaunchKernelGGL(k_plain_step<8>, dim3((uint32_t)grid), dim3(bs), 0, st, (uint8_t *)buf, half_n,
                           target, cmask);
    else
        hipLaunchKernelGGL(k_plain_step<16>, dim3((uint32_t)grid), dim3(bs), 0, st, (uint8_t *)buf, half_n,
                           target, cmask);
    return hipGetLastError();
}

hipError_t launch_plain_run(uint32_t elem, void *buf, uint32_t M, uint32_t target, const uint64_t *cmasks,
                            uint32_t k, hipStream_t st) {
    if (k < 1 || k > kPlainRunMax) return hipErrorInvalidValue;
    PlainRun r{};
    for (uint32_t j = 0; j < k; ++j) r.cm[j] = cmasks[j];
    r.k = k;
    const uint64_t half_n = 1ull << (M - 1);
    const uint32_t bs = 256;
    const uint64_t grid = std::min<uint64_t>((half_n + bs - 1) / bs, 1ull << 22);
    if (elem == 8)
        hipLaunchKernelGGL(k_plain_run<8>, dim3((uint32_t)grid), dim3(bs), 0, st, (uint8_t *)buf, half_n, target, r);
    else
        hipLaunchKernelGGL(k_plain_run<16>, dim3((uint32_t)grid), dim3(bs), 0, st, (uint8_t *)buf, half_n, target, r);
    return hipGetLastError();
}

hipError_t launch_plain_phase(uint32_t elem, void *buf, uint32_t M, uint64_t mask, hipStream_t st) {
    const uint64_t n_rows = 1ull << (M - (uint32_t)__builtin_popcountll(mask));
    const uint32_t bs = 256;
    const uint64_t grid = std::min<uint64_t>((n_rows + bs - 1) / bs, 1ull << 22);
    if (elem == 8)
        hipLaunchKernelGGL(k_plain_phase<8>, dim3((uint32_t)grid), dim3(bs), 0, st, (uint8_t *)buf, n_rows, mask, M);
    else
        hipLaunchKernelGGL(k_plain_phase<16>, dim3((uint32_t)grid), dim3(bs), 0, st, (uint8_t *)buf, n_rows, mask, M);
    return hipGetLastError();
}

template <int ELEM, bool SIGN>
hipError_t batch_kernel_grid(uint32_t tb, size_t lds, uint64_t *grid) {
    const uint32_t threads = 1u << tb;
    auto kern = k_batch<ELEM, SIGN>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    *grid = resident_blocks(kern, threads, lds);
    if (*grid == 0) *grid = 256;
    return hipSuccess;
}

hipError_t batch_grid(uint32_t elem, uint32_t tb, bool sign, size_t lds, uint64_t *grid) {
    if (tb > 8 || lds > 160 * 1024) return hipErrorInvalidValue;
    if (elem == 8) return sign ? batch_kernel_grid<8, true>(tb, lds, grid) : batch_kernel_grid<8, false>(tb, lds, grid);
    return sign ? batch_kernel_grid<16, true>(tb, lds, grid) : batch_kernel_grid<16, false>(tb, lds, grid);
}

hipError_t launch_batch(uint32_t elem, uint32_t tb, bool sign, const BatchPass *passes, const BatchSmall *smalls,
                        const uint64_t *items, uint32_t n_items, uint32_t *counters, uint32_t spin_limit,
                        uint32_t tiles_per_item, uint32_t rec_stride, size_t lds, hipStream_t st) {
    const uint32_t threads = 1u << tb;
    const uint32_t tile_entries = 1u << (tb + 5);
    uint64_t grid = 0;
    hipError_t e = batch_grid(elem, tb, sign, lds, &grid);
    if (e != hipSuccess) return e;
    if (grid > n_items) grid = n_items;
    if (grid == 0) return hipSuccess;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(threads), lds, st, passes, smalls, items, n_items,
                           counters, spin_limit, tiles_per_item, rec_stride, tile_entries);
        return hipGetLastError();
    };
    if (elem == 8) return sign ? go(k_batch<8, true>) : go(k_batch<8, false>);
    return sign ? go(k_batch<16, true>) : go(k_batch<16, false>);
}

hipError_t launch_product(uint32_t elem, void *out, uint32_t M, const void *qubits, hipStream_t st) {
    const uint64_t n = 1ull << M;
    if (M < 1 || M > kMaxQubits) return hipErrorInvalidValue;
    // blocks of 2^13 (float) / 2^12 (double) entries: 256 / 128 threads and
    // 64 KiB of LDS; smaller states one entry per thread
    const uint32_t tb = elem == 8 ? 8u : 7u;
    auto go = [&](auto a, auto *o, auto kern, auto small) {
        std::memcpy(a.q, qubits, sizeof(a.q[0]) * 4 * M);
        a.M = M;
        if (M < tb + 5) {
            hipLaunchKernelGGL(small, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, o, a, n);
            return hipGetLastError();
        }
        const size_t lds = (size_t)elem << (tb + 5);
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        const uint64_t blocks = n >> (tb + 5);
        uint64_t grid = resident_blocks(kern, 1u << tb, lds);
        if (grid == 0) grid = 512;
        grid = std::min<uint64_t>(blocks, 8 * grid);
        hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(1u << tb), lds, st, o, a, blocks, tb);
        return hipGetLastError();
    };
    if (elem == 8)
        return go(ProductArgs<float>{}, (float *)out, k_product<float>, k_product_small<float>);
    return go(ProductArgs<double>{}, (double *)out, k_product<double>, k_product_small<double>);
}

hipError_t launch_tile_product(uint32_t elem, void *dst, uint64_t n_tiles, const TileArgs &a,
                               const ProductTileArgs &pa, hipStream_t st) {
    const uint32_t threads = 1u << a.tb;
    if (a.eb != 5 || threads > 512u || pa.cut > 2u) return hipErrorInvalidValue;
    // the partials, 256 bytes for the table of folded-in factors (CUT > 0),
    // 64 shared prefixes
    const size_t lds = ((size_t)elem << (a.tb + 5 - pa.cut)) + 256u + 64u * elem;
    auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((uint32_t)n_tiles), dim3(threads), lds, st, (vec16 *)dst, a, pa, n_tiles);
        return hipGetLastError();
    };
    auto by_cut = [&](auto e8, auto sign) {
        constexpr int E = decltype(e8)::value;
        constexpr bool S = decltype(sign)::value;
        if (pa.cut == 1) return go(k_tile_product<E, S, 1>);
        if (pa.cut == 2) return go(k_tile_product<E, S, 2>);
        return go(k_tile_product<E, S, 0>);
    };
    using I8 = std::integral_constant<int, 8>;
    using I16 = std::integral_constant<int, 16>;
    using ST = std::true_type;
    using SF = std::false_type;
    if (elem == 8) return a.sign ? by_cut(I8{}, ST{}) : by_cut(I8{}, SF{});
    return a.sign ? by_cut(I16{}, ST{}) : by_cut(I16{}, SF{});
}

hipError_t launch_iota(uint64_t *out, uint64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_iota, dim3(stride_grid(n)), dim3(256), 0, st, out, n);
    return hipGetLastError();
}

hipError_t launch_narrow(const uint64_t *in, uint32_t *out, uint64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_narrow, dim3(stride_grid(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

hipError_t launch_gather(uint32_t elem, const void *src, void *dst, const uint32_t *x, uint64_t n, hipStream_t st) {
    if (n < 2 || (n & (n - 1))) return hipErrorInvalidValue;
    // one thread per pair of rows, at most 2^31 threads (2^32 rows)
    const dim3 grid((uint32_t)std::min<uint64_t>((n / 2 + 255) / 256, 1ull << 23));
    if (elem == 8)
        hipLaunchKernelGGL(k_gather<8>, grid, dim3(256), 0, st, (const uint8_t *)src, (uint8_t *)dst, x, n);
    else
        hipLaunchKernelGGL(k_gather<16>, grid, dim3(256), 0, st, (const uint8_t *)src, (uint8_t *)dst, x, n);
    return hipGetLastError();
}

hipError_t launch_put(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes & 3u) return hipErrorInvalidValue;
    const uint8_t *p = static_cast<const uint8_t *>(src);
    uint8_t *d = static_cast<uint8_t *>(dst);
    for (size_t off = 0; off < bytes; off += kPutChunkBytes) {
        const size_t n = std::min<size_t>(kPutChunkBytes, bytes - off);
        PutArgs a;
        std::memcpy(a.words, p + off, n);
        hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t *>(d + off), a,
                           (uint32_t)(n / 4));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t st) {
    const uint64_t nvec = bytes / 16;
    if (nvec == 0) return hipSuccess;
    const uint32_t bs = 256;
    const uint64_t grid = std::min<uint64_t>((nvec + bs - 1) / bs, 1ull << 23);   // at most 2^31 threads
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)grid), dim3(bs), 0, st, (const vec16 *)src, (vec16 *)dst, nvec);
    return hipGetLastError();
}

}  // namespace qsim
