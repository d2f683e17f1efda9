// qh_device.h -- device-side building blocks for CDNA4 (gfx950, wave64).
//
// * wave-wide inclusive prefix sums with DPP row shifts and row broadcasts;
// * block-wide exclusive scans built on them;
// * a single-pass decoupled-lookback scan (Merrill & Garland, "Single-pass
//   Parallel Prefix Scan with Decoupled Look-back", 2016) over dynamically
//   numbered tiles, carrying two 31-bit counters in one 64-bit status word;
// * the workspace records shared by the round kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qh {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// DPP wave scans
// ---------------------------------------------------------------------------
template <int Ctrl, int RowMask = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, true);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    v += dpp_u32<0x111>(v);        // row_shr:1
    v += dpp_u32<0x112>(v);        // row_shr:2
    v += dpp_u32<0x114>(v);        // row_shr:4
    v += dpp_u32<0x118>(v);        // row_shr:8
    v += dpp_u32<0x142, 0xa>(v);   // row_bcast:15 -> rows 1 and 3
    v += dpp_u32<0x143, 0xc>(v);   // row_bcast:31 -> rows 2 and 3
    return v;
}

__device__ __forceinline__ uint32_t wave_read(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return wave_read(wave_incl_sum(v), kWave - 1);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Block-wide exclusive scan of NV independent 32-bit values per thread.
// scratch: NV * (BLOCK / 64) words of LDS.  Returns the block totals in tot[].
template <int BLOCK, int NV>
__device__ __forceinline__ void block_excl_scan(uint32_t (&v)[NV], uint32_t (&tot)[NV],
                                                uint32_t *scratch) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    uint32_t inc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        inc[i] = wave_incl_sum(v[i]);
        if (lane == kWave - 1) scratch[i * NW + w] = inc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            uint32_t t = scratch[i * NW + j];
            before += (j < w) ? t : 0u;
            all += t;
        }
        v[i] = before + inc[i] - v[i];
        tot[i] = all;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Decoupled look-back over dynamically numbered tiles.
//
// status word: bits 63..62 flag (0 = nothing yet, 1 = tile aggregate,
// 2 = inclusive prefix), bits 61..31 counter A, bits 30..0 counter B.
// Every count is below 2^31, so packed words add field by field.
// ---------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint64_t kPayload = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t pack2(uint32_t a, uint32_t b) {
    return ((uint64_t)a << 31) | (uint64_t)b;
}
__device__ __forceinline__ uint32_t unpackA(uint64_t p) { return (uint32_t)((p >> 31) & 0x7fffffffu); }
__device__ __forceinline__ uint32_t unpackB(uint64_t p) { return (uint32_t)(p & 0x7fffffffu); }

__device__ __forceinline__ uint64_t status_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every lane of ONE wave.  Publishes the tile aggregate, walks back
// over the predecessors 64 at a time and returns the exclusive prefix of the
// tile (packed).  The tile's inclusive prefix is published before returning.
// The wait is bounded: after kSpinLimit polls the tile gives up, raises
// kErrStall in *err and proceeds, so a bug can never hang the device.
constexpr int kSpinLimit = 1 << 20;

__device__ __forceinline__ uint64_t lookback_excl(uint64_t *status, int tile, uint64_t agg,
                                                  int32_t *err) {
    const int lane = lane_id();
    if (tile == 0) {
        if (lane == 0) status_store(&status[0], kFlagPre | agg);
        return 0;
    }
    if (lane == 0) status_store(&status[tile], kFlagAgg | agg);
    uint32_t exA = 0, exB = 0;
    int base = tile - 1;
    while (true) {
        // lane l looks at tile base - l; tiles before 0 read as a zero prefix
        const int i = base - lane;
        uint64_t v, pm, need;
        int spins = 0;
        while (true) {
            v = (i >= 0) ? status_load(&status[i]) : kFlagPre;
            pm = __ballot((v >> 62) == 2);
            const uint64_t zm = __ballot((v >> 62) == 0);
            // lanes up to and including the nearest published prefix
            need = pm ? (((pm & (~pm + 1)) << 1) - 1) : ~0ull;
            if ((zm & need) == 0) break;
            if (++spins >= kSpinLimit) {
                if (lane == 0) atomicOr(err, 16);
                pm = ~0ull;
                need = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        const bool take = (need >> lane) & 1;
        exA += wave_sum(take ? unpackA(v) : 0u);
        exB += wave_sum(take ? unpackB(v) : 0u);
        if (pm != 0) break;
        base -= kWave;
    }
    const uint64_t ex = pack2(exA, exB);
    if (lane == 0) status_store(&status[tile], kFlagPre | (ex + agg));
    return ex;
}

// ---------------------------------------------------------------------------
// Records shared by the 2D kernels
// ---------------------------------------------------------------------------

// A segment of the survivor array: the points of [start, start + len) of one
// region lie strictly outside the directed hull edge u -> v, and f is the
// farthest of them (the apex found when the segment was made).
struct SegGeo {
    int32_t start, len;
    int32_t ux, uy, fx, fy, vx, vy;
};

// Bookkeeping of a segment: f's input index, the compact hull ids of u and v,
// and the instance the segment belongs to.
struct SegTop {
    int32_t fidx, uc, vc, inst;
};

// Best point of a child segment seen by one tile (or the reduction of several
// tiles).  key1 is the exact distance (0 = no point), key2 the tie-break
// (lower is better), then the point itself and the number of the child's
// points the record covers.
struct Best {
    uint64_t key1;
    uint64_t key2;
    int32_t x, y, idx, cnt;
};

__device__ __forceinline__ bool best_better(const Best &a, const Best &b) {
    return a.key1 > b.key1 || (a.key1 == b.key1 && a.key1 != 0 && a.key2 < b.key2);
}

// Per-round control values (two copies, by round parity).
struct RoundState {
    int32_t n[2];       // points in region 0 / 1
    int32_t s[2];       // segments in table 0 / 1
    int32_t hbase;      // first compact hull id of this round's apexes
    int32_t npc[2];     // non-empty pieces of region 0 / 1 (rounds after the first split)
    uint32_t seg_ctr;   // dynamic tile counter of the segment kernel
    uint32_t piece_ctr; // dynamic tile counter of the piece scan
    int32_t nmulti;     // tiles with several segments (listed for the round kernel)
};

enum : int32_t {
    kErrRange = 1,
    kErrSegCap = 2,
    kErrHullCap = 4,
    kErrOffsets = 8,
    kErrStall = 16,     // a look-back wait gave up (internal error)
    kErrInternal = 32,  // an internal index check failed
};

constexpr int kAccSlots = 64;

struct Control {
    RoundState rs[2];
    int32_t error;
    int32_t rounds_done;
    int32_t max_segments;
    int32_t final_round;              // parity source of the final state
    unsigned long long points_in;     // points read by the rounds after the first split
    unsigned long long points_out;    // survivors written by those rounds
    unsigned long long first_in;      // points read by the first split
    unsigned long long first_out;     // survivors of the first split (counted, not written)
    unsigned long long second_in;     // input points read by the round after it
    unsigned long long second_out;    // survivors written by that round
    // FP32-filter counters (tests, fallbacks, argmax candidates), spread
    // over kAccSlots words each like nacc
    unsigned long long fstat[3][64];
    unsigned long long rounds_with_work;
    // survivors per region counted by the round kernels, by parity, spread
    // over kAccSlots words each (the blocks add into the word of their number
    // modulo kAccSlots, so that few additions meet at one address)
    unsigned int nacc[2][2][64];
    int32_t tper[2];                  // tiles per block of the round kernel, by parity
    int32_t tper_ext;                 // tiles per block of the extremes kernel
    int32_t maxseg[2];                // largest segment of the round, by parity
    uint32_t fin_ids;                 // hull ids taken by the finishing pass
    int32_t fin_round;                // the round that finished every segment (-1: none)
    int32_t fin_runs;                 // ... in runs of small segments (1) or one by one (0)
    int32_t H;                        // compact hull ids used
    long long h_total;                // hull vertices of all instances
    int32_t nstamps;
    int32_t setup_error;              // errors of the set-up phases only
    uint32_t cspan;                   // largest |coordinate| of the input plus kCoordMax2D
    uint32_t cspan_slot[64];          // ... per group of extremes blocks (merged into cspan)
    long long stamps[256];            // wall-clock stamps at phase ends (timing only)
};

}  // namespace qh
