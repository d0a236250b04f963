// peel_common.h - peel state, work items and device helpers shared by the
// single-graph peel (peel.hip) and the batch peel (peel_multi.hip): coherent
// loads and stores of shared state, wave-level slot allocation, chunked work
// items, the two-level grid barrier and the state initialisation kernels.
#pragma once

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "pipeline.h"

namespace bt {

// Cooperative peel kernels hold every CU until their last round; two of
// them at once (from different threads or engine slots) could each wait at
// a grid barrier for blocks the other keeps from being scheduled.  They
// therefore take turns in the process, in the order they asked.  While a
// turn is held, a waiter that weighs under 1/8 of the holder raises the
// holder's yield word (pinned host memory that the kernel reads every few
// rounds); the peel kernel then ends its launch between two rounds, and its
// host thread queues again and relaunches from the state left in device
// memory.
class CoopTurn {
  public:
    // Blocks until this turn comes.  The turn weighs `weight` (the peel's
    // edges) unless the calling thread set another weight for its turns.
    explicit CoopTurn(int64_t weight);
    ~CoopTurn();
    CoopTurn(const CoopTurn &) = delete;
    CoopTurn &operator=(const CoopTurn &) = delete;
    // Device address of the yield word (nonzero: a lighter peel waits).
    // With force, a word that always reads 1, for tests of the resume path.
    const int32_t *yield_word(bool force) const;
    // Gives the device up, queues behind every current waiter and returns
    // when the turn comes again.
    void requeue();

  private:
    uint64_t ticket_ = 0;
    int64_t weight_ = 0;
};

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLinkChunk = kWave;   // links per phase-A work item (one per lane)
// Progressive mode: edge ids in wedge records and link twins carry this bit
// when the edge's bitruss number was fixed in an earlier pass; such edges
// keep their blooms alive but are never decremented or removed.
constexpr uint32_t kFixedBit = 0x80000000u;
constexpr uint32_t kEdgeMask = 0x7fffffffu;
constexpr int kWedgeChunk = kWave;  // wedges per phase-B work item (one per lane)
inline int grid_a() {
    static int g = std::getenv("BT_PEEL_GRID_A") ? std::atoi(std::getenv("BT_PEEL_GRID_A")) : 2048;
    return g;
}
inline int grid_b() {
    static int g = std::getenv("BT_PEEL_GRID_B") ? std::atoi(std::getenv("BT_PEEL_GRID_B")) : 2048;
    return g;
}

typedef unsigned long long u64;

enum : int32_t { kNormal = 0, kGather = 1 };

// A counter alone on its cache line (contended atomics do not share lines).
struct alignas(128) Counter {
    u64 v;
};

struct PeelCtl {
    Counter nf[2];      // frontier work items by round parity
    Counter ntc[2];     // bloom work items by round parity
    Counter na[2];      // active-set entries by buffer
    Counter updates;
    Counter bloom_visits;
    Counter unbatched;  // extra decrements if survivors took one per kill (no bloom batching)
    Counter touched;    // live wedges visited in phase B (survivors of touched blooms)
    // Round state, indexed by round parity.  Round r's entry is derived
    // from round r - 1's final counters (every block computes the same
    // values; block 0 stores them for round r + 1).
    int32_t mode[2];    // kNormal or kGather
    int32_t level[2];
    int32_t cur[2];     // active-set buffer in use
    int32_t gmin[2];    // gather rounds: minimum support above the level
    int32_t stall;
    int32_t thresh;     // active threshold T
    int32_t max_level;  // largest level at which edges were removed
    int32_t pad;
    u64 rounds, levels;
    u64 prof[6];        // persistent kernel, BT_PEEL_PROFILE=1: block-0 clock ticks
    // BT_PEEL_PROFILE=1: frontier pushes by twin (phase A) and survivor
    // (phase B) decrements, by list parity; rounds whose frontier came from
    // twin decrements alone; log2 histograms of per-round work items.
    Counter push_twin[2], push_surv[2];
    u64 twin_only_rounds, twin_pushes, surv_pushes;
    u64 hist_nf[32], hist_ntc[32];
    // Block-0 clock ticks of whole rounds by log2 of their frontier items,
    // and of phase B by log2 of its bloom items.
    u64 time_nf[32], time_ntc[32];
};

struct alignas(16) FrontItem {
    int32_t e;
    int32_t level;    // level of the round that removes e
    uint32_t lo, hi;  // link positions of this chunk
};

struct alignas(16) BloomItem {
    int32_t b;
    int32_t nch;    // chunks of this bloom (the last one to finish finalizes)
    uint32_t lo, hi;  // wedge range of this chunk
};

struct PeelArgs {
    PeelCtl *ctl;
    int32_t *sup;
    int32_t *phi;
    uint32_t *alive;
    int32_t *bc;
    int32_t *bk;
    int32_t *bdone;
    const uint32_t *bwoff;
    const int32_t *wea;
    const int32_t *web;
    const int32_t *wbl;
    const int64_t *link_off;
    const uint3 *link;  // {wedge, bloom, twin edge}
    int32_t prof;       // count profile statistics
    int32_t unit;       // ablation without batch bloom processing (BiT-BU+)
    FrontItem *front[2];
    BloomItem *tc[2];
    int32_t *act[2];
};

// Coherent access to state that blocks share within one launch.  The eight
// XCDs keep separate L2 caches; device-scope loads and stores (relaxed
// atomics) go to the point of coherence, so no round needs the L2 write-back
// and invalidation that a device-scope fence costs, and the read-only index
// stays cached in L2 across rounds.  Every access to mutable peel state
// inside a launch goes through these.
template <typename T> __device__ __forceinline__ T ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ void st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// 16-byte work items move as two coherent 8-byte halves.
template <typename Item> __device__ __forceinline__ void st_item(Item *p, const Item &v) {
    static_assert(sizeof(Item) == 16, "work items are 16 bytes");
    u64 h[2];
    __builtin_memcpy(h, &v, 16);
    st(reinterpret_cast<u64 *>(p), h[0]);
    st(reinterpret_cast<u64 *>(p) + 1, h[1]);
}
template <typename Item> __device__ __forceinline__ Item ld_item(const Item *p) {
    u64 h[2];
    h[0] = ld(reinterpret_cast<const u64 *>(p));
    h[1] = ld(reinterpret_cast<const u64 *>(p) + 1);
    Item v;
    __builtin_memcpy(&v, h, 16);
    return v;
}

// Each lane asks for `cnt` consecutive slots of *counter; one atomic per
// wave.  Must be called by all 64 lanes.
__device__ __forceinline__ u64 wave_alloc(uint32_t cnt, u64 *counter) {
    const u64 inc = wave_inclusive_sum<u64>((u64)cnt);
    const u64 total = __shfl(inc, kWave - 1, kWave);
    u64 base = 0;
    if (lane_id() == kWave - 1 && total) base = atomicAdd(counter, total);
    base = __shfl(base, kWave - 1, kWave);
    return base + inc - cnt;
}

// Slot requests against up to three counters (a null counter takes no
// requests): each wave issues its atomics together and waits once.  Must be
// called by all 64 lanes.
__device__ __forceinline__ void wave_alloc3(uint32_t c0, u64 *k0, uint32_t c1, u64 *k1,
                                            uint32_t c2, u64 *k2, u64 (&base)[3]) {
    const uint32_t cnt[3] = {c0, c1, c2};
    u64 *const ctr[3] = {k0, k1, k2};
    uint32_t inc[3], tot[3];  // a wave's requests stay far below 2^32
    u64 r[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        inc[k] = wave_inclusive_sum<uint32_t>(cnt[k]);
        tot[k] = __shfl(inc[k], kWave - 1, kWave);
    }
    if (lane_id() == kWave - 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (tot[k]) r[k] = atomicAdd(ctr[k], (u64)tot[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) base[k] = __shfl(r[k], kWave - 1, kWave) + (inc[k] - cnt[k]);
}

// Frontier work items of an edge: its links in chunks of 64, at least one
// chunk so that an edge without links still receives its bitruss number.
__device__ __forceinline__ uint32_t link_chunks(uint32_t lo, uint32_t hi) {
    return hi - lo <= (uint32_t)kLinkChunk ? 1u : (hi - lo + kLinkChunk - 1) / kLinkChunk;
}

// The pusher also records the edge's bitruss number: an edge is queued at
// the level of the round that removes it (a queued frontier keeps the
// level), and only a gather, which runs once the frontier is empty, reads
// phi while the peel runs.
// Writes the cnt 64-element chunks of a lane's range [lo, hi) as items
// {id, aux, a, min(a + 64, hi)} at slots base, base + 1, ...  A lane writes
// up to kOwnChunks of its own; the rest of a longer range is written by the
// whole wave, 64 chunks at a time, so a hub edge or a large bloom does not
// hold up its wave (and the round) with thousands of serial stores.  All 64
// lanes must call.
constexpr uint32_t kOwnChunks = 4;
template <typename Item>
__device__ __forceinline__ void put_chunks(Item *list, u64 base, uint32_t cnt, int32_t id,
                                           int32_t aux, uint32_t lo, uint32_t hi) {
    const uint32_t own = min(cnt, kOwnChunks);
    for (uint32_t c = 0; c < own; ++c) {
        const uint32_t a = lo + c * kWave;
        st_item(&list[base + c], Item{id, aux, a, min(a + (uint32_t)kWave, hi)});
    }
    unsigned long long big = __ballot(cnt > own);
    while (big) {
        const int l = __ffsll(big) - 1;
        big &= big - 1;
        const uint32_t n = __shfl(cnt, l, kWave);
        const u64 b = __shfl(base, l, kWave);
        const int32_t lid = __shfl(id, l, kWave), laux = __shfl(aux, l, kWave);
        const uint32_t llo = __shfl(lo, l, kWave), lhi = __shfl(hi, l, kWave);
        for (uint32_t c = kOwnChunks + lane_id(); c < n; c += kWave) {
            const uint32_t a = llo + c * kWave;
            st_item(&list[b + c], Item{lid, laux, a, min(a + (uint32_t)kWave, lhi)});
        }
    }
}

__device__ __forceinline__ void put_front(const PeelArgs &P, int q, u64 base, int32_t e,
                                          uint32_t lo, uint32_t hi, uint32_t k, int32_t level) {
    if (k) st(&P.phi[e], level);
    put_chunks(P.front[q], base, k, e, level, lo, hi);  // the item carries the level
}

enum : int { kSrcTwin = 0, kSrcSurvivor = 1 };

// Profile statistics: frontier pushes by the decrement that caused them.
__device__ __forceinline__ void count_push(const PeelArgs &P, int q, int src, uint32_t n) {
    const u64 t = wave_sum<u64>((u64)n);
    if (lane_id() == 0 && t)
        atomicAdd(src == kSrcTwin ? &P.ctl->push_twin[q].v : &P.ctl->push_surv[q].v, t);
}

// --- cooperative kernels: workgroup size and the grid barrier ------------

constexpr int kPBlock = 1024;  // 16 waves per CU (up to 128 VGPRs: four waves per SIMD)

struct GridBar {
    Counter group[8];  // arrivals per group (monotonic)
    Counter top;       // completed groups (monotonic)
    Counter rel[8];    // per-group release: the number of the last open barrier
    int32_t fail;
};

// Waits until this wave's memory operations have completed: its device-scope
// stores and atomics have reached the point of coherence.
__device__ __forceinline__ void drain_memory() {
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Two-level barrier, thread 0 of each block; `k` counts the barriers this
// block has passed.  Blocks arrive at one of eight group counters (group g
// holds the blocks of XCD g), the last of each group at the top counter; the
// last of those writes the barrier's number to every group's release word,
// and each block polls its own group's word, so no address takes the polls
// of the whole grid.  Counters only grow, so nothing is reset between
// barriers.  Shared state is only touched through device-scope accesses, so
// draining every wave's outstanding operations before arrival (done by the
// caller for all waves) orders them before the barrier, with no cache
// write-back or invalidation.  A waiter gives up after a bounded spin (the
// kernel then stops with `fail` set) so no bug can hang the device.
__device__ bool grid_arrive_wait(GridBar *B, u64 &k) {
    const unsigned nb = gridDim.x;
    const unsigned g = blockIdx.x & 7;
    const unsigned ngroups = nb < 8 ? nb : 8;
    const unsigned gsize = (nb - g + 7) / 8;
    k += 1;
    if (atomicAdd(&B->group[g].v, 1ull) == k * gsize - 1) {
        if (atomicAdd(&B->top.v, 1ull) == k * ngroups - 1) {
            for (unsigned j = 0; j < ngroups; ++j) st(&B->rel[j].v, k);
        }
    }
    bool ok = true;
    int64_t spins = 0;
    while (ld(&B->rel[g].v) < k) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (int64_t(1) << 28) || ld(&B->fail)) {
            st(&B->fail, 1);
            ok = false;
            break;
        }
    }
    drain_memory();
    return ok;
}

// Edges whose bitruss number is already fixed (progressive mode) start
// removed-looking (phi >= 0) with an unreachable support, so no gather,
// refill or crossing ever takes them.
__global__ void k_init_peel(const uint64_t *supl, int64_t m, const int32_t *fixed, int32_t *sup,
                            int32_t *phi, int64_t *sup_out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = (int32_t)(supl[e] & 0xffffffffu);
        const bool fx = fixed && fixed[e];
        sup[e] = fx ? INT_MAX : s;
        phi[e] = fx ? INT_MAX : -1;
        if (sup_out) sup_out[e] = s;
    }
}

__global__ void k_init_alive(const uint64_t *cursor, uint32_t *alive) {
    const int64_t nw = (int64_t)(*cursor & 0xffffffffu);
    const int64_t words = (nw + 31) / 32;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rem = nw - i * 32;
        alive[i] = rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
    }
}

__global__ void k_phi_out(const int32_t *phi, int64_t *out, int64_t m) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = phi[e];
}

}  // namespace

}  // namespace bt
