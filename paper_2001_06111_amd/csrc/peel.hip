// peel.hip - bulk-synchronous peel through blooms (Algorithm 5: batch edge
// and batch bloom processing), driven entirely on the device.
//
// State: sup (int32, unclamped), phi (int32, -1 while the edge remains),
// one alive bit per wedge, per bloom its live wedge count k and the count C
// of wedges removed this round.  A round with level L and frontier F (the
// remaining edges with support <= L):
//   A. every edge of F gets phi = L; each of its wedges still alive is
//      killed (one winner per wedge), C[B] += 1 for its bloom B, and the
//      twin edge loses all of its k[B] - 1 butterflies in B;
//   B. in every bloom touched in A, each surviving wedge's two edges lose
//      C[B] butterflies (the bloom shrinks from k to k - C); then
//      k[B] -= C[B], C[B] = 0.  Once k[B] <= 1 the bloom holds no
//      butterfly and its last wedge is retired.
// The paper clamps decremented supports at the round's minimum (max(MBS,
// .)); subtracting unclamped and treating every support <= L as "at level
// L" gives the same bitruss numbers, since max(M, max(M, a - d1) - d2) =
// max(M, a - d1 - d2).  A decrement that takes a support from above L to at
// most L puts the edge in the next frontier.  When a frontier is empty the
// level rises to the minimum remaining support.
//
// Device-driven rounds.  A round is two kernels that read their sizes from
// a control block, so rounds are replayed from a captured HIP graph with
// no host round trip:
//   k_phase_a  normal round: the frontier edges' links, 64 per work item;
//              gather round (first round of a level): the frontier becomes
//              the active edges with support <= level, and the active set
//              is compacted;
//   k_phase_b  touched blooms, 64 wedges per work item; the last block to
//              finish picks the next round: normal while a frontier exists,
//              else a gather round at level + 1 (or, when a gather finds
//              nothing, at the smallest support it saw).
// One element per lane keeps every wave's chain of dependent atomics short.
// The active set holds the remaining edges with support below a threshold T
// (a decrement that crosses T appends the edge).  When no active edge
// remains the device raises `stall` and the host rebuilds the set with a
// larger T from a histogram of the remaining supports.  Lists that one
// round fills and the next consumes are double-buffered by round parity;
// every counter is reset by a kernel that does not read it.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pipeline.h"

namespace bt {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLinkChunk = kWave;   // links per phase-A work item (one per lane)
constexpr int kWedgeChunk = kWave;  // wedges per phase-B work item (one per lane)
int grid_a() {
    static int g = std::getenv("BT_PEEL_GRID_A") ? std::atoi(std::getenv("BT_PEEL_GRID_A")) : 2048;
    return g;
}
int grid_b() {
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
    // Round state, indexed by round parity.  Phase A of round r derives its
    // own entry from round r - 1's final counters (every block computes the
    // same values; block 0 stores them for phase B and for round r + 1).
    int32_t mode[2];    // kNormal or kGather
    int32_t level[2];
    int32_t cur[2];     // active-set buffer in use
    int32_t gmin[2];    // gather rounds: minimum support above the level
    int32_t stall;
    int32_t thresh;     // active threshold T
    int32_t max_level;  // largest level at which edges were removed
    int32_t pad;        // persistent kernel: parity of the next round
    u64 rounds, levels;
    u64 prof[6];        // persistent kernel, BT_PEEL_PROFILE=1: block-0 clock ticks
};

struct FrontItem {
    int32_t e;
    int32_t first;    // 1 for the edge's first chunk: assigns phi
    uint32_t lo, hi;  // link positions of this chunk
};

struct BloomItem {
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
    const uint2 *link;  // {wedge, bloom}
    FrontItem *front[2];
    BloomItem *tc[2];
    int32_t *act[2];
};

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

// Append frontier work items (64-link chunks of edge e) where `take`.
__device__ __forceinline__ void push_front(bool take, int32_t e, const PeelArgs &P, int q) {
    uint32_t lo = 0, hi = 0, k = 0;
    if (take) {
        lo = (uint32_t)P.link_off[e];
        hi = (uint32_t)P.link_off[(int64_t)e + 1];
        k = hi - lo <= (uint32_t)kLinkChunk ? 1u : (hi - lo + kLinkChunk - 1) / kLinkChunk;
    }
    const u64 base = wave_alloc(k, &P.ctl->nf[q].v);
    for (uint32_t c = 0; c < k; ++c) {
        const uint32_t a = lo + c * kLinkChunk;
        P.front[q][base + c] = FrontItem{e, c == 0 ? 1 : 0, a, min(a + (uint32_t)kLinkChunk, hi)};
    }
}

// Lower supports by d where `active`; both atomics issue before either
// result is used.  Crossings of the level go to the next frontier, of the
// threshold to the active set.
__device__ __forceinline__ void dec_support2(bool act1, int32_t e1, bool act2, int32_t e2,
                                             int32_t d, int32_t level, int32_t thresh,
                                             const PeelArgs &P, int q, int cur) {
    int32_t o1 = 0, o2 = 0;
    if (act1) o1 = atomicSub(&P.sup[e1], d);
    if (act2) o2 = atomicSub(&P.sup[e2], d);
    const bool f1 = act1 && o1 > level && o1 - d <= level;
    const bool f2 = act2 && o2 > level && o2 - d <= level;
    const bool a1 = act1 && o1 >= thresh && o1 - d < thresh;
    const bool a2 = act2 && o2 >= thresh && o2 - d < thresh;
    push_front(f1, e1, P, q);
    push_front(f2, e2, P, q);
    const u64 slot = wave_alloc((a1 ? 1u : 0u) + (a2 ? 1u : 0u), &P.ctl->na[cur].v);
    if (a1) P.act[cur][slot] = e1;
    if (a2) P.act[cur][slot + (a1 ? 1 : 0)] = e2;
}

template <typename T> __device__ __forceinline__ T ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Round {
    int32_t mode, level, cur;
    u64 nf;  // frontier work items (normal rounds)
};

// Decide round r (parity p) from round r - 1's final counters.  Every
// caller computes the same result; the lead stores it for phase B and for
// round r + 1.  Returns false when the active set has run out (stall): the
// host then rebuilds it, or finds that no edge remains.
__device__ __forceinline__ bool decide_round(PeelCtl *C, int p, bool lead, Round &R) {
    const int q = p ^ 1;
    const int32_t pmode = ld(&C->mode[q]), plevel = ld(&C->level[q]), pcur = ld(&C->cur[q]);
    const int32_t pgmin = ld(&C->gmin[q]);
    const u64 nfp = ld(&C->nf[p].v);
    R.cur = pmode == kGather ? pcur ^ 1 : pcur;
    R.nf = nfp;
    if (nfp > 0) {
        R.mode = kNormal;
        R.level = plevel;
    } else if (pmode == kGather) {
        if (pgmin == INT_MAX) {  // no active edge left (or none at all)
            if (lead) C->stall = 1;
            return false;
        }
        R.mode = kGather;
        R.level = pgmin;  // jump to the smallest support the gather saw
    } else {
        R.mode = kGather;
        R.level = plevel + 1;
    }
    if (lead) {
        C->mode[p] = R.mode;
        C->level[p] = R.level;
        C->cur[p] = R.cur;
        C->ntc[q].v = 0;
        C->rounds += 1;
        if (pmode == kGather && nfp > 0) C->levels += 1;
        if (R.mode == kNormal && R.level > C->max_level) C->max_level = R.level;
    }
    return true;
}

// Phase A.  Normal round: remove the frontier edges' wedges.  Gather round
// (first round of a level): frontier = active edges with support <= level,
// queued for the next round, while the active set is compacted into the
// other buffer.  Work is spread over waves [wid, +nwaves).
__device__ __forceinline__ void phase_a_work(const PeelArgs &P, int p, const Round &R,
                                             int64_t wid, int64_t nwaves, u64 &upd) {
    PeelCtl *C = P.ctl;
    const int q = p ^ 1;
    const int32_t level = R.level;
    const int cur = R.cur;
    const int32_t thresh = C->thresh;
    if (R.mode == kGather) {
        const int64_t na = (int64_t)ld(&C->na[cur].v);
        int32_t mn = INT_MAX;
        for (int64_t i0 = wid * kWave; i0 < na; i0 += nwaves * kWave) {
            const int64_t i = i0 + lane_id();
            bool take = false, keep = false;
            int32_t e = 0;
            if (i < na) {
                e = P.act[cur][i];
                if (P.phi[e] < 0) {
                    const int32_t sv = P.sup[e];
                    take = sv <= level;
                    keep = !take;
                    if (keep) mn = min(mn, sv);
                }
            }
            push_front(take, e, P, q);
            const u64 slot = wave_alloc(keep ? 1u : 0u, &C->na[cur ^ 1].v);
            if (keep) P.act[cur ^ 1][slot] = e;
        }
        mn = wave_min(mn);
        if (lane_id() == 0 && mn != INT_MAX) atomicMin(&C->gmin[p], mn);
        return;
    }
    const int64_t nf = (int64_t)R.nf;
    int64_t i = wid;
    FrontItem it{};
    if (i < nf) it = P.front[p][i];
    while (i < nf) {
        const int64_t inext = i + nwaves;
        FrontItem nx{};
        if (inext < nf) nx = P.front[p][inext];  // next item, loaded early
        const int32_t e = it.e;
        if (it.first && lane_id() == 0) P.phi[e] = level;
        const uint32_t j = it.lo + lane_id();
        const uint32_t l1 = it.hi;
        bool won = false;
        int32_t blm = 0, twin = 0, d = 0;
        uint32_t w0 = 0, w1 = 0;
        if (j < l1) {
            const uint2 lk = P.link[j];
            const uint32_t w = lk.x;
            blm = (int32_t)lk.y;
            const uint32_t bit = 1u << (w & 31);
            const uint32_t old = atomicAnd(&P.alive[w >> 5], ~bit);
            const int32_t ea = P.wea[w], eb = P.web[w];
            const int32_t kb = P.bk[blm];
            const uint32_t b0 = P.bwoff[blm], b1 = P.bwoff[blm + 1];
            if (old & bit) {
                won = true;
                twin = ea == e ? eb : ea;
                d = kb - 1;
                w0 = b0;
                w1 = b1;
            }
        }
        // First kill in the bloom this round queues the bloom for phase B;
        // the twin loses its k - 1 butterflies in the bloom.
        bool first = false;
        int32_t otw = 0;
        const bool dec = won && d > 0;
        if (won) first = atomicAdd(&P.bc[blm], 1) == 0;
        if (dec) otw = atomicSub(&P.sup[twin], d);
        const uint32_t nch = first ? (w1 - w0 + kWedgeChunk - 1) / kWedgeChunk : 0u;
        const u64 cbase = wave_alloc(nch, &C->ntc[p].v);
        for (uint32_t c = 0; c < nch; ++c) {
            const uint32_t a = w0 + c * kWedgeChunk;
            P.tc[p][cbase + c] = BloomItem{blm, (int32_t)nch, a, min(a + (uint32_t)kWedgeChunk, w1)};
        }
        const bool tf = dec && otw > level && otw - d <= level;
        const bool ta = dec && otw >= thresh && otw - d < thresh;
        push_front(tf, twin, P, q);
        const u64 slot = wave_alloc(ta ? 1u : 0u, &C->na[cur].v);
        if (ta) P.act[cur][slot] = twin;
        upd += dec ? 1 : 0;
        it = nx;
        i = inext;
    }
}

// Phase B: survivors of every touched bloom lose C[B]; the last chunk of a
// bloom to finish sets k[B] -= C[B], C[B] = 0.  The lead clears counters
// this round consumed (none of them is read in this phase).
__device__ __forceinline__ void phase_b_work(const PeelArgs &P, int p, const Round &R,
                                             int64_t wid, int64_t nwaves, bool lead, u64 &upd,
                                             u64 &visits) {
    PeelCtl *C = P.ctl;
    const int q = p ^ 1;
    const int32_t level = R.level;
    const int cur = R.cur;
    if (lead) {
        C->nf[p].v = 0;
        C->gmin[q] = INT_MAX;
        if (R.mode == kGather) C->na[cur].v = 0;  // compacted into the other buffer
    }
    if (R.mode == kGather) return;
    const int32_t thresh = C->thresh;
    const int64_t ntc = (int64_t)ld(&C->ntc[p].v);
    int64_t i = wid;
    BloomItem it{};
    if (i < ntc) it = P.tc[p][i];
    while (i < ntc) {
        const int64_t inext = i + nwaves;
        BloomItem nx{};
        if (inext < ntc) nx = P.tc[p][inext];  // next item, loaded early
        const int32_t b = it.b;
        const uint32_t w = it.lo + lane_id();
        const bool inr = w < it.hi;
        const uint32_t word = inr ? P.alive[w >> 5] : 0u;
        int32_t ea = 0, eb = 0;
        if (inr) {
            ea = P.wea[w];
            eb = P.web[w];
        }
        const int32_t c = P.bc[b];
        const int32_t kn = P.bk[b] - c;
        const bool live = inr && kn > 0 && ((word >> (w & 31)) & 1u);
        dec_support2(live, ea, live, eb, c, level, thresh, P, q, cur);
        upd += live ? 2 : 0;
        if (live && kn <= 1) atomicAnd(&P.alive[w >> 5], ~(1u << (w & 31)));
        if (lane_id() == 0) {
            if (it.nch == 1 || atomicAdd(&P.bdone[b], 1) == it.nch - 1) {
                P.bk[b] = kn;
                P.bc[b] = 0;
                P.bdone[b] = 0;
                visits += 1;
            }
        }
        it = nx;
        i = inext;
    }
}

// Adds per-lane statistics to the control block (one atomic per wave).
__device__ __forceinline__ void flush_stats(PeelCtl *C, u64 upd, u64 visits) {
    upd = wave_sum(upd);
    visits = wave_sum(visits);
    if (lane_id() == 0) {
        if (upd) atomicAdd(&C->updates.v, upd);
        if (visits) atomicAdd(&C->bloom_visits.v, visits);
    }
}

// --- one kernel per phase (rounds replayed from a captured HIP graph) ---

__global__ __launch_bounds__(kBlock) void k_phase_a(PeelArgs P, int p) {
    PeelCtl *C = P.ctl;
    if (C->stall) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    Round R;
    if (!decide_round(C, p, lead, R)) return;
    u64 upd = 0;
    phase_a_work(P, p, R, blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave,
                 (int64_t)gridDim.x * kWavesPerBlock, upd);
    flush_stats(C, upd, 0);
}

__global__ __launch_bounds__(kBlock) void k_phase_b(PeelArgs P, int p) {
    PeelCtl *C = P.ctl;
    if (C->stall) return;
    Round R;
    R.mode = C->mode[p];
    R.level = C->level[p];
    R.cur = C->cur[p];
    R.nf = 0;
    u64 upd = 0, visits = 0;
    phase_b_work(P, p, R, blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave,
                 (int64_t)gridDim.x * kWavesPerBlock, blockIdx.x == 0 && threadIdx.x == 0, upd,
                 visits);
    flush_stats(C, upd, visits);
}

// --- persistent cooperative kernel: rounds separated by grid barriers ---

constexpr int kPBlock = 512;

struct GridBar {
    Counter group[8];
    Counter top;
    Counter gen;
    int32_t fail;
};

// Two-level barrier: blocks arrive at one of eight group counters, the last
// of each group at the top counter, and the last of those opens the next
// generation.  Release and acquire fences make every block's writes before
// the barrier visible to every block after it.  A waiter gives up after a
// bounded spin (the kernel then stops with `fail` set) so no bug can hang
// the device.
__device__ bool grid_sync(GridBar *B, u64 &gen_local) {
    __shared__ int ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        const unsigned nb = gridDim.x;
        const unsigned g = blockIdx.x & 7;
        const unsigned ngroups = nb < 8 ? nb : 8;
        const unsigned gsize = (nb - g + 7) / 8;
        bool opener = false;
        if (atomicAdd(&B->group[g].v, 1ull) == gsize - 1) {
            __hip_atomic_store(&B->group[g].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            if (atomicAdd(&B->top.v, 1ull) == ngroups - 1) {
                __hip_atomic_store(&B->top.v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
                atomicAdd(&B->gen.v, 1ull);
                opener = true;
            }
        }
        if (!opener) {
            int64_t spins = 0;
            while (ld(&B->gen.v) == gen_local) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (int64_t(1) << 28) || ld(&B->fail)) {
                    __hip_atomic_store(&B->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        gen_local += 1;
        __threadfence();
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

__global__ __launch_bounds__(kPBlock) void k_peel_persistent(PeelArgs P, GridBar *B,
                                                             int64_t max_rounds, int prof) {
    PeelCtl *C = P.ctl;
    u64 gen_local = 0;
    if (threadIdx.x == 0) gen_local = ld(&B->gen.v);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const int64_t wid = blockIdx.x * (int64_t)(kPBlock / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kPBlock / kWave);
    int p = 0;
    u64 t[5] = {0, 0, 0, 0, 0}, acc[6] = {0, 0, 0, 0, 0, 0};
    u64 upd = 0, visits = 0;
    for (int64_t r = 0; r < max_rounds; ++r) {
        if (prof && lead) t[0] = wall_clock64();
        Round R;
        if (!decide_round(C, p, lead, R)) break;
        phase_a_work(P, p, R, wid, nwaves, upd);
        if (prof && lead) t[1] = wall_clock64();
        if (!grid_sync(B, gen_local)) break;
        if (prof && lead) t[2] = wall_clock64();
        phase_b_work(P, p, R, wid, nwaves, lead, upd, visits);
        if (prof && lead) t[3] = wall_clock64();
        if (!grid_sync(B, gen_local)) break;
        if (prof && lead) {
            t[4] = wall_clock64();
            for (int k = 0; k < 4; ++k) acc[k] += t[k + 1] - t[k];
            if (R.mode == kGather) {
                acc[4] += t[2] - t[0];
                acc[5] += 1;
            }
        }
        p ^= 1;
    }
    flush_stats(C, upd, visits);
    if (lead) {
        C->pad = p;
        for (int k = 0; k < 6; ++k) C->prof[k] += acc[k];
    }
}

// ---------------------------------------------------------------- refill

__global__ __launch_bounds__(kBlock) void k_refill_compact(const int32_t *list, int64_t n,
                                                           const int32_t *phi, const int32_t *sup,
                                                           int32_t *out, u64 *nout,
                                                           int32_t *min_out) {
    int32_t mn = INT_MAX;
    const int64_t nthr = (int64_t)gridDim.x * kBlock;
    for (int64_t i0 = blockIdx.x * (int64_t)kBlock + (threadIdx.x & ~(kWave - 1)); i0 < n;
         i0 += nthr) {
        const int64_t i = i0 + lane_id();
        bool keep = false;
        int32_t e = 0;
        if (i < n) {
            e = list ? list[i] : (int32_t)i;
            keep = phi[e] < 0;
            if (keep) mn = min(mn, sup[e]);
        }
        const u64 slot = wave_alloc(keep ? 1u : 0u, nout);
        if (keep) out[slot] = e;
    }
    mn = wave_min(mn);
    if (lane_id() == 0 && mn != INT_MAX) atomicMin(min_out, mn);
}

__global__ __launch_bounds__(kBlock) void k_refill_hist(const int32_t *list, int64_t n,
                                                        const int32_t *sup, int32_t mn,
                                                        u64 *hist) {
    __shared__ u64 h[33];
    if (threadIdx.x < 33) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const uint32_t d = (uint32_t)(sup[list[i]] - mn) + 1u;
        atomicAdd(&h[31 - __clz(d)], 1ull);
    }
    __syncthreads();
    if (threadIdx.x < 33 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(kBlock) void k_refill_gather(const int32_t *list, int64_t n,
                                                          const int32_t *sup, int32_t thresh,
                                                          int32_t *act, u64 *na) {
    const int64_t nthr = (int64_t)gridDim.x * kBlock;
    for (int64_t i0 = blockIdx.x * (int64_t)kBlock + (threadIdx.x & ~(kWave - 1)); i0 < n;
         i0 += nthr) {
        const int64_t i = i0 + lane_id();
        bool take = false;
        int32_t e = 0;
        if (i < n) {
            e = list[i];
            take = sup[e] < thresh;
        }
        const u64 slot = wave_alloc(take ? 1u : 0u, na);
        if (take) act[slot] = e;
    }
}

__global__ void k_init_peel(const uint64_t *supl, int64_t m, int32_t *sup, int32_t *phi,
                            int64_t *sup_out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = (int32_t)(supl[e] & 0xffffffffu);
        sup[e] = s;
        phi[e] = -1;
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

// ----------------------------------------------------------- host side

void launch_round(const PeelArgs &P, int p, hipStream_t s) {
    k_phase_a<<<grid_a(), kBlock, 0, s>>>(P, p);
    k_phase_b<<<grid_b(), kBlock, 0, s>>>(P, p);
}

// Captured chunks of `rounds` rounds, cached in the workspace by argument
// bytes.
hipGraphExec_t chunk_graph(const PeelArgs &P, int rounds, Workspace &ws) {
    std::vector<unsigned char> key(sizeof(PeelArgs));
    std::memcpy(key.data(), &P, sizeof(PeelArgs));
    auto &cache = ws.graphs;
    for (auto &g : cache)
        if (g.rounds == rounds && g.key == key) return g.exec;
    if (cache.size() >= 16) {
        (void)hipGraphExecDestroy(cache.front().exec);
        cache.erase(cache.begin());
    }
    hipStream_t cs;
    BT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g;
    BT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < rounds; ++r) launch_round(P, r & 1, cs);
    BT_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t ex;
    BT_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    cache.push_back(Workspace::GraphEntry{key, rounds, ex});
    return ex;
}

}  // namespace

void peel(const RankCSR &r, IndexArrays &ix, int64_t *sup_out, int64_t *phi_out,
          PeelCounters &pc, Workspace &ws, hipStream_t s) {
    const int64_t m = r.m;
    if (m == 0) return;
    if (2 * ix.n_w >= (int64_t)UINT32_MAX)
        throw Error{BT_EOVERFLOW, "edge-to-wedge links must be below 2^32"};
    const int64_t nb = ix.n_b > 0 ? ix.n_b : 1;
    const int64_t words = (ix.n_w + 31) / 32 + 1;
    const int64_t max_tc = nb + ix.n_w / kWedgeChunk + 1;
    const int64_t max_front = m + 2 * ix.n_w / kLinkChunk + 1;

    PeelArgs P{};
    P.sup = ws.get<int32_t>("peel_sup", m);
    P.phi = ws.get<int32_t>("peel_phi", m);
    P.alive = ws.get<uint32_t>("peel_alive", words);
    P.bc = ws.get<int32_t>("peel_bc", nb);
    P.bdone = ws.get<int32_t>("peel_bdone", nb);
    P.bk = ix.bk;
    P.bwoff = ix.bwoff;
    P.wea = ix.wea;
    P.web = ix.web;
    P.wbl = ix.wbl;
    P.link_off = ix.link_off;
    P.link = ix.link;
    P.front[0] = ws.get<FrontItem>("peel_front0", max_front);
    P.front[1] = ws.get<FrontItem>("peel_front1", max_front);
    P.tc[0] = ws.get<BloomItem>("peel_tc0", max_tc);
    P.tc[1] = ws.get<BloomItem>("peel_tc1", max_tc);
    P.act[0] = ws.get<int32_t>("peel_act0", m);
    P.act[1] = ws.get<int32_t>("peel_act1", m);
    P.ctl = ws.get<PeelCtl>("peel_ctl", 1);
    int32_t *glist[2] = {ws.get<int32_t>("peel_all0", m), ws.get<int32_t>("peel_all1", m)};
    u64 *rs = ws.get<u64>("peel_refill", 40);  // [0] count, [1] min, [2..34] histogram

    k_init_peel<<<grid_for(m, 256, 16384), 256, 0, s>>>(ix.supl, m, P.sup, P.phi, sup_out);
    BT_CHECK_LAUNCH();
    k_init_alive<<<grid_for(words, 256, 16384), 256, 0, s>>>(ix.cursor, P.alive);
    BT_CHECK_LAUNCH();
    BT_HIP(hipMemsetAsync(P.bc, 0, sizeof(int32_t) * nb, s));
    BT_HIP(hipMemsetAsync(P.bdone, 0, sizeof(int32_t) * nb, s));
    PeelCtl init{};
    init.gmin[0] = init.gmin[1] = INT_MAX;
    BT_HIP(hipMemcpyAsync(P.ctl, &init, sizeof init, hipMemcpyHostToDevice, s));

    PeelCtl *hc = reinterpret_cast<PeelCtl *>(ws.host((int)(sizeof(PeelCtl) / 8 + 40)));
    u64 *hr = reinterpret_cast<u64 *>(hc + 1);
    // BT_PEEL_MODE=graph replays captured two-kernel rounds instead of the
    // persistent kernel; BT_PEEL_GRAPH=0 launches those rounds directly.
    const char *mv = std::getenv("BT_PEEL_MODE");
    const bool persistent = ws.coop && !(mv && std::strcmp(mv, "graph") == 0);
    const char *gv = std::getenv("BT_PEEL_GRAPH");
    const bool use_graph = !(gv && std::atoi(gv) == 0);
    GridBar *bar = ws.get<GridBar>("peel_bar", 1);
    BT_HIP(hipMemsetAsync(bar, 0, sizeof(GridBar), s));
    int pblocks = 0;
    if (persistent) {
        int dev = 0, cus = 0, occ = 0;
        BT_HIP(hipGetDevice(&dev));
        BT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_peel_persistent, kPBlock, 0));
        const char *pb = std::getenv("BT_PEEL_PBLOCKS");
        pblocks = pb ? std::atoi(pb) : 96;
        pblocks = std::max(1, std::min(pblocks, occ * cus));
    }

    hipEvent_t ev0, ev1;  // around each peel launch: the kernel's device time
    BT_HIP(hipEventCreate(&ev0));
    BT_HIP(hipEventCreate(&ev1));
    struct EvFree {
        hipEvent_t a, b;
        ~EvFree() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev_free{ev0, ev1};
    int64_t n_all = m;
    int cur = -1;  // -1: all edges, in id order
    int chunk = 4;
    bool need_refill = true;
    for (int64_t guard = 0;; ++guard) {
        if (need_refill) {
            // Rebuild the active set: compact the remaining edges, find their
            // minimum support, histogram supports above it, pick T so that
            // the set holds a few percent of the remaining edges.
            const int nxt = cur < 0 ? 0 : cur ^ 1;
            BT_HIP(hipMemsetAsync(rs, 0, sizeof(u64) * 40, s));
            fill_i32(reinterpret_cast<int32_t *>(rs + 1), INT_MAX, 1, s);
            k_refill_compact<<<grid_for(n_all, kBlock, 4096), kBlock, 0, s>>>(
                cur < 0 ? nullptr : glist[cur], n_all, P.phi, P.sup, glist[nxt], rs,
                reinterpret_cast<int32_t *>(rs + 1));
            BT_CHECK_LAUNCH();
            BT_HIP(hipMemcpyAsync(hr, rs, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            cur = nxt;
            n_all = (int64_t)hr[0];
            if (n_all == 0) break;
            const int32_t mn = *reinterpret_cast<int32_t *>(hr + 1);
            k_refill_hist<<<grid_for(n_all, kBlock, 2048), kBlock, 0, s>>>(glist[cur], n_all,
                                                                          P.sup, mn, rs + 2);
            BT_CHECK_LAUNCH();
            BT_HIP(hipMemcpyAsync(hr + 2, rs + 2, 33 * sizeof(u64), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            const int64_t target = std::max<int64_t>(65536, n_all / 32);
            int64_t thresh = INT_MAX, acc = 0;
            for (int b = 0; b < 33; ++b) {
                acc += (int64_t)hr[2 + b];
                if (acc >= target) {
                    thresh = std::min<int64_t>((int64_t)mn + (int64_t(2) << b) - 1, INT_MAX);
                    break;
                }
            }
            BT_HIP(hipMemsetAsync(&P.ctl->na[0].v, 0, sizeof(u64), s));
            k_refill_gather<<<grid_for(n_all, kBlock, 4096), kBlock, 0, s>>>(
                glist[cur], n_all, P.sup, (int32_t)thresh, P.act[0], &P.ctl->na[0].v);
            BT_CHECK_LAUNCH();
            // Round state back to a clean start: a gather round at the
            // minimum remaining support.
            BT_HIP(hipMemcpyAsync(hc, P.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            PeelCtl st = *hc;
            // As if the previous round (parity 1) were a gather that found
            // no frontier and saw minimum support mn in buffer 0.
            st.nf[0].v = st.nf[1].v = st.ntc[0].v = st.ntc[1].v = 0;
            st.na[1].v = 0;
            st.mode[1] = kGather;
            st.cur[1] = 1;
            st.gmin[1] = mn;
            st.gmin[0] = INT_MAX;
            st.stall = 0;
            st.thresh = (int32_t)thresh;
            BT_HIP(hipMemcpyAsync(P.ctl, &st, sizeof st, hipMemcpyHostToDevice, s));
            need_refill = false;
        }
        BT_HIP(hipEventRecord(ev0, s));
        if (persistent) {
            int64_t max_rounds = 4 * m + 64;
            int prof = std::getenv("BT_PEEL_PROFILE") ? 1 : 0;
            void *args[] = {&P, &bar, &max_rounds, &prof};
            BT_HIP(hipLaunchCooperativeKernel((const void *)k_peel_persistent, dim3(pblocks),
                                              dim3(kPBlock), args, 0, s));
        } else if (use_graph) {
            BT_HIP(hipGraphLaunch(chunk_graph(P, chunk, ws), s));
        } else {
            for (int rr = 0; rr < chunk; ++rr) launch_round(P, rr & 1, s);
            BT_CHECK_LAUNCH();
        }
        BT_HIP(hipEventRecord(ev1, s));
        BT_HIP(hipMemcpyAsync(hc, P.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
        BT_HIP(hipStreamSynchronize(s));
        {
            float t = 0.f;
            BT_HIP(hipEventElapsedTime(&t, ev0, ev1));
            pc.kernel_ms += t;
            pc.launches += 1;
        }
        if (persistent) {
            int32_t fail = 0;
            BT_HIP(hipMemcpy(&fail, &bar->fail, sizeof fail, hipMemcpyDeviceToHost));
            if (fail) throw Error{BT_EDEVICE, "peel grid barrier timed out"};
            if (!hc->stall) throw Error{BT_EDEVICE, "peel stopped early"};
        }
        if (hc->stall) need_refill = true;
        chunk = std::min(chunk * 2, 64);
        if (guard > 4 * m + 64) throw Error{BT_EDEVICE, "peel made no progress"};
    }
    BT_HIP(hipMemcpyAsync(hc, P.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    pc.levels = (int64_t)hc->levels;
    pc.rounds = (int64_t)hc->rounds;
    pc.max_phi = hc->max_level;
    pc.updates = (int64_t)hc->updates.v;
    pc.bloom_visits = (int64_t)hc->bloom_visits.v;
    if (std::getenv("BT_PEEL_PROFILE"))
        std::fprintf(stderr, "[peel] rounds %llu  block0 us: phaseA %.0f bar1 %.0f phaseB %.0f bar2 %.0f; gather rounds %llu phaseA+bar1 %.0f\n",
                     hc->rounds, hc->prof[0] / 100.0, hc->prof[1] / 100.0, hc->prof[2] / 100.0,
                     hc->prof[3] / 100.0, hc->prof[5], hc->prof[4] / 100.0);
    k_phi_out<<<grid_for(m, 256, 16384), 256, 0, s>>>(P.phi, phi_out, m);
    BT_CHECK_LAUNCH();
}

}  // namespace bt
