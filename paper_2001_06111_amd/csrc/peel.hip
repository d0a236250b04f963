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
// most L puts the edge in the next frontier (and fixes its phi = L: the
// next round keeps the level).  When a frontier is empty the level rises to
// the minimum remaining support.
//
// Device-driven rounds.  The default is one persistent cooperative kernel
// whose rounds are separated by grid barriers; the alternative is two
// kernels per round replayed from a captured HIP graph (used where the
// peel shares the device with other work).  Either way:
//   phase A  normal round: the frontier edges' links, 64 per work item;
//            gather round (first round of a level): the frontier becomes
//            the active edges with support <= level, and the active set is
//            compacted;
//   phase B  touched blooms, 64 wedges per work item.
// After each round one thread per block derives the next round from the
// control block: normal while a frontier exists, else a gather at level + 1
// (or, when a gather finds nothing, at the smallest support it saw).
// Rounds are chains of dependent memory accesses, so the kernels keep those
// chains short: one element per lane, independent accesses issued
// together, small rounds spread over many CUs.
// The active set holds the remaining edges with support below a threshold T
// (a decrement that crosses T appends the edge).  When no active edge
// remains, the persistent kernel rebuilds the set itself with a larger T
// from a histogram of the remaining supports (in the two-kernel form the
// device raises `stall` and the host rebuilds it), so one launch peels the
// whole graph.  Lists that one round fills and the next consumes are
// double-buffered by round parity; every counter is reset in a phase that
// does not read it.
// An ablation mode (`unit`) drops batch bloom processing: each survivor
// takes C[B] decrements of one instead of one decrement of C[B].
// Batches of graphs peel in k_peel_multi, each graph at its own level.
#include <condition_variable>
#include <map>
#include <memory>

#include "peel_common.h"

namespace bt {

namespace {

// Turns of the cooperative peels: tickets in asking order, the waiting
// tickets with their weights (edges), and the yield word the holder's
// kernel reads.  Never destroyed: it outlives static teardown.
struct Gate {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t next = 0;
    bool busy = false;
    int64_t holder_weight = 0;
    std::map<uint64_t, int64_t> waiting;
    int32_t *word = nullptr;  // pinned, coherent: [0] yield request, [1] always 1
    int32_t *dword = nullptr;  // its device address
};

constexpr int64_t kYieldRatio = 8;

Gate &gate() {
    static Gate *g = new Gate();
    return *g;
}

// Under g.mu: raise the yield word when some waiter is much lighter than
// the holder, clear it otherwise.
void update_yield(Gate &g) {
    bool ask = false;
    if (g.busy)
        for (const auto &w : g.waiting)
            if (w.second * kYieldRatio < g.holder_weight) {
                ask = true;
                break;
            }
    if (!g.word) return;
    static const bool verbose = std::getenv("BT_PEEL_VERBOSE") != nullptr;
    if (verbose && (g.word[0] != 0) != ask)
        std::fprintf(stderr, "[peel] yield word %d (holder weight %lld, %zu waiting)\n", ask ? 1 : 0,
                     (long long)g.holder_weight, g.waiting.size());
    __atomic_store_n(&g.word[0], ask ? 1 : 0, __ATOMIC_RELEASE);
}

// Under g.mu, with `ticket` in g.waiting: waits for it to be the oldest
// waiter while the device is free, then takes the turn.
void take_turn(Gate &g, std::unique_lock<std::mutex> &lk, uint64_t ticket, int64_t weight) {
    update_yield(g);
    g.cv.wait(lk, [&] { return !g.busy && g.waiting.begin()->first == ticket; });
    g.waiting.erase(ticket);
    g.busy = true;
    g.holder_weight = weight;
    update_yield(g);
}

}  // namespace

namespace {
thread_local int64_t t_turn_weight = -1;
}  // namespace

void set_turn_weight(int64_t w) { t_turn_weight = w; }

CoopTurn::CoopTurn(int64_t weight) : weight_(t_turn_weight >= 0 ? t_turn_weight : weight) {
    Gate &g = gate();
    std::unique_lock<std::mutex> lk(g.mu);
    if (!g.word) {
        void *h = nullptr, *d = nullptr;
        BT_HIP(hipHostMalloc(&h, 2 * sizeof(int32_t),
                             hipHostMallocMapped | hipHostMallocCoherent));
        BT_HIP(hipHostGetDevicePointer(&d, h, 0));
        g.word = static_cast<int32_t *>(h);
        g.word[0] = 0;
        g.word[1] = 1;
        g.dword = static_cast<int32_t *>(d);
    }
    ticket_ = g.next++;
    g.waiting[ticket_] = weight_;
    take_turn(g, lk, ticket_, weight_);
}

CoopTurn::~CoopTurn() {
    Gate &g = gate();
    std::lock_guard<std::mutex> lk(g.mu);
    g.busy = false;
    g.holder_weight = 0;
    update_yield(g);
    g.cv.notify_all();
}

const int32_t *CoopTurn::yield_word(bool force) const { return gate().dword + (force ? 1 : 0); }

void CoopTurn::requeue() {
    Gate &g = gate();
    std::unique_lock<std::mutex> lk(g.mu);
    g.busy = false;
    g.holder_weight = 0;
    ticket_ = g.next++;
    g.waiting[ticket_] = weight_;
    g.cv.notify_all();
    take_turn(g, lk, ticket_, weight_);
}

namespace {

// Round parameters.  One thread per block reads them from the control block
// after each barrier and hands them to the block through LDS, so the
// control block sees one request per block, not one per wave.
struct Round {
    int32_t mode, level, cur, thresh;
    u64 nf;   // frontier work items (normal rounds)
    u64 na;   // active-set entries (gather rounds)
    u64 ntc;  // bloom work items (phase B; read after the first barrier)
};

// Round counters kept in the lead's registers while it runs.
struct LeadStats {
    u64 rounds, levels;
    int32_t max_level;
    __device__ void load(PeelCtl *C) {
        rounds = ld(&C->rounds);
        levels = ld(&C->levels);
        max_level = ld(&C->max_level);
    }
    __device__ void store(PeelCtl *C) const {
        st(&C->rounds, rounds);
        st(&C->levels, levels);
        st(&C->max_level, max_level);
    }
};

// Decide round r (parity p) from round r - 1's final counters.  Every block
// computes the same result; the lead stores it for round r + 1.  Returns
// false when the active set has run out (stall): the host then rebuilds it,
// or finds that no edge remains.
__device__ __forceinline__ bool decide_round(PeelCtl *C, int p, bool lead, Round &R,
                                             LeadStats &L, int prof) {
    const int q = p ^ 1;
    const int32_t pmode = ld(&C->mode[q]), plevel = ld(&C->level[q]), pcur = ld(&C->cur[q]);
    const int32_t pgmin = ld(&C->gmin[q]);
    const u64 nfp = ld(&C->nf[p].v);
    const u64 na0 = ld(&C->na[0].v), na1 = ld(&C->na[1].v);
    R.cur = pmode == kGather ? pcur ^ 1 : pcur;
    R.nf = nfp;
    R.thresh = ld(&C->thresh);
    R.ntc = 0;
    if (nfp > 0) {
        R.mode = kNormal;
        R.level = plevel;
    } else if (pmode == kGather) {
        if (pgmin == INT_MAX) {  // no active edge left (or none at all)
            if (lead) st(&C->stall, 1);
            return false;
        }
        R.mode = kGather;
        R.level = pgmin;  // jump to the smallest support the gather saw
    } else {
        R.mode = kGather;
        R.level = plevel + 1;
    }
    R.na = R.mode == kGather ? (R.cur ? na1 : na0) : 0;
    if (lead) {
        const u64 ntc_prev = prof ? ld(&C->ntc[q].v) : 0;
        st(&C->mode[p], R.mode);
        st(&C->level[p], R.level);
        st(&C->cur[p], R.cur);
        st(&C->ntc[q].v, (u64)0);
        L.rounds += 1;
        if (pmode == kGather && nfp > 0) L.levels += 1;
        if (R.mode == kNormal && R.level > L.max_level) L.max_level = R.level;
        if (prof) {
            const u64 pt = ld(&C->push_twin[p].v), ps = ld(&C->push_surv[p].v);
            st(&C->push_twin[p].v, (u64)0);
            st(&C->push_surv[p].v, (u64)0);
            st(&C->twin_pushes, ld(&C->twin_pushes) + pt);
            st(&C->surv_pushes, ld(&C->surv_pushes) + ps);
            if (pmode == kNormal && pt > 0 && ps == 0)
                st(&C->twin_only_rounds, ld(&C->twin_only_rounds) + 1);
            if (R.mode == kNormal) {
                const int bnf = 63 - __clzll(nfp | 1);
                st(&C->hist_nf[bnf], ld(&C->hist_nf[bnf]) + 1);
            }
            if (pmode == kNormal) {
                const int bntc = 63 - __clzll(ntc_prev | 1);
                st(&C->hist_ntc[bntc], ld(&C->hist_ntc[bntc]) + 1);
            }
        }
    }
    return true;
}

// Phase A.  Normal round: remove the frontier edges' wedges.  Gather round
// (first round of a level): frontier = active edges with support <= level,
// queued for the next round, while the active set is compacted into the
// other buffer.  Work is spread over waves [wid, +nwaves).  Memory
// operations that do not depend on each other are issued together: a round
// is a chain of dependent accesses, so the chain length sets its time.
__device__ __forceinline__ void phase_a_work(const PeelArgs &P, int p, const Round &R,
                                             int64_t wid, int64_t nwaves, u64 &upd) {
    PeelCtl *C = P.ctl;
    const int q = p ^ 1;
    const int32_t level = R.level;
    const int cur = R.cur;
    const int32_t thresh = R.thresh;
    if (R.mode == kGather) {
        // Block-strided, so the block can pool its compaction slots and its
        // minimum: one atomic per block instead of one per wave on each of
        // the two contended counters.
        __shared__ uint32_t s_wcnt[32];
        __shared__ u64 s_base;
        __shared__ int32_t s_min;
        const int64_t na = (int64_t)R.na;
        const int wv = threadIdx.x / kWave, nwv = blockDim.x / kWave;
        if (threadIdx.x == 0) s_min = INT_MAX;
        int32_t mn = INT_MAX;
        for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < na;
             i0 += (int64_t)gridDim.x * blockDim.x) {
            const int64_t i = i0 + threadIdx.x;
            bool take = false, keep = false;
            int32_t e = 0;
            if (i < na) {
                e = ld(&P.act[cur][i]);
                const int32_t ph = ld(&P.phi[e]);
                const int32_t sv = ld(&P.sup[e]);
                if (ph < 0) {
                    take = sv <= level;
                    keep = !take;
                    if (keep) mn = min(mn, sv);
                }
            }
            uint32_t lo = 0, hi = 0;
            if (take) {
                lo = (uint32_t)P.link_off[e];
                hi = (uint32_t)P.link_off[(int64_t)e + 1];
            }
            const uint32_t k = take ? link_chunks(lo, hi) : 0u;
            u64 base[3];
            wave_alloc3(k, &C->nf[q].v, 0u, nullptr, 0u, nullptr, base);
            put_front(P, q, base[0], e, lo, hi, k, level);
            const unsigned long long kb = __ballot(keep);
            if (lane_id() == 0) s_wcnt[wv] = (uint32_t)__popcll(kb);
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t t = 0;
                for (int w = 0; w < nwv; ++w) {
                    const uint32_t c = s_wcnt[w];
                    s_wcnt[w] = t;
                    t += c;
                }
                s_base = t ? atomicAdd(&C->na[cur ^ 1].v, (u64)t) : 0;
            }
            __syncthreads();
            if (keep)
                st(&P.act[cur ^ 1][s_base + s_wcnt[wv] + __popcll(kb & lanemask_lt())], e);
            __syncthreads();
        }
        mn = wave_min(mn);
        if (lane_id() == 0 && mn != INT_MAX) atomicMin(&s_min, mn);
        __syncthreads();
        if (threadIdx.x == 0 && s_min != INT_MAX) atomicMin(&C->gmin[p], s_min);
        return;
    }
    const int64_t nf = (int64_t)R.nf;
    int64_t i = wid;
    FrontItem it{};
    if (i < nf) it = ld_item(&P.front[p][i]);
    while (i < nf) {
        const int64_t inext = i + nwaves;
        FrontItem nx{};
        if (inext < nf) nx = ld_item(&P.front[p][inext]);  // next item, loaded early
        const uint32_t j = it.lo + lane_id();
        const bool has = j < it.hi;
        uint32_t bit = 0, old = 0, w0 = 0, w1 = 0, tlo = 0, thi = 0;
        int32_t blm = 0, twin = 0, kb = 0;
        bool tfix = false;
        if (has) {
            const uint3 lk = P.link[j];
            const uint32_t w = lk.x;
            blm = (int32_t)lk.y;
            twin = (int32_t)(lk.z & kEdgeMask);
            tfix = (lk.z & kFixedBit) != 0;
            bit = 1u << (w & 31);
            w0 = P.bwoff[blm];
            w1 = P.bwoff[blm + 1];
            kb = ld(&P.bk[blm]);
            // The twin's link range is fetched with the kill; it is used
            // only if the twin drops to the level.
            tlo = (uint32_t)P.link_off[twin];
            thi = (uint32_t)P.link_off[(int64_t)twin + 1];
            old = atomicAnd(&P.alive[w >> 5], ~bit);
        }
        // First kill in the bloom this round queues the bloom for phase B;
        // the twin loses its k - 1 butterflies in the bloom.
        // A live wedge's bloom holds at least two live wedges, so d >= 1.
        const bool won = has && (old & bit);
        const int32_t d = max(kb - 1, 0);
        const bool dec = won && d > 0 && !tfix;
        int32_t oc = 1, otw = 0;
        if (won) {  // both atomics issue before either result is used
            oc = atomicAdd(&P.bc[blm], 1);
            if (!tfix) otw = atomicSub(&P.sup[twin], d);
        }
        const bool first = oc == 0;
        const uint32_t nch = first ? (w1 - w0 + kWedgeChunk - 1) / kWedgeChunk : 0u;
        const bool tf = dec && otw > level && otw - d <= level;
        const bool ta = dec && otw >= thresh && otw - d < thresh;
        const uint32_t tk = tf ? link_chunks(tlo, thi) : 0u;
        if (P.prof) count_push(P, q, kSrcTwin, tf ? 1u : 0u);
        u64 base[3];
        wave_alloc3(nch, &C->ntc[p].v, tk, &C->nf[q].v, ta ? 1u : 0u, &C->na[cur].v, base);
        put_chunks(P.tc[p], base[0], nch, blm, (int32_t)nch, w0, w1);
        put_front(P, q, base[1], twin, tlo, thi, tk, level);
        if (ta) st(&P.act[cur][base[2]], twin);
        upd += dec ? 1 : 0;
        it = nx;
        i = inext;
    }
}

// Phase B: survivors of every touched bloom lose C[B]; the last chunk of a
// bloom to finish sets k[B] -= C[B], C[B] = 0.  The lead clears counters
// this round consumed (none of them is read in this phase).  A decrement
// that takes a support across the level queues the edge for the next
// round; across the threshold, adds it to the active set.
__device__ __forceinline__ void phase_b_work(const PeelArgs &P, int p, const Round &R,
                                             int64_t wid, int64_t nwaves, bool lead, u64 &upd,
                                             u64 &visits, u64 &unb, u64 &touch) {
    PeelCtl *C = P.ctl;
    const int q = p ^ 1;
    const int32_t level = R.level;
    const int cur = R.cur;
    if (lead) {
        st(&C->nf[p].v, (u64)0);
        st(&C->gmin[q], (int32_t)INT_MAX);
        if (R.mode == kGather) st(&C->na[cur].v, (u64)0);  // compacted into the other buffer
    }
    if (R.mode == kGather) return;
    const int32_t thresh = R.thresh;
    const int64_t ntc = (int64_t)R.ntc;
    int64_t i = wid;
    BloomItem it{};
    if (i < ntc) it = ld_item(&P.tc[p][i]);
    while (i < ntc) {
        const int64_t inext = i + nwaves;
        BloomItem nx{};
        if (inext < ntc) nx = ld_item(&P.tc[p][inext]);  // next item, loaded early
        const int32_t b = it.b;
        const uint32_t w = it.lo + lane_id();
        const bool inr = w < it.hi;
        uint32_t word = 0, ra = 0, rb = 0;
        if (inr) {
            ra = (uint32_t)P.wea[w];
            rb = (uint32_t)P.web[w];
            word = ld(&P.alive[w >> 5]);
        }
        const int32_t ea = (int32_t)(ra & kEdgeMask), eb = (int32_t)(rb & kEdgeMask);
        const int32_t c = ld(&P.bc[b]);
        const int32_t kn = ld(&P.bk[b]) - c;
        const bool live = inr && kn > 0 && ((word >> (w & 31)) & 1u);
        const bool da = live && !(ra & kFixedBit), db = live && !(rb & kFixedBit);
        bool f1 = false, f2 = false, a1 = false, a2 = false;
        if (live && P.unit) {
            // Ablation: each of the C[B] kills takes one unit from every
            // survivor, as removing the edges one at a time would.  Only the
            // unit decrement from level + 1 (from the threshold) reports the
            // crossing of the level (of the threshold).
            for (int32_t t = 0; t < c; ++t) {
                const int32_t u1 = da ? atomicSub(&P.sup[ea], 1) : 0;
                const int32_t u2 = db ? atomicSub(&P.sup[eb], 1) : 0;
                f1 |= da && u1 == level + 1;
                f2 |= db && u2 == level + 1;
                a1 |= da && u1 == thresh;
                a2 |= db && u2 == thresh;
            }
        } else {
            int32_t o1 = 0, o2 = 0;
            if (live) {
                if (da) o1 = atomicSub(&P.sup[ea], c);
                if (db) o2 = atomicSub(&P.sup[eb], c);
            }
            f1 = da && o1 > level && o1 - c <= level;
            f2 = db && o2 > level && o2 - c <= level;
            a1 = da && o1 >= thresh && o1 - c < thresh;
            a2 = db && o2 >= thresh && o2 - c < thresh;
        }
        // The chunk counts itself done only once its reads of C[B] and k[B]
        // have returned (the condition uses them), so the last chunk's
        // update of both cannot overtake them.
        bool last = false;
        if (lane_id() == 0 && kn != INT_MIN)
            last = it.nch == 1 || atomicAdd(&P.bdone[b], 1) == it.nch - 1;
        uint32_t lo1 = 0, hi1 = 0, lo2 = 0, hi2 = 0;
        if (f1) {
            lo1 = (uint32_t)P.link_off[ea];
            hi1 = (uint32_t)P.link_off[(int64_t)ea + 1];
        }
        if (f2) {
            lo2 = (uint32_t)P.link_off[eb];
            hi2 = (uint32_t)P.link_off[(int64_t)eb + 1];
        }
        const uint32_t k1 = f1 ? link_chunks(lo1, hi1) : 0u;
        const uint32_t k2 = f2 ? link_chunks(lo2, hi2) : 0u;
        if (P.prof) count_push(P, q, kSrcSurvivor, (f1 ? 1u : 0u) + (f2 ? 1u : 0u));
        u64 base[3];
        wave_alloc3(k1 + k2, &C->nf[q].v, (a1 ? 1u : 0u) + (a2 ? 1u : 0u), &C->na[cur].v, 0u,
                    nullptr, base);
        put_front(P, q, base[0], ea, lo1, hi1, k1, level);
        put_front(P, q, base[0] + k1, eb, lo2, hi2, k2, level);
        if (a1) st(&P.act[cur][base[1]], ea);
        if (a2) st(&P.act[cur][base[1] + (a1 ? 1 : 0)], eb);
        touch += live ? 1 : 0;
        const int32_t per = P.unit ? c : 1;  // decrements per survivor edge
        upd += (u64)((da ? per : 0) + (db ? per : 0));
        // Without batch bloom processing each of the C kills would lower each
        // survivor by one: C unit updates where one update of C is issued.
        if (!P.unit) unb += (u64)((da ? c - 1 : 0) + (db ? c - 1 : 0));
        if (live && kn <= 1) atomicAnd(&P.alive[w >> 5], ~(1u << (w & 31)));
        if (last) {
            st(&P.bk[b], kn);
            st(&P.bc[b], 0);
            st(&P.bdone[b], 0);
            visits += 1;
        }
        it = nx;
        i = inext;
    }
}

// Adds per-lane statistics to the control block (one atomic per wave).
__device__ __forceinline__ void flush_stats(PeelCtl *C, u64 upd, u64 visits, u64 unb = 0,
                                            u64 touch = 0) {
    upd = wave_sum(upd);
    visits = wave_sum(visits);
    unb = wave_sum(unb);
    touch = wave_sum(touch);
    if (lane_id() == 0) {
        if (upd) atomicAdd(&C->updates.v, upd);
        if (visits) atomicAdd(&C->bloom_visits.v, visits);
        if (unb) atomicAdd(&C->unbatched.v, unb);
        if (touch) atomicAdd(&C->touched.v, touch);
    }
}

// --- one kernel per phase (rounds replayed from a captured HIP graph) ---

__global__ __launch_bounds__(kBlock) void k_phase_a(PeelArgs P, int p) {
    PeelCtl *C = P.ctl;
    __shared__ Round sR;
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        const bool lead = blockIdx.x == 0;
        LeadStats L{};
        if (lead) L.load(C);
        s_ok = !ld(&C->stall) && decide_round(C, p, lead, sR, L, P.prof);
        if (lead) L.store(C);
    }
    __syncthreads();
    if (!s_ok) return;
    const Round R = sR;
    u64 upd = 0;
    phase_a_work(P, p, R, (int64_t)(threadIdx.x / kWave) * gridDim.x + blockIdx.x,
                 (int64_t)gridDim.x * kWavesPerBlock, upd);
    flush_stats(C, upd, 0);
}

__global__ __launch_bounds__(kBlock) void k_phase_b(PeelArgs P, int p) {
    PeelCtl *C = P.ctl;
    __shared__ Round sR;
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        s_ok = !ld(&C->stall);
        if (s_ok) {
            sR.mode = ld(&C->mode[p]);
            sR.level = ld(&C->level[p]);
            sR.cur = ld(&C->cur[p]);
            sR.thresh = ld(&C->thresh);
            sR.nf = sR.na = 0;
            sR.ntc = ld(&C->ntc[p].v);
        }
    }
    __syncthreads();
    if (!s_ok) return;
    const Round R = sR;
    u64 upd = 0, visits = 0, unb = 0, touch = 0;
    phase_b_work(P, p, R, (int64_t)(threadIdx.x / kWave) * gridDim.x + blockIdx.x,
                 (int64_t)gridDim.x * kWavesPerBlock, blockIdx.x == 0 && threadIdx.x == 0, upd,
                 visits, unb, touch);
    flush_stats(C, upd, visits, unb, touch);
}

// --- persistent cooperative kernel: rounds separated by grid barriers ---

// Rebuild of the active set inside the persistent kernel, when it has run
// dry: the remaining edges (phi < 0) are compacted from one list into the
// other while their minimum support mn is found; a log2 histogram of
// support - mn picks the threshold T that puts a few percent of them (at
// least active_min) in the active set; the edges below T are gathered into
// active buffer 0; and the round state is set as if the previous round had
// been a gather that saw minimum support mn.  Counters are pooled per
// workgroup.  Every workgroup derives T from the same histogram.
struct RefillState {
    Counter count;     // entries of the list being written
    int32_t min;       // minimum remaining support (INT_MAX: none)
    int32_t cur;       // list holding the remaining edges; -1: all edges, in id order
    int64_t n_all;     // its length
    int32_t done;      // set when no edge remains
    int32_t yield_req;  // the yield word as the lead last read it
    int32_t yielded;    // set when the launch ended early to give way
    int32_t resume_p;   // -1: start with a rebuild; else decide round parity resume_p
    u64 yield_src;      // address of the host-written yield word (0: none)
    u64 hist[33];
};

// Every kYieldEvery rounds the lead reads the host's yield word (one read
// over the host link, off the rounds' critical path but for one barrier).
constexpr int64_t kYieldEvery = 32;

struct RefillArgs {
    RefillState *rs;
    int32_t *list[2];
    int32_t min_level;  // progressive mode: the first level is at least this
    int32_t active_min;  // the set holds at least this many edges (or all)
};

// Reserves `keep` slots of *ctr for each thread, one atomic per workgroup.
// All threads of the workgroup must call.
__device__ __forceinline__ u64 block_alloc(bool keep, u64 *ctr) {
    __shared__ uint32_t s_w[32];
    __shared__ u64 s_b;
    const int wv = threadIdx.x / kWave, nwv = blockDim.x / kWave;
    const unsigned long long kb = __ballot(keep);
    if (lane_id() == 0) s_w[wv] = (uint32_t)__popcll(kb);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < nwv; ++w) {
            const uint32_t c = s_w[w];
            s_w[w] = t;
            t += c;
        }
        s_b = t ? atomicAdd(ctr, (u64)t) : 0;
    }
    __syncthreads();
    const u64 slot = s_b + s_w[wv] + __popcll(kb & lanemask_lt());
    __syncthreads();
    return slot;
}

// Returns the number of remaining edges (0: the peel is complete); *ok is
// cleared if a barrier gave up.  All threads of the grid must call.
__device__ int64_t grid_refill(const PeelArgs &P, const RefillArgs &RA, GridBar *B,
                               u64 &gen_local, bool lead, int &ok) {
    __shared__ int64_t s_n;
    __shared__ int32_t s_cur, s_mn, s_T;
    __shared__ int s_ok2;
    __shared__ unsigned s_hist[33];
    PeelCtl *C = P.ctl;
    RefillState *RS = RA.rs;
    if (threadIdx.x == 0) {
        s_cur = ld(&RS->cur);
        s_n = ld(&RS->n_all);
    }
    if (lead) {
        st(&C->na[0].v, (u64)0);
        st(&C->na[1].v, (u64)0);
    }
    __syncthreads();
    const int32_t cur = s_cur, nxt = cur < 0 ? 0 : cur ^ 1;
    const int64_t n0 = s_n;
    int32_t mn = INT_MAX;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n0; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        int32_t e = 0;
        bool keep = false;
        if (i < n0) {
            e = cur < 0 ? (int32_t)i : ld(&RA.list[cur][i]);
            keep = ld(&P.phi[e]) < 0;
            if (keep) mn = min(mn, ld(&P.sup[e]));
        }
        const u64 slot = block_alloc(keep, &RS->count.v);
        if (keep) st(&RA.list[nxt][slot], e);
    }
    mn = wave_min(mn);
    if (lane_id() == 0 && mn != INT_MAX) atomicMin(&RS->min, mn);
    drain_memory();
    __syncthreads();
    if (threadIdx.x == 0) {
        s_ok2 = grid_arrive_wait(B, gen_local);
        s_n = (int64_t)ld(&RS->count.v);
        s_mn = ld(&RS->min);
    }
    if (threadIdx.x < 33) s_hist[threadIdx.x] = 0;
    __syncthreads();
    if (!s_ok2) {
        ok = 0;
        return 0;
    }
    const int64_t n = s_n;
    if (n == 0) {
        if (lead) st(&RS->done, 1);
        return 0;
    }
    const int32_t m0 = s_mn;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t d = (uint32_t)(ld(&P.sup[ld(&RA.list[nxt][i])]) - m0) + 1u;
        atomicAdd(&s_hist[31 - __clz(d)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 33 && s_hist[threadIdx.x]) atomicAdd(&RS->hist[threadIdx.x], (u64)s_hist[threadIdx.x]);
    drain_memory();
    __syncthreads();
    if (threadIdx.x == 0) {
        s_ok2 = grid_arrive_wait(B, gen_local);
        // Threshold: the set holds at least max(active_min, n / 32) edges, and
        // every edge at or below the first level.
        const int32_t lvl = max(m0, RA.min_level);
        const int64_t target = max((int64_t)RA.active_min, n / 32);
        int64_t T = INT_MAX, acc = 0;
        for (int b = 0; b < 33; ++b) {
            acc += (int64_t)ld(&RS->hist[b]);
            if (acc >= target) {
                T = min((int64_t)m0 + (int64_t(2) << b) - 1, (int64_t)INT_MAX);
                break;
            }
        }
        T = max(T, min((int64_t)lvl + 1, (int64_t)INT_MAX));
        s_T = (int32_t)T;
        s_mn = lvl;
    }
    __syncthreads();
    if (!s_ok2) {
        ok = 0;
        return 0;
    }
    const int32_t T = s_T;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        int32_t e = 0;
        bool take = false;
        if (i < n) {
            e = ld(&RA.list[nxt][i]);
            take = ld(&P.sup[e]) < T;
        }
        const u64 slot = block_alloc(take, &C->na[0].v);
        if (take) st(&P.act[0][slot], e);
    }
    drain_memory();
    __syncthreads();
    if (threadIdx.x == 0) s_ok2 = grid_arrive_wait(B, gen_local);
    __syncthreads();
    if (!s_ok2) {
        ok = 0;
        return 0;
    }
    if (lead) {
        // As if the previous round (parity 1) had been a gather that found no
        // frontier and saw minimum support s_mn in buffer 0.
        for (int k = 0; k < 2; ++k) {
            st(&C->nf[k].v, (u64)0);
            st(&C->ntc[k].v, (u64)0);
        }
        st(&C->mode[1], (int32_t)kGather);
        st(&C->cur[1], 1);
        st(&C->gmin[1], s_mn);
        st(&C->gmin[0], (int32_t)INT_MAX);
        st(&C->stall, 0);
        st(&C->thresh, T);
        // The next refill starts from this list.
        st(&RS->cur, nxt);
        st(&RS->n_all, n);
        st(&RS->count.v, (u64)0);
        st(&RS->min, (int32_t)INT_MAX);
        for (int b = 0; b < 33; ++b) st(&RS->hist[b], (u64)0);
    }
    drain_memory();
    __syncthreads();
    if (threadIdx.x == 0) s_ok2 = grid_arrive_wait(B, gen_local);
    __syncthreads();
    if (!s_ok2) ok = 0;
    return s_ok2 ? n : 0;
}

__global__ __launch_bounds__(kPBlock) void k_peel_persistent(PeelArgs P, GridBar *B,
                                                             int64_t max_rounds, int prof,
                                                             RefillArgs RA) {
    PeelCtl *C = P.ctl;
    RefillState *RS = RA.rs;
    __shared__ Round sR;
    __shared__ int s_ok, s_fail, s_y, s_p;
    __shared__ const int32_t *s_ys;
    u64 gen_local = 0;  // barriers passed (the host clears the barrier per launch)
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // Wave ids run across blocks first: a small round spreads its work items
    // over many CUs (and all XCDs) instead of filling a few CUs' memory
    // pipelines with scattered accesses.
    const int64_t wid = (int64_t)(threadIdx.x / kWave) * gridDim.x + blockIdx.x;
    const int64_t nwaves = (int64_t)gridDim.x * (kPBlock / kWave);
    // The lead's clocks and counters live in LDS, not in every lane's
    // registers (which would push the kernel past 128 VGPRs into spills).
    __shared__ u64 t[5], acc[6];
    __shared__ LeadStats L;
    u64 upd = 0, visits = 0, unb = 0, touch = 0;
    if (lead) {
        L.load(C);
        for (int k = 0; k < 6; ++k) acc[k] = 0;
    }
    if (threadIdx.x == 0) {
        s_fail = 0;
        s_y = 0;
        s_p = ld(&RS->resume_p);
        s_ys = reinterpret_cast<const int32_t *>(ld(&RS->yield_src));
    }
    __syncthreads();
    // A launch resumes where the previous one yielded (deciding the round
    // of parity s_p), or starts with a rebuild of the active set.
    int p = s_p;
    int64_t r = 0;  // rounds of this launch
    while (r < max_rounds) {
    // The active set is (re)built here whenever it runs dry; the peel ends
    // when no edge remains.
    if (p < 0) {
        int ok = 1;
        if (grid_refill(P, RA, B, gen_local, lead, ok) == 0) {
            if (!ok && threadIdx.x == 0) s_fail = 1;
            break;
        }
        p = 0;
    }
    if (threadIdx.x == 0) s_ok = decide_round(C, p, lead, sR, L, P.prof);
    __syncthreads();
    for (; r < max_rounds && s_ok; ++r) {
        if (prof && lead) t[0] = wall_clock64();
        Round R = sR;
        phase_a_work(P, p, R, wid, nwaves, upd);
        if (prof && lead) t[1] = wall_clock64();
        drain_memory();
        __syncthreads();
        if (threadIdx.x == 0) {
            s_ok = grid_arrive_wait(B, gen_local);
            if (!s_ok) s_fail = 1;
            sR.ntc = ld(&C->ntc[p].v);
        }
        __syncthreads();
        if (!s_ok) break;
        R.ntc = sR.ntc;
        if (prof && lead) t[2] = wall_clock64();
        phase_b_work(P, p, R, wid, nwaves, lead, upd, visits, unb, touch);
        if (prof && lead) t[3] = wall_clock64();
        drain_memory();
        __syncthreads();
        if (threadIdx.x == 0) {
            // Every kYieldEvery rounds (the same rounds in every block) the
            // lead publishes the host's yield word before the barrier and
            // every block reads it after: all stop together, before deciding
            // the next round, and the next launch decides it.
            const bool chk = s_ys && ((r + 1) & (kYieldEvery - 1)) == 0;
            if (chk && lead) {
                st(&RS->yield_req, __hip_atomic_load(s_ys, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_SYSTEM));
                drain_memory();
            }
            const bool bar = grid_arrive_wait(B, gen_local);
            if (!bar) s_fail = 1;
            const bool y = bar && chk && ld(&RS->yield_req) != 0;
            if (y) s_y = 1;
            s_ok = bar && !y && decide_round(C, p ^ 1, lead, sR, L, P.prof);
        }
        __syncthreads();
        if (prof && lead) {
            t[4] = wall_clock64();
            for (int k = 0; k < 4; ++k) acc[k] += t[k + 1] - t[k];
            if (R.mode == kGather) {
                acc[4] += t[2] - t[0];
                acc[5] += 1;
            } else {
                const int bnf = 63 - __clzll(R.nf | 1), bntc = 63 - __clzll(R.ntc | 1);
                st(&C->time_nf[bnf], ld(&C->time_nf[bnf]) + (t[4] - t[0]));
                st(&C->time_ntc[bntc], ld(&C->time_ntc[bntc]) + (t[4] - t[2]));
            }
        }
        p ^= 1;
    }
    if (s_fail || s_y) break;
    p = -1;
    }
    flush_stats(C, upd, visits, unb, touch);
    if (lead) {
        L.store(C);
        for (int k = 0; k < 6; ++k) st(&C->prof[k], ld(&C->prof[k]) + acc[k]);
        st(&RS->yielded, s_y);
        st(&RS->resume_p, s_y ? p : -1);
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
          PeelCounters &pc, Workspace &ws, hipStream_t s, const PeelOptions *opt) {
    const int32_t *fixed = opt ? opt->fixed : nullptr;
    const int32_t min_level = opt ? opt->min_level : 0;
    const int32_t unit = opt && opt->unit_updates ? 1 : 0;
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
    P.prof = std::getenv("BT_PEEL_PROFILE") ? 1 : 0;
    P.unit = unit;
    int32_t *glist[2] = {ws.get<int32_t>("peel_all0", m), ws.get<int32_t>("peel_all1", m)};
    u64 *rs = ws.get<u64>("peel_refill", 40);  // [0] count, [1] min, [2..34] histogram

    k_init_peel<<<grid_for(m, 256, 16384), 256, 0, s>>>(ix.supl, m, fixed, P.sup, P.phi,
                                                         sup_out);
    BT_CHECK_LAUNCH();
    k_init_alive<<<grid_for(words, 256, 16384), 256, 0, s>>>(ix.cursor, P.alive);
    BT_CHECK_LAUNCH();
    zero_bytes(P.bc, sizeof(int32_t) * nb, s);
    zero_bytes(P.bdone, sizeof(int32_t) * nb, s);
    PeelCtl init{};
    init.gmin[0] = init.gmin[1] = INT_MAX;
    BT_HIP(hipMemcpyAsync(P.ctl, &init, sizeof init, hipMemcpyHostToDevice, s));

    PeelCtl *hc = reinterpret_cast<PeelCtl *>(ws.host((int)(sizeof(PeelCtl) / 8 + 40)));
    u64 *hr = reinterpret_cast<u64 *>(hc + 1);
    // BT_PEEL_MODE=graph replays captured two-kernel rounds instead of the
    // persistent kernel; BT_PEEL_GRAPH=0 launches those rounds directly.
    // BT_PEEL_VERBOSE=1 prints the time of the persistent launch.
    const bool verbose = std::getenv("BT_PEEL_VERBOSE") != nullptr;
    const char *mv = std::getenv("BT_PEEL_MODE");
    const PeelTraceFn *trace = opt && opt->trace && *opt->trace ? opt->trace : nullptr;
    const bool persistent = ws.coop && !trace && !(mv && std::strcmp(mv, "graph") == 0);
    const char *gv = std::getenv("BT_PEEL_GRAPH");
    const bool use_graph = !trace && !(gv && std::atoi(gv) == 0);
    GridBar *bar = ws.get<GridBar>("peel_bar", 1);
    zero_bytes(bar, sizeof(GridBar), s);
    int pblocks = 0;
    if (persistent) {
        int dev = 0, cus = 0, occ = 0;
        BT_HIP(hipGetDevice(&dev));
        BT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_peel_persistent, kPBlock, 0));
        const char *pb = std::getenv("BT_PEEL_PBLOCKS");
        pblocks = pb ? std::max(1, std::min(std::atoi(pb), occ * cus))
                     : peel_grid(r.tp, cus, occ * cus);
    }

    std::unique_ptr<CoopTurn> turn;
    if (persistent) turn.reset(new CoopTurn(m));
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
    if (persistent) {
        // One launch: the kernel rebuilds the active set itself whenever it
        // runs dry and stops when no edge remains; or, when a lighter peel
        // waits for the device, it stops between two rounds and is launched
        // again, to decide the next round, once that peel has had its turn.
        // BT_PEEL_YIELD=1 makes every launch stop at its first check (a test
        // of the resume path).
        const char *yv = std::getenv("BT_PEEL_YIELD");
        const bool force_yield = yv && std::atoi(yv) == 1;
        RefillState rs0{};
        rs0.min = INT_MAX;
        rs0.cur = -1;  // all edges, in id order
        rs0.n_all = m;
        rs0.resume_p = -1;
        rs0.yield_src = reinterpret_cast<u64>(turn->yield_word(force_yield));
        RefillState *drs = ws.get<RefillState>("peel_refill_state", 1);
        BT_HIP(hipMemcpyAsync(drs, &rs0, sizeof rs0, hipMemcpyHostToDevice, s));
        RefillArgs RA{drs, {glist[0], glist[1]}, min_level, r.tp.active_min};
        int64_t max_rounds = 4 * m + 64;
        int prof = std::getenv("BT_PEEL_PROFILE") ? 1 : 0;
        void *args[] = {&P, &bar, &max_rounds, &prof, &RA};
        for (int64_t launch = 0;; ++launch) {
            // A launch that yields has run kYieldEvery rounds.
            if (launch * kYieldEvery > max_rounds)
                throw Error{BT_EDEVICE, "peel made no progress"};
            if (launch > 0) zero_bytes(bar, sizeof(GridBar), s);
            BT_HIP(hipEventRecord(ev0, s));
            BT_HIP(hipLaunchCooperativeKernel((const void *)k_peel_persistent, dim3(pblocks),
                                              dim3(kPBlock), args, 0, s));
            BT_HIP(hipEventRecord(ev1, s));
            int32_t fail = 0;
            BT_HIP(hipMemcpyAsync(&fail, &bar->fail, sizeof fail, hipMemcpyDeviceToHost, s));
            BT_HIP(hipMemcpyAsync(&rs0, drs, sizeof rs0, hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            float t = 0.f;
            BT_HIP(hipEventElapsedTime(&t, ev0, ev1));
            pc.kernel_ms += t;
            pc.launches += 1;
            if (fail) throw Error{BT_EDEVICE, "peel grid barrier timed out"};
            if (verbose)
                std::fprintf(stderr, "[peel] launch %lld: %.1f ms%s\n", (long long)launch,
                             (double)t, rs0.yielded ? " (yielded)" : "");
            if (rs0.done) break;
            if (!rs0.yielded) throw Error{BT_EDEVICE, "peel stopped early"};
            pc.yields += 1;
            turn->requeue();
        }
    } else {
    int64_t n_all = m;
    int cur = -1;  // -1: all edges, in id order
    int chunk = 4;
    int tp = 0;  // trace mode: parity of the next round
    bool need_refill = true;
    for (int64_t guard = 0;; ++guard) {
        if (need_refill) {
            // Rebuild the active set: compact the remaining edges, find their
            // minimum support, histogram supports above it, pick T so that
            // the set holds a few percent of the remaining edges.
            const int nxt = cur < 0 ? 0 : cur ^ 1;
            zero_bytes(rs, sizeof(u64) * 40, s);
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
            // The first level is at least min_level: every edge at or below
            // it goes in one level (progressive mode), and the active set
            // must then hold all of them.
            const int32_t mn0 = *reinterpret_cast<int32_t *>(hr + 1);
            const int32_t mn = std::max(mn0, min_level);
            k_refill_hist<<<grid_for(n_all, kBlock, 2048), kBlock, 0, s>>>(glist[cur], n_all,
                                                                          P.sup, mn0, rs + 2);
            BT_CHECK_LAUNCH();
            BT_HIP(hipMemcpyAsync(hr + 2, rs + 2, 33 * sizeof(u64), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            const int64_t target = std::max<int64_t>(r.tp.active_min, n_all / 32);
            int64_t thresh = INT_MAX, acc = 0;
            for (int b = 0; b < 33; ++b) {
                acc += (int64_t)hr[2 + b];
                if (acc >= target) {
                    thresh = std::min<int64_t>((int64_t)mn0 + (int64_t(2) << b) - 1, INT_MAX);
                    break;
                }
            }
            thresh = std::max<int64_t>(thresh, std::min<int64_t>((int64_t)mn + 1, INT_MAX));
            zero_bytes(&P.ctl->na[0].v, sizeof(u64), s);
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
        if (trace) {
            // One round at a time: the frontier it removes is read before it
            // runs, supports and bloom numbers after.
            BT_HIP(hipMemcpyAsync(hc, P.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            const int64_t nf = hc->stall ? 0 : (int64_t)hc->nf[tp].v;
            std::vector<FrontItem> items((size_t)nf);
            if (nf)
                BT_HIP(hipMemcpy(items.data(), P.front[tp], sizeof(FrontItem) * nf,
                                 hipMemcpyDeviceToHost));
            launch_round(P, tp, s);
            BT_CHECK_LAUNCH();
            BT_HIP(hipMemcpyAsync(hc, P.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            if (hc->stall) {
                need_refill = true;
                tp = 0;
                continue;
            }
            if (hc->mode[tp] == kNormal) {
                PeelTraceRound tr;
                tr.level = hc->level[tp];
                for (const FrontItem &it : items)
                    if (tr.removed.empty() || tr.removed.back() != it.e) tr.removed.push_back(it.e);
                tr.sup.resize((size_t)m);
                tr.bloom_k.resize((size_t)ix.n_b);
                BT_HIP(hipMemcpy(tr.sup.data(), P.sup, sizeof(int32_t) * m,
                                 hipMemcpyDeviceToHost));
                if (ix.n_b)
                    BT_HIP(hipMemcpy(tr.bloom_k.data(), ix.bk, sizeof(int32_t) * ix.n_b,
                                     hipMemcpyDeviceToHost));
                (*trace)(tr);
            }
            tp ^= 1;
            if (guard > 4 * m + 64) throw Error{BT_EDEVICE, "peel made no progress"};
            continue;
        }
        BT_HIP(hipEventRecord(ev0, s));
        if (use_graph) {
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
        if (hc->stall) need_refill = true;
        chunk = std::min(chunk * 2, 64);
        if (guard > 4 * m + 64) throw Error{BT_EDEVICE, "peel made no progress"};
    }
    }
    BT_HIP(hipMemcpyAsync(hc, P.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    pc.levels = (int64_t)hc->levels;
    pc.rounds = (int64_t)hc->rounds;
    pc.max_phi = hc->max_level;
    pc.updates = (int64_t)hc->updates.v;
    pc.bloom_visits = (int64_t)hc->bloom_visits.v;
    pc.updates_unbatched = pc.updates + (int64_t)hc->unbatched.v;
    pc.touched = (int64_t)hc->touched.v;
    if (std::getenv("BT_PEEL_PROFILE"))
        std::fprintf(stderr, "[peel] rounds %llu  block0 us: phaseA %.0f bar1 %.0f phaseB %.0f bar2 %.0f; gather rounds %llu phaseA+bar1 %.0f\n",
                     hc->rounds, hc->prof[0] / 100.0, hc->prof[1] / 100.0, hc->prof[2] / 100.0,
                     hc->prof[3] / 100.0, hc->prof[5], hc->prof[4] / 100.0);
    if (P.prof) {
        std::fprintf(stderr, "[peel] pushes: twin %llu survivor %llu; twin-only rounds %llu\n[peel] frontier items log2 histogram:",
                     hc->twin_pushes, hc->surv_pushes, hc->twin_only_rounds);
        for (int b = 0; b < 32; ++b)
            if (hc->hist_nf[b]) std::fprintf(stderr, " %d:%llu", b, hc->hist_nf[b]);
        std::fprintf(stderr, "\n[peel] bloom items log2 histogram:");
        for (int b = 0; b < 32; ++b)
            if (hc->hist_ntc[b]) std::fprintf(stderr, " %d:%llu", b, hc->hist_ntc[b]);
        std::fprintf(stderr, "\n[peel] normal-round us by log2 frontier items:");
        for (int b = 0; b < 32; ++b)
            if (hc->time_nf[b]) std::fprintf(stderr, " %d:%.0f", b, hc->time_nf[b] / 100.0);
        std::fprintf(stderr, "\n[peel] phase-B+barrier us by log2 bloom items:");
        for (int b = 0; b < 32; ++b)
            if (hc->time_ntc[b]) std::fprintf(stderr, " %d:%.0f", b, hc->time_ntc[b] / 100.0);
        std::fprintf(stderr, "\n");
    }
    k_phi_out<<<grid_for(m, 256, 16384), 256, 0, s>>>(P.phi, phi_out, m);
    BT_CHECK_LAUNCH();
}

}  // namespace bt
