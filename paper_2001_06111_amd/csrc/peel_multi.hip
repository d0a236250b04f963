// peel_multi.hip - the peel of a batch of graphs (one disjoint union) in one
// cooperative kernel, each graph at its own level.
#include "peel_common.h"

namespace bt {

namespace {

// --- grid-wide peel of many graphs, each at its own level ------------------
//
// A batch is a disjoint union, but its graphs need not share levels: here
// every graph has its own state (level, whether it has frontier work, the
// result of its last gather) and the grid advances all of them in each
// round.  Work items carry their graph's level, so the crossing test needs
// no lookup.  A graph's level change is decided at the start of a round from
// what the previous round left (a frontier for this round, or the result of
// its gather) and, when needed, a gather over the graph's edges is scheduled
// for the next round: per level a graph spends its normal rounds, one idle
// round and one gather round.  A gather rescans the graph's whole edge range
// (no active set): batch graphs are small, and the scan is coalesced.

enum : int32_t { kGsNormal = 0, kGsDone = 1 };
constexpr int kGatherPerLane = 8;  // edges per lane of a gather item
constexpr uint32_t kGatherChunk = kWave * kGatherPerLane;
// Unions at least this large peel on every CU by default (see peel_multi).
constexpr int64_t kMultiAllCusEdges = int64_t(1) << 24;

struct alignas(64) GState {
    int32_t state;      // kGsNormal or kGsDone
    int32_t level;
    int32_t gmin[2];    // minimum remaining support above the level, by round parity
    int32_t fr[2];      // frontier items exist for the round of this parity
    int32_t e0, e1;     // edge range in the union
    int64_t gather_round;  // round of the last scheduled gather (-1: none)
    int32_t levels;        // levels this graph visited
    int32_t max_level;
};

struct alignas(16) MBloomItem {
    int32_t b;
    int32_t level;
    uint32_t lo;
    uint32_t meta;  // (chunks of the bloom << 7) | (wedges in this chunk)
};

struct alignas(16) GatherItem {
    int32_t g;
    int32_t level;
    uint32_t lo, hi;  // positions in the graph's current remaining list
};

struct MultiCtl {
    Counter nf[2], ntc[2], ngth[2];
    Counter updates, bloom_visits;
    Counter touched;  // live wedges visited in phase B
    Counter left;  // graphs not done
    u64 rounds;    // rounds run so far (a resumed launch starts at this round)
    u64 prof[5];   // BT_PEEL_PROFILE=1: block-0 clock ticks (decide, A, bar, B, bar)
    u64 yield_src;      // address of the host-written yield word (0: none)
    int32_t yield_req;  // the yield word as the lead last read it
    int32_t yielded;    // set when the launch ended early to give way
};

// Every kMultiYieldEvery rounds the lead reads the host's yield word.
constexpr int64_t kMultiYieldEvery = 32;

struct MultiArgs {
    MultiCtl *ctl;
    GState *gs;
    const int32_t *gid;  // graph of each edge
    int32_t ng;
    FrontItem *front[2];
    MBloomItem *tc[2];
    GatherItem *gth[2];
};

__device__ __forceinline__ void set_front_flag(const MultiArgs &M, int32_t g, int q) {
    st(&M.gs[g].fr[q], 1);
}

// Bloom items of the lanes' first kills, written cooperatively (as put_chunks).
__device__ __forceinline__ void put_bloom_items(MBloomItem *list, u64 base, uint32_t cnt,
                                                int32_t b, int32_t level, uint32_t lo,
                                                uint32_t hi) {
    const uint32_t own = min(cnt, kOwnChunks);
    for (uint32_t c = 0; c < own; ++c) {
        const uint32_t a = lo + c * kWave;
        st_item(&list[base + c], MBloomItem{b, level, a, (cnt << 7) | (min(a + (uint32_t)kWave, hi) - a)});
    }
    unsigned long long big = __ballot(cnt > own);
    while (big) {
        const int l = __ffsll(big) - 1;
        big &= big - 1;
        const uint32_t n = __shfl(cnt, l, kWave);
        const u64 bb = __shfl(base, l, kWave);
        const int32_t lb = __shfl(b, l, kWave), ll = __shfl(level, l, kWave);
        const uint32_t llo = __shfl(lo, l, kWave), lhi = __shfl(hi, l, kWave);
        for (uint32_t c = kOwnChunks + lane_id(); c < n; c += kWave) {
            const uint32_t a = llo + c * kWave;
            st_item(&list[bb + c], MBloomItem{lb, ll, a, (n << 7) | (min(a + (uint32_t)kWave, lhi) - a)});
        }
    }
}

// Decides, at the start of round r (parity p), what each of this thread's
// graphs does next; schedules gathers for round r + 1 into gth[q].  All
// state reads are issued together.
__device__ void multi_decide(const MultiArgs &M, int64_t r, int p, int64_t tid, int64_t nthreads) {
    const int q = p ^ 1;
    for (int64_t g0 = tid - lane_id(); g0 < M.ng; g0 += nthreads) {
        const int64_t g = g0 + lane_id();
        bool sched = false;
        int32_t lvl = 0, e0 = 0, e1 = 0;
        if (g < M.ng) {
            GState *G = &M.gs[g];
            const int32_t state = ld(&G->state);
            const int64_t gr = ld(&G->gather_round);
            const int32_t fr = ld(&G->fr[p]);
            const int32_t level = ld(&G->level);
            const int32_t gm = ld(&G->gmin[q]);
            e0 = ld(&G->e0);
            e1 = ld(&G->e1);
            if (state != kGsDone) {
                if (fr) st(&G->fr[p], 0);
                if (gr != r && !fr) {
                    // No frontier this round: the level is exhausted.  After a
                    // gather that took nothing, jump to the smallest remaining
                    // support, or finish when nothing remains.
                    int32_t next = level + 1;
                    if (gr == r - 1) {
                        next = gm;
                        if (gm == INT_MAX) {
                            st(&G->state, (int32_t)kGsDone);
                            atomicAdd(&M.ctl->left.v, ~0ull);
                        }
                    }
                    if (next != INT_MAX) {
                        sched = true;
                        lvl = next;
                        st(&G->level, lvl);
                        st(&G->gather_round, r + 1);
                        st(&G->gmin[q], (int32_t)INT_MAX);
                        atomicAdd(&G->levels, 1);
                    }
                }
            }
        }
        const uint32_t n = sched ? (uint32_t)(e1 - e0) : 0u;
        const uint32_t cnt = (n + kGatherChunk - 1) / kGatherChunk;
        u64 base[3];
        wave_alloc3(cnt, &M.ctl->ngth[q].v, 0u, nullptr, 0u, nullptr, base);
        // Items {g, level, lo, hi} over the edge range, kGatherChunk edges each.
        const uint32_t own = min(cnt, kOwnChunks);
        for (uint32_t c = 0; c < own; ++c) {
            const uint32_t a = (uint32_t)e0 + c * kGatherChunk;
            st_item(&M.gth[q][base[0] + c],
                    GatherItem{(int32_t)g, lvl, a, min(a + kGatherChunk, (uint32_t)e1)});
        }
        unsigned long long big = __ballot(cnt > own);
        while (big) {
            const int l = __ffsll(big) - 1;
            big &= big - 1;
            const uint32_t nc = __shfl(cnt, l, kWave);
            const u64 b = __shfl(base[0], l, kWave);
            const int32_t lg = __shfl((int32_t)g, l, kWave), ll = __shfl(lvl, l, kWave);
            const uint32_t le0 = (uint32_t)__shfl(e0, l, kWave), le1 = (uint32_t)__shfl(e1, l, kWave);
            for (uint32_t c = kOwnChunks + lane_id(); c < nc; c += kWave) {
                const uint32_t a = le0 + c * kGatherChunk;
                st_item(&M.gth[q][b + c], GatherItem{lg, ll, a, min(a + kGatherChunk, le1)});
            }
        }
    }
}

__device__ __forceinline__ void multi_phase_a(const PeelArgs &P, const MultiArgs &M, int p,
                                              u64 nf, u64 ngth, int64_t wid, int64_t nwaves,
                                              u64 &upd) {
    MultiCtl *C = M.ctl;
    const int q = p ^ 1;
    const int64_t total = (int64_t)(nf + ngth);
    for (int64_t i = wid; i < total; i += nwaves) {
        if (i >= (int64_t)nf) {
            // Gather item: the graph's remaining edges at or below its level
            // become the next frontier; the smallest support above it is kept
            // for a jump.  Each lane reads kGatherPerLane edges at once.
            const GatherItem it = ld_item(&M.gth[p][i - (int64_t)nf]);
            int32_t ph[kGatherPerLane], sv[kGatherPerLane];
#pragma unroll
            for (int k = 0; k < kGatherPerLane; ++k) {
                const uint32_t e = it.lo + k * kWave + lane_id();
                ph[k] = 0;
                sv[k] = INT_MAX;
                if (e < it.hi) {
                    ph[k] = ld(&P.phi[e]);
                    sv[k] = ld(&P.sup[e]);
                }
            }
            int32_t mn = INT_MAX;
            uint32_t lo[kGatherPerLane], hi[kGatherPerLane];
            bool take[kGatherPerLane];
            bool any = false;
#pragma unroll
            for (int k = 0; k < kGatherPerLane; ++k) {
                const uint32_t e = it.lo + k * kWave + lane_id();
                const bool live = e < it.hi && ph[k] < 0;
                take[k] = live && sv[k] <= it.level;
                if (live && !take[k]) mn = min(mn, sv[k]);
                lo[k] = hi[k] = 0;
                if (take[k]) {
                    lo[k] = (uint32_t)P.link_off[e];
                    hi[k] = (uint32_t)P.link_off[(int64_t)e + 1];
                }
                any |= take[k];
            }
            uint32_t kk[kGatherPerLane], tot = 0;
#pragma unroll
            for (int k = 0; k < kGatherPerLane; ++k) {
                kk[k] = take[k] ? link_chunks(lo[k], hi[k]) : 0u;
                tot += kk[k];
            }
            u64 base[3];
            wave_alloc3(tot, &C->nf[q].v, 0u, nullptr, 0u, nullptr, base);
            u64 b = base[0];
#pragma unroll
            for (int k = 0; k < kGatherPerLane; ++k) {
                put_front(P, q, b, (int32_t)(it.lo + k * kWave + lane_id()), lo[k], hi[k], kk[k],
                          it.level);
                b += kk[k];
            }
            mn = wave_min(mn);
            if (__ballot(any) != 0 && lane_id() == 0) set_front_flag(M, it.g, q);
            if (lane_id() == 0 && mn != INT_MAX) atomicMin(&M.gs[it.g].gmin[p], mn);
            continue;
        }
        const FrontItem it = ld_item(&P.front[p][i]);
        const int32_t level = it.level;
        const uint32_t j = it.lo + lane_id();
        const bool has = j < it.hi;
        uint32_t bit = 0, old = 0, w0 = 0, w1 = 0, tlo = 0, thi = 0;
        int32_t blm = 0, twin = 0, kb = 0, tg = 0;
        if (has) {
            const uint3 lk = P.link[j];
            const uint32_t w = lk.x;
            blm = (int32_t)lk.y;
            twin = (int32_t)(lk.z & kEdgeMask);
            bit = 1u << (w & 31);
            w0 = P.bwoff[blm];
            w1 = P.bwoff[blm + 1];
            kb = ld(&P.bk[blm]);
            tlo = (uint32_t)P.link_off[twin];
            thi = (uint32_t)P.link_off[(int64_t)twin + 1];
            tg = M.gid[twin];
            old = atomicAnd(&P.alive[w >> 5], ~bit);
        }
        const bool won = has && (old & bit);
        const int32_t d = max(kb - 1, 0);
        const bool dec = won && d > 0;
        int32_t oc = 1, otw = 0;
        if (won) {
            oc = atomicAdd(&P.bc[blm], 1);
            otw = atomicSub(&P.sup[twin], d);
        }
        const bool first = oc == 0;
        const uint32_t nch = first ? (w1 - w0 + kWedgeChunk - 1) / kWedgeChunk : 0u;
        const bool tf = dec && otw > level && otw - d <= level;
        const uint32_t tk = tf ? link_chunks(tlo, thi) : 0u;
        u64 base[3];
        wave_alloc3(nch, &C->ntc[p].v, tk, &C->nf[q].v, 0u, nullptr, base);
        put_bloom_items(M.tc[p], base[0], nch, blm, level, w0, w1);
        put_front(P, q, base[1], twin, tlo, thi, tk, level);
        if (tf) set_front_flag(M, tg, q);
        upd += dec ? 1 : 0;
    }
}

__device__ __forceinline__ void multi_phase_b(const PeelArgs &P, const MultiArgs &M, int p,
                                              u64 ntc, int64_t wid, int64_t nwaves, u64 &upd,
                                              u64 &visits, u64 &touch) {
    MultiCtl *C = M.ctl;
    const int q = p ^ 1;
    for (int64_t i = wid; i < (int64_t)ntc; i += nwaves) {
        const MBloomItem it = ld_item(&M.tc[p][i]);
        const int32_t b = it.b;
        const int32_t level = it.level;
        const uint32_t nch = it.meta >> 7;
        const uint32_t w = it.lo + lane_id();
        const bool inr = w < it.lo + (it.meta & 127u);
        uint32_t word = 0;
        int32_t ea = 0, eb = 0;
        if (inr) {
            ea = P.wea[w];
            eb = P.web[w];
            word = ld(&P.alive[w >> 5]);
        }
        const int32_t c = ld(&P.bc[b]);
        const int32_t kn = ld(&P.bk[b]) - c;
        const bool live = inr && kn > 0 && ((word >> (w & 31)) & 1u);
        int32_t o1 = 0, o2 = 0;
        if (live) {
            o1 = atomicSub(&P.sup[ea], c);
            o2 = atomicSub(&P.sup[eb], c);
        }
        bool last = false;
        if (lane_id() == 0 && kn != INT_MIN)
            last = nch == 1 || atomicAdd(&P.bdone[b], 1) == (int32_t)nch - 1;
        const bool f1 = live && o1 > level && o1 - c <= level;
        const bool f2 = live && o2 > level && o2 - c <= level;
        uint32_t lo1 = 0, hi1 = 0, lo2 = 0, hi2 = 0;
        int32_t g1 = 0, g2 = 0;
        if (f1) {
            lo1 = (uint32_t)P.link_off[ea];
            hi1 = (uint32_t)P.link_off[(int64_t)ea + 1];
            g1 = M.gid[ea];
        }
        if (f2) {
            lo2 = (uint32_t)P.link_off[eb];
            hi2 = (uint32_t)P.link_off[(int64_t)eb + 1];
            g2 = M.gid[eb];
        }
        const uint32_t k1 = f1 ? link_chunks(lo1, hi1) : 0u;
        const uint32_t k2 = f2 ? link_chunks(lo2, hi2) : 0u;
        u64 base[3];
        wave_alloc3(k1 + k2, &C->nf[q].v, 0u, nullptr, 0u, nullptr, base);
        put_front(P, q, base[0], ea, lo1, hi1, k1, level);
        put_front(P, q, base[0] + k1, eb, lo2, hi2, k2, level);
        if (f1) set_front_flag(M, g1, q);
        if (f2) set_front_flag(M, g2, q);
        upd += live ? 2 : 0;
        touch += live ? 1 : 0;
        if (live && kn <= 1) atomicAnd(&P.alive[w >> 5], ~(1u << (w & 31)));
        if (last) {
            st(&P.bk[b], kn);
            st(&P.bc[b], 0);
            st(&P.bdone[b], 0);
            visits += 1;
        }
    }
}

__global__ __launch_bounds__(kPBlock) void k_peel_multi(PeelArgs P, MultiArgs M, GridBar *B,
                                                        int64_t max_rounds, int prof) {
    MultiCtl *C = M.ctl;
    __shared__ u64 s_nf, s_ngth, s_ntc, s_left, s_r0;
    __shared__ int s_ok, s_y;
    __shared__ const int32_t *s_ys;
    u64 gen_local = 0;
    const int64_t wid = (int64_t)(threadIdx.x / kWave) * gridDim.x + blockIdx.x;
    const int64_t nwaves = (int64_t)gridDim.x * (kPBlock / kWave);
    const int64_t tid = wid * kWave + lane_id();
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    u64 upd = 0, visits = 0, touch = 0;
    if (threadIdx.x == 0) {
        // A launch resumes at the round where the previous one yielded.
        s_r0 = ld(&C->rounds);
        s_left = ld(&C->left.v);
        s_nf = ld(&C->nf[s_r0 & 1].v);
        s_ngth = ld(&C->ngth[s_r0 & 1].v);
        s_ys = reinterpret_cast<const int32_t *>(ld(&C->yield_src));
        s_ok = 1;
        s_y = 0;
    }
    if (lead) st(&C->yielded, 0);
    __syncthreads();
    int64_t r = (int64_t)s_r0;
    for (; r < max_rounds && s_left > 0 && s_ok; ++r) {
        const int p = (int)(r & 1), q = p ^ 1;
        const u64 nf = s_nf, ngth = s_ngth;
        u64 t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
        if (prof && lead) t0 = wall_clock64();
        if (lead) st(&C->ntc[q].v, (u64)0);
        multi_decide(M, r, p, tid, nwaves * kWave);
        if (prof && lead) t1 = wall_clock64();
        multi_phase_a(P, M, p, nf, ngth, wid, nwaves, upd);
        if (prof && lead) t2 = wall_clock64();
        drain_memory();
        __syncthreads();
        if (threadIdx.x == 0) {
            s_ok = grid_arrive_wait(B, gen_local);
            s_ntc = ld(&C->ntc[p].v);
        }
        __syncthreads();
        if (!s_ok) break;
        if (prof && lead) t3 = wall_clock64();
        if (lead) {
            st(&C->nf[p].v, (u64)0);
            st(&C->ngth[p].v, (u64)0);
        }
        multi_phase_b(P, M, p, s_ntc, wid, nwaves, upd, visits, touch);
        drain_memory();
        __syncthreads();
        if (threadIdx.x == 0) {
            // Every kMultiYieldEvery rounds the lead publishes the host's
            // yield word before the barrier and every block reads it after,
            // so all blocks stop after the same round.
            const bool chk = s_ys && ((r + 1) % kMultiYieldEvery) == 0;
            if (chk && lead) {
                st(&C->yield_req, __hip_atomic_load(s_ys, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM));
                drain_memory();
            }
            s_ok = grid_arrive_wait(B, gen_local);
            s_left = ld(&C->left.v);
            s_nf = ld(&C->nf[q].v);
            s_ngth = ld(&C->ngth[q].v);
            s_y = s_ok && chk && ld(&C->yield_req) != 0;
        }
        __syncthreads();
        if (prof && lead) {
            t4 = wall_clock64();
            C->prof[0] += t1 - t0;
            C->prof[1] += t2 - t1;
            C->prof[2] += t3 - t2;
            C->prof[4] += t4 - t3;
        }
        if (s_y) {
            ++r;
            if (lead && s_left > 0) st(&C->yielded, 1);
            break;
        }
    }
    upd = wave_sum(upd);
    visits = wave_sum(visits);
    touch = wave_sum(touch);
    if (lane_id() == 0) {
        if (upd) atomicAdd(&C->updates.v, upd);
        if (visits) atomicAdd(&C->bloom_visits.v, visits);
        if (touch) atomicAdd(&C->touched.v, touch);
    }
    if (lead) st(&C->rounds, (u64)r);
}

}  // namespace

namespace {

__global__ void k_max_phi(const int32_t *phi, int64_t m, unsigned long long *out) {
    unsigned long long v = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        v = max(v, (unsigned long long)max(phi[e], 0));
    for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, (unsigned long long)__shfl_xor(v, d, kWave));
    if (lane_id() == 0) atomicMax(out, v);
}

__global__ void k_multi_init(const int64_t *off, int32_t ng, int32_t *gid) {
    for (int32_t g = blockIdx.x; g < ng; g += gridDim.x)
        for (int64_t e = off[g] + threadIdx.x; e < off[g + 1]; e += blockDim.x) gid[e] = g;
}

}  // namespace

int64_t peel_state_bytes(int64_t m, int64_t n_b, int64_t n_w, int64_t graphs, bool multi) {
    const int64_t nb = n_b > 0 ? n_b : 1;
    const int64_t words = (n_w + 31) / 32 + 1;
    const int64_t max_tc = nb + n_w / kWedgeChunk + 1;
    const int64_t max_front = m + 2 * n_w / kLinkChunk + 1;
    const int64_t max_gth = m / kGatherChunk + graphs + 1;
    // Buffers of peel() or of peel_multi().
    const int64_t shared = 4 * m * 2 + 4 * words + 4 * nb * 2 + 16 * max_front * 2;
    const int64_t single = 16 * max_tc * 2 + 4 * m * 4 + 4096;
    const int64_t per_graph = 64 * graphs + 4 * m + 16 * max_tc * 2 + 16 * max_gth * 2 +
                              8 * (graphs + 1) + 4096;
    const int64_t buffers = 24;  // each rounded up to 256 bytes
    const int64_t t = shared + (multi ? per_graph : single) + 256 * buffers;
    return t + t / 8;
}

void peel_multi(const RankCSR &r, IndexArrays &ix, int64_t *sup_out, int64_t *phi_out,
                const std::vector<int64_t> &off, PeelCounters &pc, Workspace &ws, hipStream_t s) {
    const int64_t m = r.m;
    const int32_t ng = (int32_t)off.size() - 1;
    if (m == 0) return;
    if (2 * ix.n_w >= (int64_t)UINT32_MAX)
        throw Error{BT_EOVERFLOW, "edge-to-wedge links must be below 2^32"};
    const int64_t nb = ix.n_b > 0 ? ix.n_b : 1;
    const int64_t words = (ix.n_w + 31) / 32 + 1;
    const int64_t max_tc = nb + ix.n_w / kWedgeChunk + 1;
    const int64_t max_front = m + 2 * ix.n_w / kLinkChunk + 1;
    const int64_t max_gth = m / kGatherChunk + ng + 1;
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
    P.prof = 0;
    MultiArgs M{};
    M.ctl = ws.get<MultiCtl>("pm_ctl", 1);
    M.gs = ws.get<GState>("pm_gs", ng);
    int32_t *gid = ws.get<int32_t>("pm_gid", m);
    M.gid = gid;
    M.ng = ng;
    M.front[0] = P.front[0];
    M.front[1] = P.front[1];
    M.tc[0] = ws.get<MBloomItem>("pm_tc0", max_tc);
    M.tc[1] = ws.get<MBloomItem>("pm_tc1", max_tc);
    M.gth[0] = ws.get<GatherItem>("pm_gth0", max_gth);
    M.gth[1] = ws.get<GatherItem>("pm_gth1", max_gth);
    int64_t *doff = ws.get<int64_t>("pm_off", ng + 1);

    k_init_peel<<<grid_for(m, 256, 16384), 256, 0, s>>>(ix.supl, m, nullptr, P.sup, P.phi, sup_out);
    BT_CHECK_LAUNCH();
    k_init_alive<<<grid_for(words, 256, 16384), 256, 0, s>>>(ix.cursor, P.alive);
    BT_CHECK_LAUNCH();
    zero_bytes(P.bc, sizeof(int32_t) * nb, s);
    zero_bytes(P.bdone, sizeof(int32_t) * nb, s);
    BT_HIP(hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * (ng + 1), hipMemcpyHostToDevice, s));
    k_multi_init<<<std::min(ng, 4096), 256, 0, s>>>(doff, ng, gid);
    BT_CHECK_LAUNCH();
    // Every graph starts as if round -1 had been a gather that took nothing
    // and saw minimum support 0: round 0 schedules its gather at level 0.
    std::vector<GState> gs(ng);
    int64_t left = 0;
    for (int32_t g = 0; g < ng; ++g) {
        GState &G = gs[g];
        std::memset(&G, 0, sizeof G);
        const int64_t mg = off[g + 1] - off[g];
        G.state = mg > 0 ? kGsNormal : kGsDone;
        G.level = -1;
        G.gmin[0] = INT_MAX;
        G.gmin[1] = 0;
        G.e0 = (int32_t)off[g];
        G.e1 = (int32_t)off[g + 1];
        G.gather_round = -1;
        left += mg > 0 ? 1 : 0;
    }
    BT_HIP(hipMemcpyAsync(M.gs, gs.data(), sizeof(GState) * ng, hipMemcpyHostToDevice, s));
    // The turn on the device comes first: the control block carries the
    // address of its yield word.  A batch peel yields to one of under 1/8 of
    // its edges; BT_PEEL_YIELD=1 makes it stop at every check instead.
    CoopTurn turn(m);
    const char *yv = std::getenv("BT_PEEL_YIELD");
    MultiCtl mc{};
    mc.left.v = (u64)left;
    mc.yield_src = reinterpret_cast<u64>(turn.yield_word(yv && std::atoi(yv) == 1));
    BT_HIP(hipMemcpyAsync(M.ctl, &mc, sizeof mc, hipMemcpyHostToDevice, s));
    GridBar *bar = ws.get<GridBar>("peel_bar", 1);
    zero_bytes(bar, sizeof(GridBar), s);
    int dev = 0, cus = 0, occ = 0;
    BT_HIP(hipGetDevice(&dev));
    BT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    BT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_peel_multi, kPBlock, 0));
    // A large union is bound by atomic throughput rather than by the
    // latency of its rounds, so by default it takes every CU (whole 4,096-
    // graph pool: 9.08 s against 9.40 s with three CUs of four).
    const int pblocks = r.tp.peel_blocks == 0 && m >= kMultiAllCusEdges
                            ? std::max(1, std::min(cus, occ * cus))
                            : peel_grid(r.tp, cus, occ * cus);
    int64_t max_rounds = 8 * m + 64;
    int prof = std::getenv("BT_PEEL_PROFILE") ? 1 : 0;
    hipEvent_t ev0, ev1;
    BT_HIP(hipEventCreate(&ev0));
    BT_HIP(hipEventCreate(&ev1));
    struct EvFree {
        hipEvent_t a, b;
        ~EvFree() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev_free{ev0, ev1};
    void *args[] = {&P, &M, &bar, &max_rounds, &prof};
    MultiCtl hc{};
    for (;;) {
        BT_HIP(hipEventRecord(ev0, s));
        BT_HIP(hipLaunchCooperativeKernel((const void *)k_peel_multi, dim3(pblocks),
                                          dim3(kPBlock), args, 0, s));
        BT_HIP(hipEventRecord(ev1, s));
        int32_t fail = 0;
        BT_HIP(hipMemcpyAsync(&hc, M.ctl, sizeof hc, hipMemcpyDeviceToHost, s));
        BT_HIP(hipMemcpyAsync(&fail, &bar->fail, sizeof fail, hipMemcpyDeviceToHost, s));
        BT_HIP(hipStreamSynchronize(s));
        float t = 0.f;
        BT_HIP(hipEventElapsedTime(&t, ev0, ev1));
        pc.kernel_ms += t;
        pc.launches += 1;
        if (fail) throw Error{BT_EDEVICE, "peel grid barrier timed out"};
        if (hc.left.v == 0) break;
        if (!hc.yielded) throw Error{BT_EDEVICE, "batch peel stopped early"};
        // Each launch that yields has run kMultiYieldEvery rounds.
        if ((int64_t)hc.rounds >= max_rounds) throw Error{BT_EDEVICE, "batch peel made no progress"};
        pc.yields += 1;
        turn.requeue();
        zero_bytes(bar, sizeof(GridBar), s);
    }
    BT_HIP(hipMemcpyAsync(gs.data(), M.gs, sizeof(GState) * ng, hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    pc.rounds = (int64_t)hc.rounds;
    pc.updates = (int64_t)hc.updates.v;
    pc.bloom_visits = (int64_t)hc.bloom_visits.v;
    pc.touched = (int64_t)hc.touched.v;
    if (prof)
        std::fprintf(stderr, "[multi] rounds %llu block0 us: decide %.0f phaseA %.0f bar1 %.0f phaseB+bar2 %.0f\n",
                     hc.rounds, hc.prof[0] / 100.0, hc.prof[1] / 100.0, hc.prof[2] / 100.0,
                     hc.prof[4] / 100.0);
    for (const GState &G : gs) {
        pc.levels = std::max<int64_t>(pc.levels, (int64_t)G.levels);
    }
    k_phi_out<<<grid_for(m, 256, 16384), 256, 0, s>>>(P.phi, phi_out, m);
    BT_CHECK_LAUNCH();
    unsigned long long *mx = ws.get<unsigned long long>("pm_max", 1);
    zero_bytes(mx, sizeof *mx, s);
    k_max_phi<<<grid_for(m, 256, 4096), 256, 0, s>>>(P.phi, m, mx);
    BT_CHECK_LAUNCH();
    unsigned long long hmx = 0;
    BT_HIP(hipMemcpyAsync(&hmx, mx, sizeof hmx, hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    pc.max_phi = (int64_t)hmx;
}

}  // namespace bt
