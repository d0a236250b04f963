// peel.hip - bulk-synchronous peel through blooms (Algorithm 5: batch edge
// and batch bloom processing).
//
// State: sup (int32, unclamped), phi (int32, -1 while the edge remains),
// one alive bit per wedge, per bloom its live wedge count k and the count C
// of wedges removed this round.  A round with level L and frontier F (the
// remaining edges with support <= L):
//   A. every edge of F gets phi = L; for each of its wedges still alive the
//      wedge is killed (one winner per wedge), C[B] += 1 for its bloom B and
//      the twin edge loses all of its k[B] - 1 butterflies in B;
//   B. in every bloom touched in A, each surviving wedge's two edges lose
//      C[B] butterflies (the bloom shrinks from k to k - C), then
//      k[B] -= C[B], C[B] = 0; once k[B] <= 1 the bloom holds no butterfly
//      and its last wedge is retired.
// The paper clamps decremented supports at the round's minimum (max(MBS,
// .)); subtracting unclamped and treating every support <= L as "at level
// L" gives the same bitruss numbers, since max(M, max(M, a - d1) - d2) =
// max(M, a - d1 - d2).  A decrement that takes a support from above L to
// at most L puts the edge in the next frontier; when a frontier is empty
// the level rises to the minimum remaining support.
#include <climits>

#include "pipeline.h"

namespace bt {

namespace {

constexpr int kBlock = 256;

struct PeelCtl {
    int32_t n_front;
    int32_t n_next;
    int32_t n_touched;
    int32_t level;
    int32_t min_sup;
    int32_t pad;
    unsigned long long updates;
    unsigned long long bloom_visits;
};

__device__ __forceinline__ void dec_support(int32_t *sup, int32_t e, int32_t d, int32_t level,
                                            bool active, int32_t *next, int32_t *n_next) {
    bool push = false;
    if (active) {
        const int32_t old = atomicSub(&sup[e], d);
        push = old > level && old - d <= level;
    }
    wave_push(push, e, next, n_next);
}

// Phase A: one wave per frontier edge, lanes over its links.
__global__ __launch_bounds__(kBlock) void k_phase_a(
    const int32_t *front, PeelCtl *ctl, const int64_t *link_off, const uint32_t *link,
    const int32_t *wea, const int32_t *web, const int32_t *wbl, uint32_t *alive,
    const int32_t *bk, int32_t *bc, int32_t *touched, int32_t *sup, int32_t *phi,
    int32_t *next) {
    const int32_t nf = ctl->n_front;
    const int32_t level = ctl->level;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    unsigned long long upd = 0;
    for (int64_t i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < nf; i += waves) {
        const int32_t e = front[i];
        if (lane_id() == 0) phi[e] = level;
        const int64_t a = link_off[e], b = link_off[(int64_t)e + 1];
        for (int64_t j0 = a; j0 < b; j0 += kWave) {
            const int64_t j = j0 + lane_id();
            bool won = false;
            int32_t blm = 0, twin = 0, d = 0;
            if (j < b) {
                const uint32_t w = link[j];
                const uint32_t bit = 1u << (w & 31);
                if (alive[w >> 5] & bit) {
                    const uint32_t old = atomicAnd(&alive[w >> 5], ~bit);
                    if (old & bit) {
                        won = true;
                        blm = wbl[w];
                        const int32_t ea = wea[w];
                        twin = ea == e ? web[w] : ea;
                        d = bk[blm] - 1;
                    }
                }
            }
            bool first = false;
            if (won) first = atomicAdd(&bc[blm], 1) == 0;
            wave_push(first, blm, touched, &ctl->n_touched);
            dec_support(sup, twin, d, level, won && d > 0, next, &ctl->n_next);
            upd += (won && d > 0) ? 1 : 0;
        }
    }
    upd = wave_sum(upd);
    if (lane_id() == 0 && upd) atomicAdd(&ctl->updates, upd);
}

// Phase B: one wave per touched bloom, lanes over its wedge range.
__global__ __launch_bounds__(kBlock) void k_phase_b(
    const int32_t *touched, PeelCtl *ctl, const uint32_t *bwoff, const int32_t *wea,
    const int32_t *web, uint32_t *alive, int32_t *bk, int32_t *bc, int32_t *sup,
    int32_t *next) {
    const int32_t nt = ctl->n_touched;
    const int32_t level = ctl->level;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    unsigned long long upd = 0;
    for (int64_t i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < nt; i += waves) {
        const int32_t blm = touched[i];
        const int32_t c = bc[blm];
        const int32_t kn = bk[blm] - c;
        const uint32_t w0 = bwoff[blm], w1 = bwoff[blm + 1];
        if (kn > 0) {
            for (uint32_t wb = w0; wb < w1; wb += kWave) {
                const uint32_t w = wb + lane_id();
                bool live = false;
                if (w < w1) live = (alive[w >> 5] >> (w & 31)) & 1u;
                dec_support(sup, live ? wea[w] : 0, c, level, live, next, &ctl->n_next);
                dec_support(sup, live ? web[w] : 0, c, level, live, next, &ctl->n_next);
                upd += live ? 2 : 0;
                if (live && kn <= 1) atomicAnd(&alive[w >> 5], ~(1u << (w & 31)));
            }
        }
        if (lane_id() == 0) {
            bk[blm] = kn;
            bc[blm] = 0;
        }
    }
    upd = wave_sum(upd);
    if (lane_id() == 0 && upd) atomicAdd(&ctl->updates, upd);
}

// Round bookkeeping: next frontier becomes current; counts reset.
__global__ void k_advance(PeelCtl *ctl) {
    ctl->bloom_visits += (unsigned long long)ctl->n_touched;
    ctl->n_front = ctl->n_next;
    ctl->n_next = 0;
    ctl->n_touched = 0;
}

__global__ __launch_bounds__(kBlock) void k_min_alive(const int32_t *sup, const int32_t *phi,
                                                      int64_t m, PeelCtl *ctl) {
    int32_t mn = INT_MAX;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        if (phi[e] < 0 && sup[e] < mn) mn = sup[e];
    mn = wave_min(mn);
    if (lane_id() == 0 && mn != INT_MAX) atomicMin(&ctl->min_sup, mn);
}

__global__ __launch_bounds__(kBlock) void k_gather(const int32_t *sup, const int32_t *phi,
                                                   int64_t m, PeelCtl *ctl, int32_t *front) {
    const int32_t mn = ctl->min_sup;
    if (mn == INT_MAX) return;
    const int32_t level = mn > ctl->level ? mn : ctl->level;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->pad = level;
    for (int64_t e0 = blockIdx.x * (int64_t)blockDim.x; e0 < m;
         e0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e0 + threadIdx.x;
        const bool take = e < m && phi[e] < 0 && sup[e] <= level;
        wave_push(take, (int32_t)e, front, &ctl->n_front);
    }
}

__global__ void k_set_level(PeelCtl *ctl) {
    ctl->level = ctl->pad;
    ctl->min_sup = INT_MAX;
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

}  // namespace

void peel(const RankCSR &r, IndexArrays &ix, int64_t *sup_out, int64_t *phi_out,
          PeelCounters &pc, Workspace &ws, hipStream_t s) {
    const int64_t m = r.m;
    if (m == 0) return;
    int32_t *sup = ws.get<int32_t>("peel_sup", m);
    int32_t *phi = ws.get<int32_t>("peel_phi", m);
    int32_t *fa = ws.get<int32_t>("peel_front_a", m);
    int32_t *fb = ws.get<int32_t>("peel_front_b", m);
    int32_t *touched = ws.get<int32_t>("peel_touched", ix.n_b > 0 ? ix.n_b : 1);
    int32_t *bc = ws.get<int32_t>("peel_bc", ix.n_b > 0 ? ix.n_b : 1);
    uint32_t *alive = ws.get<uint32_t>("peel_alive", (ix.n_w + 31) / 32 + 1);
    PeelCtl *ctl = ws.get<PeelCtl>("peel_ctl", 1);

    k_init_peel<<<grid_for(m, 256, 16384), 256, 0, s>>>(ix.supl, m, sup, phi, sup_out);
    BT_CHECK_LAUNCH();
    k_init_alive<<<grid_for((ix.n_w + 31) / 32, 256, 16384), 256, 0, s>>>(ix.cursor, alive);
    BT_CHECK_LAUNCH();
    if (ix.n_b > 0) BT_HIP(hipMemsetAsync(bc, 0, sizeof(int32_t) * ix.n_b, s));
    PeelCtl init{};
    init.min_sup = INT_MAX;
    BT_HIP(hipMemcpyAsync(ctl, &init, sizeof init, hipMemcpyHostToDevice, s));

    PeelCtl *hctl = reinterpret_cast<PeelCtl *>(host_scalars(8));
    int64_t remaining = m;
    int32_t *front = fa, *next = fb;
    const int scan_grid = grid_for(m, kBlock, 4096);
    while (remaining > 0) {
        BT_HIP(hipMemcpyAsync(hctl, ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
        BT_HIP(hipStreamSynchronize(s));
        int32_t nf = hctl->n_front;
        if (nf == 0) {
            k_min_alive<<<scan_grid, kBlock, 0, s>>>(sup, phi, m, ctl);
            BT_CHECK_LAUNCH();
            k_gather<<<scan_grid, kBlock, 0, s>>>(sup, phi, m, ctl, front);
            BT_CHECK_LAUNCH();
            k_set_level<<<1, 1, 0, s>>>(ctl);
            BT_CHECK_LAUNCH();
            BT_HIP(hipMemcpyAsync(hctl, ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
            BT_HIP(hipStreamSynchronize(s));
            nf = hctl->n_front;
            if (nf == 0) break;  // nothing remains
            ++pc.levels;
            if (hctl->level > pc.max_phi) pc.max_phi = hctl->level;
        }
        ++pc.rounds;
        remaining -= nf;
        const int ga = grid_for((int64_t)nf * kWave, kBlock, 16384);
        k_phase_a<<<ga, kBlock, 0, s>>>(front, ctl, ix.link_off, ix.link, ix.wea, ix.web, ix.wbl,
                                         alive, ix.bk, bc, touched, sup, phi, next);
        BT_CHECK_LAUNCH();
        k_phase_b<<<16384, kBlock, 0, s>>>(touched, ctl, ix.bwoff, ix.wea, ix.web, alive, ix.bk,
                                           bc, sup, next);
        BT_CHECK_LAUNCH();
        k_advance<<<1, 1, 0, s>>>(ctl);
        BT_CHECK_LAUNCH();
        std::swap(front, next);
    }
    BT_HIP(hipMemcpyAsync(hctl, ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    pc.updates = (int64_t)hctl->updates;
    pc.bloom_visits = (int64_t)hctl->bloom_visits;
    k_phi_out<<<grid_for(m, 256, 16384), 256, 0, s>>>(phi, phi_out, m);
    BT_CHECK_LAUNCH();
}

}  // namespace bt
