// wedge.hip - priority-obeyed wedge sweeps: support counting and BE-Index
// emission (Algorithm 3; Lemmas 1-3 and 7).
//
// A task is a start vertex x (or, for heavy x, one range of end vertices z).
// Its workgroup walks every wedge (x, y, z) with p(y), p(z) < p(x) twice:
//   count: c[z] += 1 for each wedge, in an LDS table (hash or dense range);
//          then c[z] = |M(x, z)| is the bloom number of the maximal
//          priority-obeyed bloom anchored by x and z when c[z] >= 2;
//   emit:  each wedge of a bloom (c >= 2) is one twin pair {(x,y), (y,z)};
//          both edges lie in c - 1 butterflies of that bloom (Lemma 2), so
//          their supports grow by c - 1 (exact by Lemma 3), and in index
//          mode the pair is written as a wedge record of the bloom.
// Supports and link counts share one 64-bit word per edge,
// (links << 32) | support, so one atomic adds both; a support is below
// m < 2^31, so the halves never carry into each other.
#include "pipeline.h"

namespace bt {

namespace {

constexpr int kWG = 512;                 // threads per workgroup
constexpr int kNB = kWG;                 // wedge-middle entries per batch
constexpr int kHashCapMax = 4096;        // hash tasks: slots (power of two)
constexpr int kDenseCapMax = 6144;       // dense tasks: counters per range
constexpr int32_t kEmpty = -1;

struct WedgeArgs {
    const int64_t *off;
    const int32_t *adj;
    const int32_t *eid;
    const int32_t *rev;
    const int32_t *low;
    uint64_t *supl;
    int64_t *bf;
    int64_t *queue;  // dynamic task counter
    // index mode
    uint64_t *cursor;
    uint32_t *bwoff;
    int32_t *bk;
    int32_t *wea;
    int32_t *web;
    int32_t *wbl;
};

struct Smem {
    int64_t ystart[kNB];
    int64_t ypre[kNB + 1];
    uint64_t acc[kNB];
    int32_t exy[kNB];
    int64_t scr[kWG / kWave + 2];
    uint64_t scr2[kWG / kWave + 2];
    int64_t task;
    uint64_t base;
    int64_t totals[3];
};

constexpr size_t kTableBytes = (size_t)kHashCapMax * 12 > (size_t)kDenseCapMax * 8
                                   ? (size_t)kHashCapMax * 12
                                   : (size_t)kDenseCapMax * 8;
constexpr size_t kSmemBytes = sizeof(Smem) + kTableBytes;
static_assert(kHashCapMax >= 2 * kHashMaxWorkLimit, "a hash task's table must fit");
static_assert(kDenseCapMax >= kDenseChunkLimit, "a dense task's range must fit");

__device__ __forceinline__ uint32_t hash32(int32_t z) {
    return (uint32_t)z * 2654435761u;
}

// First position in adj[lo, hi) whose value is >= v (rows are ascending).
__device__ __forceinline__ int64_t lower_bound(const int32_t *adj, int64_t lo, int64_t hi,
                                               int32_t v) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (adj[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Largest j in [0, nb) with pre[j] <= idx (pre non-decreasing, pre[0] = 0).
__device__ __forceinline__ int find_batch(const int64_t *pre, int nb, int64_t idx) {
    int lo = 0, hi = nb;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= idx) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <bool DENSE>
__device__ __forceinline__ int slot_insert(int32_t z, int32_t *keys, int32_t mask,
                                           int32_t zlo) {
    if (DENSE) return z - zlo;
    uint32_t h = hash32(z) & (uint32_t)mask;
    while (true) {
        const int32_t k = keys[h];
        if (k == z) return (int)h;
        if (k == kEmpty) {
            const int32_t old = atomicCAS(&keys[h], kEmpty, z);
            if (old == kEmpty || old == z) return (int)h;
        }
        h = (h + 1) & (uint32_t)mask;
    }
}

template <bool DENSE>
__device__ __forceinline__ int slot_find(int32_t z, const int32_t *keys, int32_t mask,
                                         int32_t zlo) {
    if (DENSE) return z - zlo;
    uint32_t h = hash32(z) & (uint32_t)mask;
    while (keys[h] != z) h = (h + 1) & (uint32_t)mask;
    return (int)h;
}

// One pass over the task's wedges.  PASS 0 counts, PASS 1 emits.
template <bool DENSE, bool INDEX, int PASS>
__device__ void wedge_pass(const WedgeArgs &A, Smem &S, int32_t *keys, int32_t *v0,
                           uint32_t *v1, int32_t mask, int32_t x, int32_t zlo, int32_t zhi,
                           uint32_t wbase) {
    const int tid = threadIdx.x;
    const int64_t ox = A.off[x];
    const int32_t lx = A.low[x];
    for (int32_t jb = 0; jb < lx; jb += kNB) {
        const int32_t j = jb + tid;
        int64_t st = 0, len = 0;
        if (j < lx) {
            const int64_t p = ox + j;
            const int32_t y = A.adj[p];
            st = A.off[y];
            len = A.rev[p];
            if (DENSE) {
                const int64_t lo = lower_bound(A.adj, st, st + len, zlo);
                const int64_t hi = lower_bound(A.adj, lo, st + len, zhi);
                st = lo;
                len = hi - lo;
            }
            if (PASS == 1) S.exy[tid] = A.eid[p];
        }
        S.ystart[tid] = st;
        S.acc[tid] = 0;
        int64_t total;
        const int64_t pre = block_exclusive_sum<int64_t>(len, S.scr, &total);
        S.ypre[tid] = pre;
        __syncthreads();
        const int nb = min(kNB, lx - jb);
        for (int64_t idx = tid; idx < total; idx += kWG) {
            const int jj = find_batch(S.ypre, nb, idx);
            const int64_t t = S.ystart[jj] + (idx - S.ypre[jj]);
            const int32_t z = A.adj[t];
            if (PASS == 0) {
                const int sl = slot_insert<DENSE>(z, keys, mask, zlo);
                atomicAdd(&v0[sl], 1);
            } else {
                const int sl = slot_find<DENSE>(z, keys, mask, zlo);
                const int32_t b = v0[sl];
                if (INDEX) {
                    if (b >= 0) {
                        const uint32_t pos = atomicAdd(&v1[sl], 1u);
                        const int64_t w = (int64_t)wbase + pos;
                        const int32_t c = A.bk[b];
                        const int32_t ezy = A.eid[t];
                        A.wea[w] = S.exy[jj];
                        A.web[w] = ezy;
                        A.wbl[w] = b;
                        const uint64_t add = (uint64_t(1) << 32) | (uint32_t)(c - 1);
                        atomicAdd((unsigned long long *)&A.supl[ezy], (unsigned long long)add);
                        atomicAdd((unsigned long long *)&S.acc[jj], (unsigned long long)add);
                    }
                } else if (b >= 2) {
                    const uint64_t add = (uint32_t)(b - 1);
                    atomicAdd((unsigned long long *)&A.supl[A.eid[t]], (unsigned long long)add);
                    atomicAdd((unsigned long long *)&S.acc[jj], (unsigned long long)add);
                }
            }
        }
        __syncthreads();
        if (PASS == 1 && j < lx && S.acc[tid] != 0)
            atomicAdd((unsigned long long *)&A.supl[S.exy[tid]], (unsigned long long)S.acc[tid]);
        __syncthreads();
    }
}

template <bool DENSE, bool INDEX>
__global__ __launch_bounds__(kWG) void k_wedge(WedgeArgs A, const WedgeTask *tasks,
                                               int64_t ntasks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    unsigned char *table = smem_raw + sizeof(Smem);
    const int tid = threadIdx.x;
    while (true) {
        if (tid == 0) S.task = atomicAdd((unsigned long long *)A.queue, 1ull);
        __syncthreads();
        const int64_t ti = S.task;
        __syncthreads();
        if (ti >= ntasks) break;
        const WedgeTask T = tasks[ti];
        const int32_t cap = T.cap;
        int32_t *keys = reinterpret_cast<int32_t *>(table);
        int32_t *v0 = DENSE ? keys : keys + cap;
        uint32_t *v1 = reinterpret_cast<uint32_t *>(v0 + cap);
        for (int s = tid; s < cap; s += kWG) {
            if (!DENSE) keys[s] = kEmpty;
            v0[s] = 0;
        }
        __syncthreads();

        wedge_pass<DENSE, INDEX, 0>(A, S, keys, v0, v1, cap - 1, T.x, T.zlo, T.zhi, 0);

        // Sweep 1: blooms, their wedges and butterflies in this task.
        int64_t nb = 0, nw = 0, bfl = 0;
        for (int s = tid; s < cap; s += kWG) {
            const int32_t c = (DENSE || keys[s] != kEmpty) ? v0[s] : 0;
            if (c >= 2) {
                ++nb;
                nw += c;
                bfl += (int64_t)c * (c - 1) / 2;
            }
        }
        nb = wave_sum(nb);
        nw = wave_sum(nw);
        bfl = wave_sum(bfl);
        if (tid == 0) S.totals[0] = S.totals[1] = S.totals[2] = 0;
        __syncthreads();
        if (lane_id() == 0) {
            atomicAdd((unsigned long long *)&S.totals[0], (unsigned long long)nb);
            atomicAdd((unsigned long long *)&S.totals[1], (unsigned long long)nw);
            atomicAdd((unsigned long long *)&S.totals[2], (unsigned long long)bfl);
        }
        __syncthreads();
        if (tid == 0) {
            if (S.totals[2]) atomicAdd((unsigned long long *)A.bf, (unsigned long long)S.totals[2]);
            S.base = 0;
            if (INDEX && S.totals[0])
                S.base = atomicAdd((unsigned long long *)A.cursor,
                                   ((unsigned long long)S.totals[0] << 32) |
                                       (unsigned long long)S.totals[1]);
        }
        __syncthreads();
        if (S.totals[0] == 0) continue;  // no bloom anchored here
        const uint32_t bbase = (uint32_t)(S.base >> 32);
        const uint32_t wbase = (uint32_t)(S.base & 0xffffffffu);

        if (INDEX) {
            // Sweep 2: number blooms and lay out their wedge ranges in slot
            // order; blooms and wedges share one allocation order, so bloom
            // b's range ends where bloom b + 1's begins.
            uint64_t carry = 0;
            for (int s0 = 0; s0 < cap; s0 += kWG) {
                const int s = s0 + tid;
                const bool valid = s < cap && (DENSE || keys[s] != kEmpty);
                const int32_t c = valid ? v0[s] : 0;
                const bool isb = c >= 2;
                const uint64_t mine = isb ? ((uint64_t(1) << 32) | (uint32_t)c) : 0;
                uint64_t tot;
                const uint64_t pre = block_exclusive_sum<uint64_t>(mine, S.scr2, &tot) + carry;
                if (isb) {
                    const int32_t b = (int32_t)(bbase + (uint32_t)(pre >> 32));
                    const uint32_t lw = (uint32_t)(pre & 0xffffffffu);
                    A.bk[b] = c;
                    A.bwoff[b] = wbase + lw;
                    v0[s] = b;
                    v1[s] = lw;
                } else if (valid) {
                    v0[s] = kEmpty;
                }
                carry += tot;
            }
            __syncthreads();
        }

        wedge_pass<DENSE, INDEX, 1>(A, S, keys, v0, v1, cap - 1, T.x, T.zlo, T.zhi, wbase);
    }
}

__global__ void k_supl_to_sup(const uint64_t *supl, int64_t *sup, int64_t m) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        sup[e] = (int64_t)(supl[e] & 0xffffffffu);
}

// Sum of the supports (low halves of the packed words).
__global__ void k_support_total(const uint64_t *supl, int64_t m, unsigned long long *out) {
    unsigned long long acc = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        acc += supl[e] & 0xffffffffu;
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(out, acc);
}

__global__ void k_link_counts(const uint64_t *supl, int64_t m, int32_t *cnt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        cnt[e] = (int32_t)(supl[e] >> 32);
}

// Scatter each wedge, with its bloom and the edge's twin, into the link lists of its two
// edges.  The link count in the high half of supl is consumed as a cursor (counting down).
__global__ void k_link_scatter(const int32_t *wea, const int32_t *web, const int32_t *wbl,
                               const uint64_t *cursor, uint64_t *supl, const int64_t *link_off,
                               uint3 *link) {
    const int64_t nw = (int64_t)(*cursor & 0xffffffffu);
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int32_t ea = wea[w], eb = web[w];
        const uint32_t b = (uint32_t)wbl[w];
        const uint64_t oa = atomicAdd((unsigned long long *)&supl[ea],
                                      (unsigned long long)(-(int64_t)(uint64_t(1) << 32)));
        link[link_off[ea] + (int64_t)(oa >> 32) - 1] = make_uint3((uint32_t)w, b, (uint32_t)eb);
        const uint64_t ob = atomicAdd((unsigned long long *)&supl[eb],
                                      (unsigned long long)(-(int64_t)(uint64_t(1) << 32)));
        link[link_off[eb] + (int64_t)(ob >> 32) - 1] = make_uint3((uint32_t)w, b, (uint32_t)ea);
    }
}

__global__ void k_bloom_sentinel(const uint64_t *cursor, uint32_t *bwoff) {
    const uint64_t c = *cursor;
    bwoff[c >> 32] = (uint32_t)(c & 0xffffffffu);
}

template <bool DENSE, bool INDEX>
void launch_wedge(const WedgeArgs &A, const WedgeTask *tasks, int64_t n, int wg_per_cu,
                  hipStream_t s) {
    if (n <= 0) return;
    zero_bytes(A.queue, sizeof(int64_t), s);
    int dev = 0, cus = 0;
    BT_HIP(hipGetDevice(&dev));
    BT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t grid = std::min<int64_t>(n, (int64_t)cus * wg_per_cu);
    k_wedge<DENSE, INDEX><<<(unsigned)grid, kWG, kSmemBytes, s>>>(A, tasks, n);
    BT_CHECK_LAUNCH();
}

WedgeArgs make_args(const RankCSR &r, uint64_t *supl, int64_t *bf, int64_t *queue) {
    WedgeArgs A{};
    A.off = r.off;
    A.adj = r.adj;
    A.eid = r.eid;
    A.rev = r.rev;
    A.low = r.low;
    A.supl = supl;
    A.bf = bf;
    A.queue = queue;
    return A;
}

}  // namespace

void supl_to_sup(const uint64_t *supl, int64_t *sup, int64_t m, hipStream_t s) {
    if (m <= 0) return;
    k_supl_to_sup<<<grid_for(m, 256, 16384), 256, 0, s>>>(supl, sup, m);
    BT_CHECK_LAUNCH();
}

void check_butterfly_total(const uint64_t *supl, int64_t m, const int64_t *butterflies,
                           Workspace &ws, hipStream_t s) {
    if (m <= 0) return;
    unsigned long long *tot = ws.get<unsigned long long>("bf_check", 1);
    zero_bytes(tot, sizeof *tot, s);
    k_support_total<<<grid_for(m, 256, 4096), 256, 0, s>>>(supl, m, tot);
    BT_CHECK_LAUNCH();
    int64_t *h = ws.host(2);
    BT_HIP(hipMemcpyAsync(h, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipMemcpyAsync(h + 1, butterflies, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    if (h[0] != 4 * h[1])
        throw Error{BT_EDEVICE, "butterfly totals disagree: supports sum to " +
                                    std::to_string(h[0]) + ", blooms give 4 x " +
                                    std::to_string(h[1])};
}

void count_support(const RankCSR &r, const TaskLists &t, uint64_t *supl, int64_t *bf,
                   hipStream_t s) {
    static_assert(kSmemBytes <= 65536, "LDS budget");
    int64_t *queue = reinterpret_cast<int64_t *>(bf) + 1;  // caller gives 2 scalars
    WedgeArgs A = make_args(r, supl, bf, queue);
    launch_wedge<true, false>(A, t.dense, t.n_dense, r.tp.wedge_wg_per_cu, s);
    launch_wedge<false, false>(A, t.hash, t.n_hash, r.tp.wedge_wg_per_cu, s);
}

void build_index(const RankCSR &r, const TaskLists &t, IndexArrays &ix, Workspace &ws,
                 hipStream_t s) {
    int64_t *queue = ws.get<int64_t>("wedge_queue", 1);
    WedgeArgs A = make_args(r, ix.supl, ix.butterflies, queue);
    A.cursor = ix.cursor;
    A.bwoff = ix.bwoff;
    A.bk = ix.bk;
    A.wea = ix.wea;
    A.web = ix.web;
    A.wbl = ix.wbl;
    launch_wedge<true, true>(A, t.dense, t.n_dense, r.tp.wedge_wg_per_cu, s);
    launch_wedge<false, true>(A, t.hash, t.n_hash, r.tp.wedge_wg_per_cu, s);
    k_bloom_sentinel<<<1, 1, 0, s>>>(ix.cursor, ix.bwoff);
    BT_CHECK_LAUNCH();

    // Links: per-edge counts -> offsets -> scatter.
    const int64_t m = r.m;
    int32_t *cnt = ws.get<int32_t>("link_cnt", m);
    if (m > 0) {
        k_link_counts<<<grid_for(m, 256, 16384), 256, 0, s>>>(ix.supl, m, cnt);
        BT_CHECK_LAUNCH();
    }
    scan_exclusive_i32_to_i64(cnt, ix.link_off, m, ws, s);
    k_link_scatter<<<grid_for(ix.cap_w, 256, 65536), 256, 0, s>>>(
        ix.wea, ix.web, ix.wbl, ix.cursor, ix.supl, ix.link_off, ix.link);
    BT_CHECK_LAUNCH();
}

}  // namespace bt
