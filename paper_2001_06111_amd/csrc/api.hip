// api.hip - the C ABI: argument checks, workspace, stage orchestration.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>

#include "pipeline.h"

namespace bt {

namespace {

struct Library {
    std::mutex mu;
    Workspace ws;
};

Library &lib() {
    static Library *L = new Library();  // never destroyed: outlives static teardown
    return *L;
}

template <class F> bt_status guard(F &&f) {
    try {
        f();
        return BT_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return BT_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return BT_EDEVICE;
    }
}

}  // namespace

void check_graph(const bt_csr *g) {
    if (!g) throw Error{BT_EINVAL, "graph descriptor is NULL"};
    if (g->n_upper < 0 || g->n_lower < 0 || g->m < 0)
        throw Error{BT_EINVAL, "negative size in graph descriptor"};
    if ((int64_t)g->n_upper + g->n_lower >= INT32_MAX)
        throw Error{BT_EOVERFLOW, "n_upper + n_lower must be below 2^31"};
    if (g->m >= INT32_MAX) throw Error{BT_EOVERFLOW, "m must be below 2^31"};
    if (!g->row_ptr) throw Error{BT_EINVAL, "row_ptr is NULL"};
    if (g->m > 0 && !g->col) throw Error{BT_EINVAL, "col is NULL"};
}

namespace {

struct Events {
    bool on = false;
    hipEvent_t ev[5] = {};
    hipStream_t s = nullptr;
    Events(bool enable, hipStream_t st) : on(enable), s(st) {
        if (on)
            for (auto &e : ev) BT_HIP(hipEventCreate(&e));
    }
    ~Events() {
        if (on)
            for (auto &e : ev) (void)hipEventDestroy(e);
    }
    void mark(int i) {
        if (on) BT_HIP(hipEventRecord(ev[i], s));
    }
    float ms(int a, int b) {
        if (!on) return 0.f;
        float t = 0.f;
        BT_HIP(hipEventElapsedTime(&t, ev[a], ev[b]));
        return t;
    }
};

// Sizes the index from the wedge bound and points `ix` at buffers.
void alloc_index(const RankCSR &r, IndexArrays &ix, bool owned, Workspace &ws,
                 std::vector<void *> *own) {
    if (r.wedges_po >= (int64_t)UINT32_MAX)
        throw Error{BT_EOVERFLOW, "priority-obeyed wedges must be below 2^32"};
    ix.cap_w = r.wedges_po;
    ix.cap_b = r.wedges_po / 2;
    const int64_t m = r.m;
    auto get = [&](const char *name, size_t bytes) -> void * {
        if (!owned) return ws.get(name, bytes);
        void *p = device_alloc(bytes ? bytes : 256);
        own->push_back(p);
        return p;
    };
    ix.bwoff = (uint32_t *)get("ix_bwoff", sizeof(uint32_t) * (ix.cap_b + 1));
    ix.bk = (int32_t *)get("ix_bk", sizeof(int32_t) * (ix.cap_b + 1));
    ix.wea = (int32_t *)get("ix_wea", sizeof(int32_t) * (ix.cap_w + 1));
    ix.web = (int32_t *)get("ix_web", sizeof(int32_t) * (ix.cap_w + 1));
    ix.wbl = (int32_t *)get("ix_wbl", sizeof(int32_t) * (ix.cap_w + 1));
    ix.supl = (uint64_t *)get("ix_supl", sizeof(uint64_t) * (m + 1));
    ix.link_off = (int64_t *)get("ix_link_off", sizeof(int64_t) * (m + 1));
    ix.link = (uint3 *)get("ix_link", sizeof(uint3) * (2 * ix.cap_w + 1));
    ix.cursor = (uint64_t *)get("ix_cursor", sizeof(uint64_t) * 2);
    ix.butterflies = (int64_t *)(ix.cursor + 1);
}

int64_t index_bytes(const IndexArrays &ix, int64_t m) {
    return (int64_t)(sizeof(uint32_t) + 2 * sizeof(int32_t)) * (ix.n_b + 1) +
           (int64_t)(3 * sizeof(int32_t) + 2 * sizeof(uint3)) * ix.n_w +
           (int64_t)(sizeof(uint64_t) + sizeof(int64_t) + sizeof(int32_t) * 2) * m +
           (ix.n_w + 31) / 32 * 4;
}

// prepare -> tasks -> counting + emission + links.  Reads back the sizes.
void build_all(const bt_csr &g, RankCSR &r, IndexArrays &ix, bool owned,
               std::vector<void *> *own, Workspace &ws, hipStream_t s, Events *ev,
               bool batch = false, const Components *comps = nullptr) {
    prepare(g, r, ws, s, comps);
    if (batch) r.tp = tune_params(true, g.m);
    TaskLists t;
    make_tasks(r, t, ws, s);
    if (ev) ev->mark(1);
    alloc_index(r, ix, owned, ws, own);
    zero_bytes(ix.supl, sizeof(uint64_t) * (r.m + 1), s);
    zero_bytes(ix.cursor, sizeof(uint64_t) * 2, s);
    build_index(r, t, ix, ws, s);
    if (ev) ev->mark(2);
    check_butterfly_total(ix.supl, r.m, ix.butterflies, ws, s);
    int64_t *hs = ws.host(4);
    BT_HIP(hipMemcpyAsync(hs, ix.cursor, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    const uint64_t c = (uint64_t)hs[0];
    ix.n_b = (int64_t)(c >> 32);
    ix.n_w = (int64_t)(c & 0xffffffffu);
}

}  // namespace

namespace {
void fill_stats(bt_stats *stats, const RankCSR &r, const IndexArrays &ix, const PeelCounters &pc,
                int64_t m, int64_t butterflies, Events &ev) {
    std::memset(stats, 0, sizeof *stats);
    stats->butterflies = butterflies;
    stats->wedges_po = r.wedges_po;
    stats->blooms = ix.n_b;
    stats->bloom_wedges = ix.n_w;
    stats->index_bytes = index_bytes(ix, m);
    stats->levels = pc.levels;
    stats->rounds = pc.rounds;
    stats->max_phi = pc.max_phi;
    stats->support_updates = pc.updates;
    stats->bloom_visits = pc.bloom_visits;
    stats->ms_prepare = ev.ms(0, 1);
    stats->ms_count = ev.ms(1, 2);
    stats->ms_link = ev.ms(2, 3);
    stats->ms_peel = ev.ms(3, 4);
    stats->ms_peel_kernel = (float)pc.kernel_ms;
    stats->peel_launches = (int32_t)pc.launches;
    stats->passes = 1;
    stats->support_updates_unbatched = pc.updates_unbatched;
    stats->wedge_visits = pc.touched;
    stats->peel_yields = pc.yields;
}

const uint32_t *reorder_union(bt_csr &u, const int64_t *dvoff, int32_t ng, Workspace &ws,
                              hipStream_t s);

// Graphs from this many edges up are decomposed in the locality order (see
// reorder_union); BT_REORDER=0 keeps the caller's numbering.
constexpr int64_t kReorderMinEdges = int64_t(1) << 20;

bool reorder_single(int64_t m) {
    const char *v = std::getenv("BT_REORDER");
    return m >= kReorderMinEdges && !(v && std::atoi(v) == 0);
}

// out[perm[p]] = t[p]: results back to the caller's edge order.
__global__ void k_unpermute(const uint32_t *perm, int64_t m, const int64_t *sup_t,
                            const int64_t *phi_t, int64_t *sup_out, int64_t *phi_out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = perm[p];
        if (sup_out) sup_out[e] = sup_t[p];
        phi_out[e] = phi_t[p];
    }
}

}  // namespace

void decompose_impl(const bt_csr &g0, int64_t *sup_out0, int64_t *phi_out0, bt_stats *stats,
                    Workspace &ws, hipStream_t stream, bool unit_updates, bool auto_pc) {
    Events ev(stats != nullptr, stream);
    ev.mark(0);
    // Large graphs peel in the locality order (each layer renumbered by
    // decreasing degree, edges re-sorted), as batches do; the graph is
    // validated first, since the reorder indexes by its ids.
    bt_csr g = g0;
    int64_t *sup_out = sup_out0, *phi_out = phi_out0;
    const uint32_t *perm = nullptr;
    if (phi_out0 && reorder_single(g0.m)) {
        validate_graph(g0, ws, stream);
        int64_t *dvoff = ws.get<int64_t>("reo_voff1", 4);
        const int64_t hv[4] = {0, (int64_t)g0.n_lower, 0, (int64_t)g0.n_upper};
        BT_HIP(hipMemcpyAsync(dvoff, hv, sizeof hv, hipMemcpyHostToDevice, stream));
        perm = reorder_union(g, dvoff, 1, ws, stream);
        if (perm) {
            if (sup_out0) sup_out = ws.get<int64_t>("reo_sup", g0.m);
            phi_out = ws.get<int64_t>("reo_phi", g0.m);
        }
    }
    RankCSR r;
    IndexArrays ix;
    build_all(g, r, ix, false, nullptr, ws, stream, &ev);
    ev.mark(3);
    if (auto_pc && g.m > 0) {
        // Where support updates, not rounds, bound the peel (hub-heavy
        // graphs), BiT-PC's smaller updates pay for its extra passes.
        int64_t *hb = ws.host(2);
        BT_HIP(hipMemcpyAsync(hb, ix.butterflies, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        BT_HIP(hipStreamSynchronize(stream));
        if (hb[0] / g.m >= kAutoPcButterfliesPerEdge) {
            decompose_pc_impl(g0, kAutoPcTau, sup_out0, phi_out0, stats, ws, stream);
            return;
        }
    }
    PeelCounters pc;
    PeelOptions o;
    o.unit_updates = unit_updates;
    peel(r, ix, sup_out, phi_out, pc, ws, stream, &o);
    if (perm) {
        k_unpermute<<<grid_for(g0.m, 256, 16384), 256, 0, stream>>>(
            perm, g0.m, sup_out0 ? sup_out : nullptr, phi_out, sup_out0, phi_out0);
        BT_CHECK_LAUNCH();
    }
    ev.mark(4);
    int64_t *hs = ws.host(2);
    BT_HIP(hipMemcpyAsync(hs, ix.butterflies, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    BT_HIP(hipStreamSynchronize(stream));
    if (stats) fill_stats(stats, r, ix, pc, g.m, hs[0], ev);
}

float index_build_ms(const bt_csr &g, Workspace &ws, hipStream_t stream) {
    Events ev(true, stream);
    ev.mark(0);
    RankCSR r;
    IndexArrays ix;
    build_all(g, r, ix, false, nullptr, ws, stream, &ev);
    ev.mark(3);
    BT_HIP(hipStreamSynchronize(stream));
    return ev.ms(0, 3);
}

// BiT-PC (Section V-C, Algorithm 7).  Supports in G and k_max; then for
// eps = k_max, k_max - alpha, ..., 0 (alpha = ceil(k_max tau)): the
// subgraph G_{>=eps}, its BE-Index with the already fixed edges marked
// (Algorithm 6), and a peel whose first level is eps - 1, so that one level
// removes every edge outside the eps-bitruss (whose numbers are < eps and
// left for later passes) and the levels from eps up fix the numbers of the
// eps-bitruss.  Algorithm 7's single recount-and-drop of edges below eps is
// subsumed by that first level, which repeats it to the fixpoint.
void decompose_pc_impl(const bt_csr &g, double tau, int64_t *sup_out, int64_t *phi_out,
                       bt_stats *stats, Workspace &ws, hipStream_t s) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    const int64_t m = g.m;
    Events ev(stats != nullptr, s);
    ev.mark(0);
    RankCSR r;
    prepare(g, r, ws, s);
    TaskLists t;
    make_tasks(r, t, ws, s);
    ev.mark(1);
    uint64_t *supl = ws.get<uint64_t>("pc_supl", m + 1);
    int64_t *bf = ws.get<int64_t>("pc_bf", 2);
    zero_bytes(supl, sizeof(uint64_t) * (m + 1), s);
    zero_bytes(bf, sizeof(int64_t) * 2, s);
    count_support(r, t, supl, bf, s);
    check_butterfly_total(supl, m, bf, ws, s);
    if (sup_out && m) supl_to_sup(supl, sup_out, m, s);
    int32_t *sup0 = ws.get<int32_t>("pc_sup0", m);
    const int32_t kmax = pc_kmax(supl, m, sup0, ws, s);
    ev.mark(2);
    int64_t *hs = ws.host(2);
    BT_HIP(hipMemcpyAsync(hs, bf, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    const int64_t butterflies = hs[0];
    const int64_t wedges_po = r.wedges_po;
    int32_t *phi_glob = ws.get<int32_t>("pc_phi", m);
    int64_t *phi_sub = ws.get<int64_t>("pc_phisub", m);
    if (m) fill_i32(phi_glob, -1, m, s);
    const int32_t alpha =
        std::max<int32_t>(1, (int32_t)std::min<double>(std::ceil(kmax * tau), INT32_MAX));
    PeelCounters tot;
    int64_t blooms = 0, bloom_wedges = 0, idx_bytes = 0;
    int32_t passes = 0;
    for (int32_t eps = kmax; m > 0;) {
        PcSubgraph sg;
        pc_subgraph(g, sup0, eps, phi_glob, sg, ws, s);
        if (sg.open > 0) {
            RankCSR rs;
            IndexArrays ix;
            build_all(sg.g, rs, ix, false, nullptr, ws, s, nullptr);
            mark_fixed(ix, sg.fixed, s);
            PeelOptions o;
            o.fixed = sg.fixed;
            o.min_level = eps > 0 ? eps - 1 : 0;
            PeelCounters pc;
            peel(rs, ix, nullptr, phi_sub, pc, ws, s, &o);
            pc_collect(phi_sub, sg, eps, phi_glob, s);
            tot.levels += pc.levels;
            tot.rounds += pc.rounds;
            if (pc.max_phi >= eps) tot.max_phi = std::max(tot.max_phi, pc.max_phi);
            tot.updates += pc.updates;
            tot.bloom_visits += pc.bloom_visits;
            tot.touched += pc.touched;
            tot.yields += pc.yields;
            tot.kernel_ms += pc.kernel_ms;
            tot.launches += pc.launches;
            blooms += ix.n_b;
            bloom_wedges += ix.n_w;
            idx_bytes = std::max(idx_bytes, index_bytes(ix, sg.g.m));
            passes += 1;
        }
        if (eps == 0) break;
        eps = std::max(eps - alpha, 0);
    }
    pc_widen(phi_glob, m, phi_out, s);
    ev.mark(3);
    ev.mark(4);
    BT_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->butterflies = butterflies;
        stats->wedges_po = wedges_po;
        stats->blooms = blooms;
        stats->bloom_wedges = bloom_wedges;
        stats->index_bytes = idx_bytes;
        stats->levels = tot.levels;
        stats->rounds = tot.rounds;
        stats->max_phi = tot.max_phi;
        stats->support_updates = tot.updates;
        stats->bloom_visits = tot.bloom_visits;
        stats->ms_prepare = ev.ms(0, 1);
        stats->ms_count = ev.ms(1, 2);
        stats->ms_link = 0.f;
        stats->ms_peel = ev.ms(2, 3);  // every pass: subgraph, index, peel
        stats->ms_peel_kernel = (float)tot.kernel_ms;
        stats->peel_launches = (int32_t)tot.launches;
        stats->passes = passes;
        stats->wedge_visits = tot.touched;
        stats->peel_yields = tot.yields;
    }
}

constexpr int64_t kMultiMaxEdges = int64_t(1) << 19;
constexpr int64_t kTraceMaxEdges = int64_t(1) << 16;

// A disjoint union of graphs (edge ranges [off[g], off[g+1])): one index
// build for the union, then one peel in which every graph has its own level.
void decompose_union_impl(const bt_csr &u, const std::vector<int64_t> &off,
                          const Components &comps, int64_t *sup_out, int64_t *phi_out,
                          bt_stats *stats, Workspace &ws, hipStream_t s,
                          const SizedHook *on_sized = nullptr) {
    Events ev(stats != nullptr, s);
    ev.mark(0);
    RankCSR r;
    IndexArrays ix;
    build_all(u, r, ix, false, nullptr, ws, s, &ev, off.size() > 2, &comps);
    ev.mark(3);
    PeelCounters pc;
    // Per-graph levels pay when there are several graphs, all small: its
    // gathers rescan a graph's whole edge range, where the shared-level peel
    // keeps a threshold active set.  BT_BATCH_PEEL=union forces the latter.
    int64_t max_m = 0;
    for (size_t g = 0; g + 1 < off.size(); ++g) max_m = std::max(max_m, off[g + 1] - off[g]);
    const char *mode = std::getenv("BT_BATCH_PEEL");
    const bool multi = ws.coop && off.size() > 2 && max_m <= kMultiMaxEdges &&
                       !(mode && std::strcmp(mode, "union") == 0);
    if (on_sized && *on_sized)
        (*on_sized)((int64_t)ws.bytes(),
                    peel_state_bytes(u.m, ix.n_b, ix.n_w, (int64_t)off.size() - 1, multi));
    if (multi)
        peel_multi(r, ix, sup_out, phi_out, off, pc, ws, s);
    else
        peel(r, ix, sup_out, phi_out, pc, ws, s);
    ev.mark(4);
    int64_t *hs = ws.host(2);
    BT_HIP(hipMemcpyAsync(hs, ix.butterflies, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    if (stats) fill_stats(stats, r, ix, pc, u.m, hs[0], ev);
}

namespace {

// ---- batches: many graphs decomposed as one disjoint union --------------
// A butterfly never spans two connected components, so the supports and
// bitruss numbers of a disjoint union are those of its parts, and the
// union's vertex order restricted to one part is that part's own priority
// order (degrees are local; ids keep their order within each layer).  One
// pipeline run therefore serves every graph of a batch, and each peel
// round advances all of them together.

struct BatchEntry {
    const int64_t *row_ptr;
    const int32_t *col;
    int64_t *sup_out;
    int64_t *phi_out;
    int32_t nu, nl;
    int64_t m;
    int64_t nu_off, nl_off, m_off;
};

// Union CSR: rows and ids shifted by the graph's offsets.  Each graph's own
// bounds are checked here (the union check cannot see ids that stray into a
// neighbouring graph's range); values are only copied, never used to index.
__global__ void k_batch_union(const BatchEntry *tab, int32_t ng, int64_t *row_ptr_u,
                              int32_t *col_u, int32_t *flags) {
    for (int32_t gi = blockIdx.y; gi < ng; gi += gridDim.y) {
        const BatchEntry E = tab[gi];
        int32_t bad = 0;
        const int64_t span = E.m > (int64_t)E.nu + 1 ? E.m : (int64_t)E.nu + 1;
        for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < span;
             k += (int64_t)gridDim.x * blockDim.x) {
            if (k <= E.nu) {
                const int64_t v = E.row_ptr[k];
                if (v < 0 || v > E.m || (k == 0 && v != 0) || (k == E.nu && v != E.m)) bad = 1;
                if (k < E.nu && E.row_ptr[k + 1] < v) bad = 1;
                if (k < E.nu) row_ptr_u[E.nu_off + k] = E.m_off + v;
            }
            if (k < E.m) {
                const int32_t c = E.col[k];
                if (c < 0 || c >= E.nl) bad = 1;
                col_u[E.m_off + k] = (int32_t)(E.nl_off + c);
            }
        }
        if (bad) atomicOr(flags, 1);
    }
}

// Results back to each graph's outputs.  With perm (the union edge at each
// position of the reordered union), position p of graph g's range holds the
// result of union edge perm[p], which lies in the same range; an entry
// outside it raises *flags instead of being written.
__global__ void k_batch_scatter(const BatchEntry *tab, int32_t ng, const int64_t *sup_u,
                                const int64_t *phi_u, const uint32_t *perm, int32_t *flags) {
    for (int32_t gi = blockIdx.y; gi < ng; gi += gridDim.y) {
        const BatchEntry E = tab[gi];
        for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < E.m;
             k += (int64_t)gridDim.x * blockDim.x) {
            int64_t dst = k;
            if (perm) {
                dst = (int64_t)perm[E.m_off + k] - E.m_off;
                if (dst < 0 || dst >= E.m) {
                    atomicOr(flags, 2);
                    continue;
                }
            }
            if (E.sup_out) E.sup_out[dst] = sup_u[E.m_off + k];
            E.phi_out[dst] = phi_u[E.m_off + k];
        }
    }
}

// ---- locality order of a union's edges --------------------------------
// Support decrements are scattered atomics, and where they land decides how
// fast they go: with each graph's vertices renumbered inside the graph's
// block by decreasing degree and the edges sorted by (new upper, new lower),
// the edges that take most decrements (those of hub vertices) sit together,
// and the pool's batched peel runs 1.25x faster than on randomly numbered
// vertices (same decrements, same rounds).  Results do not depend on edge
// or vertex numbering; the map back is applied by k_batch_scatter.

__device__ __forceinline__ int32_t block_of(const int64_t *off, int32_t ng, int64_t x) {
    int32_t lo = 0, hi = ng - 1;  // largest g with off[g] <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Keys (graph, decreasing degree) of one layer's vertices; the stable sort
// keeps id order among equal degrees.
__global__ void k_reo_vertex_keys(const int64_t *row_ptr, const int32_t *deg, int32_t n,
                                  const int64_t *boff, int32_t ng, uint64_t *keys,
                                  uint32_t *vals) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t d = row_ptr ? (uint32_t)(row_ptr[x + 1] - row_ptr[x]) : (uint32_t)deg[x];
        keys[x] = ((uint64_t)block_of(boff, ng, x) << 32) | (uint64_t)(~d);
        vals[x] = (uint32_t)x;
    }
}

__global__ void k_reo_count(const int32_t *col, int64_t m, int32_t *deg) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&deg[col[e]], 1);
}

// newid[old] = position of old in the sorted order; with deg_out, the new
// vertex's degree as well.
__global__ void k_reo_newid(const uint32_t *order, int32_t n, const int64_t *row_ptr,
                            int32_t *newid, int32_t *deg_out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = order[i];
        newid[x] = (int32_t)i;
        if (deg_out) deg_out[i] = (int32_t)(row_ptr[x + 1] - row_ptr[x]);
    }
}

// One wave per row: key (new upper, new lower) and the union position of
// each edge.
__global__ void k_reo_edge_keys(const int64_t *row_ptr, const int32_t *col, int32_t nu,
                                const int32_t *new_u, const int32_t *new_l, uint64_t *keys,
                                uint32_t *vals) {
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t x = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; x < nu;
         x += nw) {
        const uint64_t hi = (uint64_t)(uint32_t)new_u[x] << 32;
        for (int64_t e = row_ptr[x] + lane_id(); e < row_ptr[x + 1]; e += kWave) {
            keys[e] = hi | (uint64_t)(uint32_t)new_l[col[e]];
            vals[e] = (uint32_t)e;
        }
    }
}

__global__ void k_reo_col(const uint64_t *keys, int64_t m, int32_t *col) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        col[i] = (int32_t)(uint32_t)keys[i];
}

// The union u rebuilt in the locality order; returns perm (union position
// of the edge now at each position) and points u at the new arrays.
const uint32_t *reorder_union(bt_csr &u, const int64_t *dvoff, int32_t ng, Workspace &ws,
                              hipStream_t s) {
    const int32_t nu = u.n_upper, nl = u.n_lower;
    const int64_t m = u.m;
    if (m == 0 || nu == 0 || nl == 0) return nullptr;
    const int cbits = bits_for((uint64_t)(ng > 1 ? ng - 1 : 1));
    const int64_t nv = std::max<int64_t>(nu, nl);
    uint64_t *vkeys = ws.get<uint64_t>("reo_vkeys", nv);
    uint32_t *vvals = ws.get<uint32_t>("reo_vvals", nv);
    int32_t *dl = ws.get<int32_t>("reo_dl", nl);
    int32_t *new_l = ws.get<int32_t>("reo_newl", nl);
    int32_t *new_u = ws.get<int32_t>("reo_newu", nu);
    int32_t *deg_new = ws.get<int32_t>("reo_degnew", nu);
    // Lower layer: degrees, order, new ids.
    zero_bytes(dl, sizeof(int32_t) * nl, s);
    k_reo_count<<<grid_for(m, 256, 16384), 256, 0, s>>>(u.col, m, dl);
    BT_CHECK_LAUNCH();
    k_reo_vertex_keys<<<grid_for(nl, 256, 8192), 256, 0, s>>>(nullptr, dl, nl, dvoff, ng, vkeys,
                                                             vvals);
    BT_CHECK_LAUNCH();
    radix_sort_u64_u32(vkeys, vvals, nl, 32 + cbits, ws, s);
    k_reo_newid<<<grid_for(nl, 256, 8192), 256, 0, s>>>(vvals, nl, nullptr, new_l, nullptr);
    BT_CHECK_LAUNCH();
    // Upper layer.
    k_reo_vertex_keys<<<grid_for(nu, 256, 8192), 256, 0, s>>>(u.row_ptr, nullptr, nu,
                                                             dvoff + (ng + 1), ng, vkeys, vvals);
    BT_CHECK_LAUNCH();
    radix_sort_u64_u32(vkeys, vvals, nu, 32 + cbits, ws, s);
    k_reo_newid<<<grid_for(nu, 256, 8192), 256, 0, s>>>(vvals, nu, u.row_ptr, new_u, deg_new);
    BT_CHECK_LAUNCH();
    // Edges sorted by (new upper, new lower).
    uint64_t *ekeys = ws.get<uint64_t>("reo_ekeys", m);
    uint32_t *perm = ws.get<uint32_t>("reo_perm", m);
    k_reo_edge_keys<<<grid_for((int64_t)nu * kWave, 256, 16384), 256, 0, s>>>(
        u.row_ptr, u.col, nu, new_u, new_l, ekeys, perm);
    BT_CHECK_LAUNCH();
    radix_sort_u64_u32(ekeys, perm, m, 32 + bits_for((uint64_t)(nu - 1 > 0 ? nu - 1 : 1)), ws,
                       s);
    int64_t *row_ptr = ws.get<int64_t>("reo_rowptr", (int64_t)nu + 1);
    int32_t *col = ws.get<int32_t>("reo_col", m);
    scan_exclusive_i32_to_i64(deg_new, row_ptr, nu, ws, s);
    k_reo_col<<<grid_for(m, 256, 16384), 256, 0, s>>>(ekeys, m, col);
    BT_CHECK_LAUNCH();
    u.row_ptr = row_ptr;
    u.col = col;
    return perm;
}

void add_stats(bt_stats &t, const bt_stats &s) {
    t.butterflies += s.butterflies;
    t.wedges_po += s.wedges_po;
    t.blooms += s.blooms;
    t.bloom_wedges += s.bloom_wedges;
    t.index_bytes = std::max(t.index_bytes, s.index_bytes);
    t.levels += s.levels;
    t.rounds += s.rounds;
    t.max_phi = std::max(t.max_phi, s.max_phi);
    t.support_updates += s.support_updates;
    t.bloom_visits += s.bloom_visits;
    t.ms_prepare += s.ms_prepare;
    t.ms_count += s.ms_count;
    t.ms_link += s.ms_link;
    t.ms_peel += s.ms_peel;
    t.ms_peel_kernel += s.ms_peel_kernel;
    t.peel_launches += s.peel_launches;
    t.passes = std::max(t.passes, s.passes);
    t.support_updates_unbatched += s.support_updates_unbatched;
    t.wedge_visits += s.wedge_visits;
    t.peel_yields += s.peel_yields;
}

// Graphs [a, b) as one union; splits the range if the union is too large.
void batch_range(const bt_csr *gs, int32_t a, int32_t b, int64_t *const *sup_out,
                 int64_t *const *phi_out, bt_stats *stats, Workspace &ws, hipStream_t s,
                 const SizedHook *on_sized = nullptr) {
    std::vector<BatchEntry> tab(b - a);
    int64_t nu = 0, nl = 0, m = 0, max_span = 1;
    for (int32_t i = a; i < b; ++i) {
        BatchEntry &E = tab[i - a];
        E.row_ptr = gs[i].row_ptr;
        E.col = gs[i].col;
        E.sup_out = sup_out ? sup_out[i] : nullptr;
        E.phi_out = phi_out[i];
        E.nu = gs[i].n_upper;
        E.nl = gs[i].n_lower;
        E.m = gs[i].m;
        E.nu_off = nu;
        E.nl_off = nl;
        E.m_off = m;
        nu += E.nu;
        nl += E.nl;
        m += E.m;
        max_span = std::max<int64_t>(max_span, std::max<int64_t>(E.m, (int64_t)E.nu + 1));
    }
    const bool splittable = b - a > 1;
    if (splittable && (nu + nl >= INT32_MAX || m >= INT32_MAX)) {
        const int32_t mid = a + (b - a) / 2;
        batch_range(gs, a, mid, sup_out, phi_out, stats, ws, s);
        batch_range(gs, mid, b, sup_out, phi_out, stats, ws, s);
        return;
    }
    BatchEntry *dtab = ws.get<BatchEntry>("batch_tab", b - a);
    int64_t *row_ptr_u = ws.get<int64_t>("batch_rowptr", nu + 1);
    int32_t *col_u = ws.get<int32_t>("batch_col", m);
    int32_t *flags = ws.get<int32_t>("batch_flags", 1);
    int64_t *sup_u = ws.get<int64_t>("batch_sup", m);
    int64_t *phi_u = ws.get<int64_t>("batch_phi", m);
    BT_HIP(hipMemcpyAsync(dtab, tab.data(), sizeof(BatchEntry) * tab.size(),
                          hipMemcpyHostToDevice, s));
    zero_bytes(flags, sizeof(int32_t), s);
    fill_i64(row_ptr_u + nu, m, 1, s);
    const dim3 grid((unsigned)std::min<int64_t>(ceil_div(max_span, 256), 64),
                    (unsigned)std::min<int32_t>(b - a, 65535));
    k_batch_union<<<grid, 256, 0, s>>>(dtab, b - a, row_ptr_u, col_u, flags);
    BT_CHECK_LAUNCH();
    int32_t hf = 0;
    BT_HIP(hipMemcpyAsync(&hf, flags, sizeof hf, hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    if (hf) throw Error{BT_EINVAL, "a graph of the batch is malformed"};
    bt_csr u{(int32_t)nu, (int32_t)nl, m, row_ptr_u, col_u};
    std::vector<int64_t> off(b - a + 1);
    for (int32_t i = a; i < b; ++i) off[i - a] = tab[i - a].m_off;
    off[b - a] = m;
    // Vertex ranges of the graphs, lower then upper offsets.
    std::vector<int64_t> voff(2 * (size_t)(b - a + 1));
    for (int32_t i = a; i < b; ++i) {
        voff[i - a] = tab[i - a].nl_off;
        voff[(b - a + 1) + (i - a)] = tab[i - a].nu_off;
    }
    voff[b - a] = nl;
    voff[2 * (b - a) + 1] = nu;
    int64_t *dvoff = ws.get<int64_t>("batch_voff", (int64_t)voff.size());
    BT_HIP(hipMemcpyAsync(dvoff, voff.data(), sizeof(int64_t) * voff.size(),
                          hipMemcpyHostToDevice, s));
    Components comps;
    comps.n = b - a;
    comps.l_off = dvoff;
    comps.u_off = dvoff + (b - a + 1);
    // BT_BATCH_REORDER=0 keeps the union in the callers' numbering.
    const char *ro = std::getenv("BT_BATCH_REORDER");
    const uint32_t *perm =
        ro && std::atoi(ro) == 0 ? nullptr : reorder_union(u, dvoff, b - a, ws, s);
    bt_stats st;
    try {
        decompose_union_impl(u, off, comps, sup_u, phi_u, stats ? &st : nullptr, ws, s,
                             on_sized);
    } catch (const Error &e) {
        if (e.status != BT_EOVERFLOW || !splittable) throw;
        const int32_t mid = a + (b - a) / 2;
        batch_range(gs, a, mid, sup_out, phi_out, stats, ws, s);
        batch_range(gs, mid, b, sup_out, phi_out, stats, ws, s);
        return;
    }
    k_batch_scatter<<<grid, 256, 0, s>>>(dtab, b - a, sup_u, phi_u, perm, flags);
    BT_CHECK_LAUNCH();
    BT_HIP(hipMemcpyAsync(&hf, flags, sizeof hf, hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    if (hf) throw Error{BT_EDEVICE, "batch results could not be mapped back to their graphs"};
    if (stats) add_stats(*stats, st);
}

// Batches are cut at about kBatchEdges edges so that each union stays well
// inside the index limits; an oversized union is split in halves.
// BT_BATCH_EDGES_LOG2 (16..30) sets another cut, for measurements.
constexpr int64_t kBatchEdges = int64_t(1) << 26;
int64_t batch_edges() {
    const char *v = std::getenv("BT_BATCH_EDGES_LOG2");
    const int l = v ? std::atoi(v) : 0;
    return l >= 16 && l <= 30 ? int64_t(1) << l : kBatchEdges;
}

}  // namespace

void decompose_batch_impl(const bt_csr *gs, int32_t n, int64_t *const *sup_out,
                          int64_t *const *phi_out, bt_stats *stats, Workspace &ws,
                          hipStream_t s, const SizedHook *on_sized) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    // Unions are cut from the graphs in decreasing edge count: a union peels
    // for as many rounds as its slowest graph needs, so the large graphs,
    // which need the most rounds, share a union instead of each stretching
    // one (whole 4,096-graph pool: 62k rounds instead of 103k, 7% faster).
    std::vector<int32_t> ord((size_t)n);
    for (int32_t i = 0; i < n; ++i) ord[(size_t)i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int32_t x, int32_t y) { return gs[x].m > gs[y].m; });
    std::vector<bt_csr> g2((size_t)n);
    std::vector<int64_t *> s2((size_t)n), p2((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t o = ord[(size_t)i];
        g2[(size_t)i] = gs[o];
        s2[(size_t)i] = sup_out ? sup_out[o] : nullptr;
        p2[(size_t)i] = phi_out[o];
    }
    const int64_t cut = batch_edges();
    int32_t a = 0;
    while (a < n) {
        int32_t b = a;
        int64_t m = 0;
        while (b < n && (b == a || m + g2[(size_t)b].m <= cut)) m += g2[(size_t)b++].m;
        // The size report is exact only when one union holds the whole batch.
        batch_range(g2.data(), a, b, sup_out ? s2.data() : nullptr, p2.data(), stats, ws, s,
                    a == 0 && b == n ? on_sized : nullptr);
        a = b;
    }
}

}  // namespace bt

namespace {

// Launch parameters across the C ABI.
bt::TuneParams from_c(const bt_tune_params &p) {
    bt::TuneParams t;
    t.hash_max_work = p.hash_max_work;
    t.dense_chunk = p.dense_chunk;
    t.wedge_wg_per_cu = p.wedge_wg_per_cu;
    t.peel_blocks = p.peel_blocks;
    t.active_min = p.active_min;
    return t;
}
bt_tune_params to_c(const bt::TuneParams &t) {
    return bt_tune_params{t.hash_max_work, t.dense_chunk, t.wedge_wg_per_cu, t.peel_blocks,
                          t.active_min};
}
}  // namespace

using namespace bt;

struct bt_index {
    IndexArrays ix;
    int64_t m = 0;
    int64_t butterflies = 0;
    int64_t wedges_po = 0;
    std::vector<void *> owned;
    ~bt_index() {
        for (void *p : owned) device_free(p);
    }
};

extern "C" {

const char *bt_version(void) { return "bt-mi355x 0.1"; }

void bt_release_workspace(void) {
    std::lock_guard<std::mutex> lk(lib().mu);
    lib().ws.release();
}

bt_status bt_set_allocator(bt_alloc_fn alloc, bt_free_fn free, void *ctx) {
    return guard([&] { set_allocator(alloc, free, ctx); });
}

bt_status bt_support(const bt_csr *g, int64_t *sup_out, int64_t *butterflies_out,
                     hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (g->m > 0 && !sup_out) throw Error{BT_EINVAL, "sup_out is NULL"};
        std::lock_guard<std::mutex> lk(lib().mu);
        Workspace &ws = lib().ws;
        RankCSR r;
        prepare(*g, r, ws, stream);
        TaskLists t;
        make_tasks(r, t, ws, stream);
        uint64_t *supl = ws.get<uint64_t>("sup_supl", g->m + 1);
        int64_t *bf = ws.get<int64_t>("sup_bf", 2);
        zero_bytes(supl, sizeof(uint64_t) * (g->m + 1), stream);
        zero_bytes(bf, sizeof(int64_t) * 2, stream);
        count_support(r, t, supl, bf, stream);
        check_butterfly_total(supl, g->m, bf, ws, stream);
        supl_to_sup(supl, sup_out, g->m, stream);
        int64_t *hs = ws.host(2);
        BT_HIP(hipMemcpyAsync(hs, bf, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        BT_HIP(hipStreamSynchronize(stream));
        if (butterflies_out) *butterflies_out = hs[0];
    });
}

bt_status bt_index_build(const bt_csr *g, bt_index **out, hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (!out) throw Error{BT_EINVAL, "out is NULL"};
        *out = nullptr;
        std::lock_guard<std::mutex> lk(lib().mu);
        Workspace &ws = lib().ws;
        bt_index *h = new bt_index();
        try {
            RankCSR r;
            build_all(*g, r, h->ix, true, &h->owned, ws, stream, nullptr);
            int64_t *hs = ws.host(2);
            BT_HIP(hipMemcpyAsync(hs, h->ix.butterflies, sizeof(int64_t), hipMemcpyDeviceToHost,
                                  stream));
            BT_HIP(hipStreamSynchronize(stream));
            h->butterflies = hs[0];
            h->m = g->m;
            h->wedges_po = r.wedges_po;
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

bt_status bt_index_info_get(const bt_index *idx, bt_index_info *info) {
    return guard([&] {
        if (!idx || !info) throw Error{BT_EINVAL, "NULL argument"};
        info->m = idx->m;
        info->blooms = idx->ix.n_b;
        info->bloom_wedges = idx->ix.n_w;
        info->links = 2 * idx->ix.n_w;
        info->butterflies = idx->butterflies;
        info->wedges_po = idx->wedges_po;
        info->bytes = index_bytes(idx->ix, idx->m);
    });
}

bt_status bt_index_export(const bt_index *idx, int64_t *bloom_woff, int32_t *wedge_ea,
                          int32_t *wedge_eb, int64_t *edge_link_off, int64_t *edge_link,
                          int64_t *sup) {
    return guard([&] {
        if (!idx) throw Error{BT_EINVAL, "index is NULL"};
        const IndexArrays &ix = idx->ix;
        if (bloom_woff) {
            std::vector<uint32_t> t(ix.n_b + 1);
            BT_HIP(hipMemcpy(t.data(), ix.bwoff, sizeof(uint32_t) * t.size(),
                             hipMemcpyDeviceToHost));
            for (size_t i = 0; i < t.size(); ++i) bloom_woff[i] = t[i];
        }
        if (wedge_ea && ix.n_w)
            BT_HIP(hipMemcpy(wedge_ea, ix.wea, sizeof(int32_t) * ix.n_w, hipMemcpyDeviceToHost));
        if (wedge_eb && ix.n_w)
            BT_HIP(hipMemcpy(wedge_eb, ix.web, sizeof(int32_t) * ix.n_w, hipMemcpyDeviceToHost));
        if (edge_link_off)
            BT_HIP(hipMemcpy(edge_link_off, ix.link_off, sizeof(int64_t) * (idx->m + 1),
                             hipMemcpyDeviceToHost));
        if (edge_link && ix.n_w) {
            std::vector<uint3> t(2 * ix.n_w);
            BT_HIP(hipMemcpy(t.data(), ix.link, sizeof(uint3) * t.size(),
                             hipMemcpyDeviceToHost));
            for (size_t i = 0; i < t.size(); ++i) edge_link[i] = t[i].x;
        }
        if (sup && idx->m) {
            std::vector<uint64_t> t(idx->m);
            BT_HIP(hipMemcpy(t.data(), ix.supl, sizeof(uint64_t) * t.size(),
                             hipMemcpyDeviceToHost));
            for (size_t i = 0; i < t.size(); ++i) sup[i] = (int64_t)(t[i] & 0xffffffffu);
        }
    });
}

void bt_index_free(bt_index *idx) { delete idx; }

bt_status bt_decompose(const bt_csr *g, int64_t *sup_out, int64_t *phi_out, bt_stats *stats,
                       hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (g->m > 0 && !phi_out) throw Error{BT_EINVAL, "phi_out is NULL"};
        std::lock_guard<std::mutex> lk(lib().mu);
        decompose_impl(*g, sup_out, phi_out, stats, lib().ws, stream);
    });
}

bt_status bt_decompose_trace(const bt_csr *g, int64_t *phi_out, int32_t max_rounds,
                             int32_t *n_rounds, int32_t *round_level, int8_t *removed,
                             int64_t *sup, int64_t max_wedges, int64_t *n_wedges,
                             int32_t *wedge_ea, int32_t *wedge_eb, int32_t *wedge_k,
                             hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (g->m > 0 && !phi_out) throw Error{BT_EINVAL, "phi_out is NULL"};
        if (g->m > kTraceMaxEdges)
            throw Error{BT_EOVERFLOW, "bt_decompose_trace takes at most 65536 edges"};
        if (max_rounds < 0 || max_wedges < 0 || !n_rounds || !n_wedges ||
            (max_rounds > 0 && (!round_level || !removed || !sup)) ||
            (max_wedges > 0 && (!wedge_ea || !wedge_eb)) ||
            (max_rounds > 0 && max_wedges > 0 && !wedge_k))
            throw Error{BT_EINVAL, "invalid trace buffers"};
        std::lock_guard<std::mutex> lk(lib().mu);
        Workspace &ws = lib().ws;
        const int64_t m = g->m;
        RankCSR r;
        IndexArrays ix;
        build_all(*g, r, ix, false, nullptr, ws, stream, nullptr);
        if (ix.n_w > max_wedges) throw Error{BT_EOVERFLOW, "more wedges than max_wedges"};
        std::vector<PeelTraceRound> rounds;
        const PeelTraceFn fn = [&](const PeelTraceRound &t) {
            if ((int64_t)rounds.size() >= max_rounds)
                throw Error{BT_EOVERFLOW, "more rounds than max_rounds"};
            rounds.push_back(t);
        };
        PeelOptions o;
        o.trace = &fn;
        PeelCounters pc;
        if (m > 0) peel(r, ix, nullptr, phi_out, pc, ws, stream, &o);
        std::vector<int32_t> wbl((size_t)ix.n_w);
        if (ix.n_w) {
            BT_HIP(hipMemcpy(wedge_ea, ix.wea, sizeof(int32_t) * ix.n_w, hipMemcpyDeviceToHost));
            BT_HIP(hipMemcpy(wedge_eb, ix.web, sizeof(int32_t) * ix.n_w, hipMemcpyDeviceToHost));
            BT_HIP(hipMemcpy(wbl.data(), ix.wbl, sizeof(int32_t) * ix.n_w, hipMemcpyDeviceToHost));
        }
        for (size_t k = 0; k < rounds.size(); ++k) {
            const PeelTraceRound &t = rounds[k];
            round_level[k] = t.level;
            int8_t *rm = removed + k * (size_t)m;
            std::memset(rm, 0, (size_t)m);
            for (int32_t e : t.removed) rm[e] = 1;
            for (int64_t e = 0; e < m; ++e) sup[k * (size_t)m + e] = t.sup[(size_t)e];
            for (int64_t w = 0; w < ix.n_w; ++w)
                wedge_k[k * (size_t)max_wedges + w] = t.bloom_k[(size_t)wbl[(size_t)w]];
        }
        *n_rounds = (int32_t)rounds.size();
        *n_wedges = ix.n_w;
    });
}

bt_status bt_decompose_variant(const bt_csr *g, int32_t variant, int64_t *sup_out,
                               int64_t *phi_out, bt_stats *stats, hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (g->m > 0 && !phi_out) throw Error{BT_EINVAL, "phi_out is NULL"};
        if (variant != BT_PEEL_BATCH_BLOOM && variant != BT_PEEL_BATCH_EDGE &&
            variant != BT_PEEL_AUTO)
            throw Error{BT_EINVAL, "unknown peel variant"};
        std::lock_guard<std::mutex> lk(lib().mu);
        decompose_impl(*g, sup_out, phi_out, stats, lib().ws, stream,
                       variant == BT_PEEL_BATCH_EDGE, variant == BT_PEEL_AUTO);
    });
}


bt_status bt_tune(const bt_csr *gs, int32_t n_graphs, uint32_t what, bt_tune_params *out,
                  hipStream_t stream) {
    return guard([&] {
        if (n_graphs < 1 || !gs) throw Error{BT_EINVAL, "bt_tune needs at least one graph"};
        if (what & ~(uint32_t)(BT_TUNE_INDEX | BT_TUNE_PEEL))
            throw Error{BT_EINVAL, "unknown bits in the tuning mask"};
        for (int32_t i = 0; i < n_graphs; ++i) check_graph(&gs[i]);
        std::lock_guard<std::mutex> lk(lib().mu);
        const TuneParams t = autotune(gs, n_graphs, what, lib().ws, stream);
        if (out) *out = to_c(t);
    });
}

bt_status bt_tune_get(int32_t batch, int64_t m, bt_tune_params *out) {
    return guard([&] {
        if (!out || m < 0) throw Error{BT_EINVAL, "bt_tune_get: bad argument"};
        *out = to_c(tune_params(batch != 0, m));
    });
}

bt_status bt_tune_set(int32_t batch, int64_t m, const bt_tune_params *p) {
    return guard([&] {
        if (!p || m < 0) throw Error{BT_EINVAL, "bt_tune_set: bad argument"};
        tune_store(batch != 0, m, from_c(*p));
    });
}

bt_status bt_tune_reset(void) {
    return guard([&] { tune_clear(); });
}

bt_status bt_tune_save(const char *path) {
    return guard([&] {
        if (!path) throw Error{BT_EINVAL, "path is NULL"};
        tune_save(path);
    });
}

bt_status bt_tune_load(const char *path) {
    return guard([&] {
        if (!path) throw Error{BT_EINVAL, "path is NULL"};
        tune_load(path);
    });
}

bt_status bt_decompose_pc(const bt_csr *g, double tau, int64_t *sup_out, int64_t *phi_out,
                          bt_stats *stats, hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (g->m > 0 && !phi_out) throw Error{BT_EINVAL, "phi_out is NULL"};
        if (!(tau > 0.0 && tau <= 1.0)) throw Error{BT_EINVAL, "tau must lie in (0, 1]"};
        std::lock_guard<std::mutex> lk(lib().mu);
        decompose_pc_impl(*g, tau, sup_out, phi_out, stats, lib().ws, stream);
    });
}

bt_status bt_bitruss_components(const bt_csr *g, const int64_t *phi, int64_t k,
                                int32_t *comp_out, int64_t *n_components_out,
                                hipStream_t stream) {
    return guard([&] {
        check_graph(g);
        if (g->m > 0 && (!phi || !comp_out)) throw Error{BT_EINVAL, "phi or comp_out is NULL"};
        std::lock_guard<std::mutex> lk(lib().mu);
        validate_graph(*g, lib().ws, stream);
        const int64_t c = bitruss_components(*g, phi, k, comp_out, lib().ws, stream);
        if (n_components_out) *n_components_out = c;
    });
}

bt_status bt_decompose_batch(const bt_csr *gs, int32_t n_graphs, int64_t *const *sup_out,
                             int64_t *const *phi_out, bt_stats *stats, hipStream_t stream) {
    return guard([&] {
        if (n_graphs < 0 || (n_graphs > 0 && (!gs || !phi_out)))
            throw Error{BT_EINVAL, "invalid batch arguments"};
        for (int32_t i = 0; i < n_graphs; ++i) {
            check_graph(&gs[i]);
            if (gs[i].m > 0 && !phi_out[i]) throw Error{BT_EINVAL, "phi_out[i] is NULL"};
        }
        std::lock_guard<std::mutex> lk(lib().mu);
        decompose_batch_impl(gs, n_graphs, sup_out, phi_out, stats, lib().ws, stream);
    });
}

}  // extern "C"
