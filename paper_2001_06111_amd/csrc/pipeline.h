// pipeline.h - stages of the hot path and the device views they share.
#pragma once

#include <functional>
#include <vector>

#include "common.h"

namespace bt {

// Rank-space adjacency (built by prepare()).
//
// Vertices are renumbered so that each layer occupies a contiguous range in
// increasing priority (Definition 6: degree, ties by id, upper ids above
// lower ids): lower layer [0, n_lower), upper layer [n_lower, n).  Row x
// lists x's neighbours (new ids) in increasing priority with the edge id of
// each entry.  low[x] counts the neighbours of lower priority than x, so
// they form the row's prefix.  For a prefix entry (x -> y), rev is the
// position of x in row y, which is the number of y's neighbours of lower
// priority than x: the wedges (x, y, z) with p(y), p(z) < p(x) are
// exactly z = adj[off[y] + t] for t < rev.
// Launch parameters of the sweeps and the peel.  None of them changes a
// result; the autotuner (tune.hip) picks them per kind of call (one graph,
// or a batch) and per size class, and prepare() copies the entry for the
// graph into its RankCSR.
struct TuneParams {
    int32_t hash_max_work = 2048;  // start vertices with at most this many wedges: one hash task
    int32_t dense_chunk = 6144;    // counter range of a dense task (hub start vertices)
    int32_t wedge_wg_per_cu = 2;   // wedge-sweep workgroups per CU
    int32_t peel_blocks = 0;       // persistent peel workgroups (0: three per four CUs)
    int32_t active_min = 16384;    // smallest active set the peel rebuilds
};
constexpr int32_t kHashMaxWorkLimit = 2048;  // hash tables hold at most 4096 slots
constexpr int32_t kDenseChunkLimit = 6144;   // dense counters per workgroup in LDS
bool tune_valid(const TuneParams &p);
// Workgroups of a cooperative peel: the parameter, or three per four CUs
// (fewer arrivals per grid barrier; a round rarely fills the chip), capped
// at what can be resident.
int peel_grid(const TuneParams &p, int cus, int resident);
TuneParams tune_params(bool batch, int64_t m);  // the entry for a call of this kind and size
void tune_store(bool batch, int64_t m, const TuneParams &p);  // throws BT_EINVAL if invalid
void tune_clear();
void tune_save(const char *path);
void tune_load(const char *path);

// The graphs of a disjoint union: graph c owns lower ids [l_off[c],
// l_off[c+1]) and upper ids n_lower + [u_off[c], u_off[c+1]) (device arrays
// of n + 1 entries).
struct Components {
    int32_t n = 0;
    const int64_t *l_off = nullptr;
    const int64_t *u_off = nullptr;
};

struct RankCSR {
    TuneParams tp;
    int32_t n_lower = 0, n = 0;
    int64_t m = 0;
    int64_t *off = nullptr;   // [n + 1]
    int32_t *adj = nullptr;   // [2m] neighbour new id
    int32_t *eid = nullptr;   // [2m] edge id
    int32_t *rev = nullptr;   // [2m] z-prefix length for prefix entries, else 0
    int32_t *low = nullptr;   // [n]
    int64_t *wpre = nullptr;  // [2m + 1] exclusive prefix of rev: wedge work
    int64_t wedges_po = 0;    // priority-obeyed wedges (host copy)
    int32_t max_deg = 0;
    // Unions only: the first rank of x's graph in x's layer (end vertices of
    // x's wedges lie in [zbase[x], x)); null for a single graph.
    int32_t *zbase = nullptr;
};

// Work items of the wedge sweeps.
struct WedgeTask {
    int32_t x;     // start vertex (new id)
    int32_t zlo;   // dense mode: counter range [zlo, zhi); hash mode: unused
    int32_t zhi;
    int32_t cap;   // hash mode: table slots (power of two); dense: zhi - zlo
};

struct TaskLists {
    WedgeTask *hash = nullptr;
    WedgeTask *dense = nullptr;
    int64_t n_hash = 0, n_dense = 0;
};

// BE-Index arrays (device).  Blooms own contiguous wedge ranges
// [bwoff[b], bwoff[b+1]); a wedge is a twin pair of edges.
struct IndexArrays {
    int64_t n_b = 0, n_w = 0;   // host copies after build
    int64_t cap_b = 0, cap_w = 0;
    uint32_t *bwoff = nullptr;  // [cap_b + 1]
    int32_t *bk = nullptr;      // [cap_b] bloom number (live wedges)
    int32_t *wea = nullptr;     // [cap_w] edge at the highest-priority vertex
    int32_t *web = nullptr;     // [cap_w] twin edge
    int32_t *wbl = nullptr;     // [cap_w] bloom of the wedge
    uint64_t *supl = nullptr;   // [m] (links << 32) | support while building
    int64_t *link_off = nullptr;  // [m + 1]
    uint3 *link = nullptr;        // [2 cap_w] {wedge, bloom of the wedge, twin edge}
    uint64_t *cursor = nullptr;   // device (blooms << 32) | wedges allocated
    int64_t *butterflies = nullptr;  // device scalar
};

// Checks the CSR on the device (BT_EINVAL with the reason if malformed).
void validate_graph(const bt_csr &g, Workspace &ws, hipStream_t s);

// Connected components of the k-bitruss (edges with phi >= k): comp[e] is
// the component of e numbered by smallest edge id, or -1.  Returns their
// number.  The graph must be valid.
int64_t bitruss_components(const bt_csr &g, const int64_t *phi, int64_t k, int32_t *comp,
                           Workspace &ws, hipStream_t s);

// Validates the CSR and builds the rank-space adjacency in `ws`.
// Throws Error{BT_EINVAL} for malformed input.
// `comps` (nullable): g is a disjoint union of these graphs; the rank order
// then puts each graph's vertices together within a layer (the order
// restricted to a graph is unchanged).
void prepare(const bt_csr &g, RankCSR &r, Workspace &ws, hipStream_t s,
             const Components *comps = nullptr);

// Splits start vertices into wedge tasks (sync point: reads counts).
void make_tasks(const RankCSR &r, TaskLists &t, Workspace &ws, hipStream_t s);

// Support only: sup_out[e] (int64, may be null) and the butterfly total
// (device scalar *bf, must be zeroed by the caller).
void count_support(const RankCSR &r, const TaskLists &t, uint64_t *supl, int64_t *bf,
                   hipStream_t s);

// Counting plus index emission into `ix` (arrays sized by the caller from
// r.wedges_po).  Fills supl and cursor; then builds the link lists.
void build_index(const RankCSR &r, const TaskLists &t, IndexArrays &ix, Workspace &ws,
                 hipStream_t s);

// Peel through the index.  sup_out (int64, nullable) receives the initial
// supports, phi_out (int64) the bitruss numbers.
struct PeelCounters {
    int64_t levels = 0, rounds = 0, max_phi = 0, updates = 0, bloom_visits = 0;
    int64_t updates_unbatched = 0;  // the same peel without batch bloom processing
    int64_t touched = 0;            // live wedges visited in phase B (L_touch)
    double kernel_ms = 0;  // HIP-event time of the peel kernel launches
    int64_t launches = 0;
    int64_t yields = 0;  // launches that ended early to give the device to a lighter peel
};
// One round of a traced peel (only rounds that remove edges): its level,
// the edges it removed, and every support and bloom number after it.
struct PeelTraceRound {
    int32_t level = 0;
    std::vector<int32_t> removed;
    std::vector<int32_t> sup;
    std::vector<int32_t> bloom_k;
};
using PeelTraceFn = std::function<void(const PeelTraceRound &)>;
// Progressive mode (Section V-C): `fixed` (per edge, nullable) marks edges
// whose bitruss numbers an earlier pass fixed; the index must carry their
// marks (mark_fixed).  The first level is at least `min_level`.
// `trace` (nullable): run the rounds one at a time from the host and report
// each (small graphs; for inspection and tests).
// The weight of this thread's later turns on the device for cooperative
// peels (w < 0: each peel's edge count).  A waiting peel that weighs under
// 1/8 of the running one makes it yield between two rounds.  The serving
// engine weighs a batch by its size class, so a batch of a smaller class
// always takes the device from a running one of a larger class.
void set_turn_weight(int64_t w);

struct PeelOptions {
    const int32_t *fixed = nullptr;
    int32_t min_level = 0;
    bool unit_updates = false;  // ablation: no batch bloom processing
    const PeelTraceFn *trace = nullptr;
};
void peel(const RankCSR &r, IndexArrays &ix, int64_t *sup_out, int64_t *phi_out,
          PeelCounters &pc, Workspace &ws, hipStream_t s, const PeelOptions *opt = nullptr);

// Peel of a disjoint union of graphs (edge ranges [off[g], off[g+1])) in
// which every graph advances at its own level (one cooperative kernel).
void peel_multi(const RankCSR &r, IndexArrays &ix, int64_t *sup_out, int64_t *phi_out,
                const std::vector<int64_t> &off, PeelCounters &pc, Workspace &ws, hipStream_t s);

// Sets the fixed-edge mark in wedge records and link twins (progressive mode).
void mark_fixed(IndexArrays &ix, const int32_t *fixed, hipStream_t s);

// Whole decompositions (api.hip): one graph, or many as disjoint unions.
// `unit_updates`: the peel without batch bloom processing (ablation).
// `auto_pc`: after the index build, switch to BiT-PC when the graph has at
// least kAutoPcButterfliesPerEdge butterflies per edge.
void decompose_impl(const bt_csr &g, int64_t *sup_out, int64_t *phi_out, bt_stats *stats,
                    Workspace &ws, hipStream_t stream, bool unit_updates = false,
                    bool auto_pc = false);
constexpr int64_t kAutoPcButterfliesPerEdge = 16384;
constexpr double kAutoPcTau = 0.05;
// Measures candidate launch parameters on these graphs (one graph, or a
// batch) and stores the best for their kind and size class (tune.hip).
TuneParams autotune(const bt_csr *gs, int32_t n, uint32_t what, Workspace &ws, hipStream_t s);
// Device time of the index build alone (priority order, sweeps, links).
float index_build_ms(const bt_csr &g, Workspace &ws, hipStream_t stream);
// Called when a batch that forms a single union has its index built: the
// bytes the workspace holds now, and at most how many the peel still adds.
using SizedHook = std::function<void(int64_t held, int64_t peel_bytes)>;
void decompose_batch_impl(const bt_csr *gs, int32_t n, int64_t *const *sup_out,
                          int64_t *const *phi_out, bt_stats *stats, Workspace &ws,
                          hipStream_t s, const SizedHook *on_sized = nullptr);
// Device bytes of peel state for a graph (or union of `graphs` graphs) with
// m edges and an index of n_b blooms and n_w wedges, for the per-graph-level
// peel (multi) or the shared-level one; an upper bound, workspace growth
// slack included.
int64_t peel_state_bytes(int64_t m, int64_t n_b, int64_t n_w, int64_t graphs, bool multi);
// BiT-PC steps (pc.hip).  A pass's subgraph G_{>=eps}: the edges of g with
// support >= eps in g, in g's order; orig maps them back, fixed marks those
// whose bitruss numbers earlier passes fixed, open counts the others.
struct PcSubgraph {
    bt_csr g{};
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr, *orig = nullptr, *fixed = nullptr;
    int64_t open = 0;
};
// Supports (low halves of supl) into sup0; returns k_max.
int32_t pc_kmax(const uint64_t *supl, int64_t m, int32_t *sup0, Workspace &ws, hipStream_t s);
int64_t pc_subgraph(const bt_csr &g, const int32_t *sup0, int32_t eps, const int32_t *phi_glob,
                    PcSubgraph &sg, Workspace &ws, hipStream_t s);
void pc_collect(const int64_t *phi_sub, const PcSubgraph &sg, int32_t eps, int32_t *phi_glob,
                hipStream_t s);
void pc_widen(const int32_t *phi_glob, int64_t m, int64_t *phi_out, hipStream_t s);
// BiT-PC (Algorithms 6-7): progressive compression with step ceil(k_max tau).
void decompose_pc_impl(const bt_csr &g, double tau, int64_t *sup_out, int64_t *phi_out,
                       bt_stats *stats, Workspace &ws, hipStream_t s);
void check_graph(const bt_csr *g);

// Device-memory estimate of decomposing g (validates g; BT_EINVAL if
// malformed): index and peel state bounded through the wedge bound
// sum over edges of min(d(u), d(v)) (Lemma 6), plus per-edge arrays.
int64_t footprint_bytes(const bt_csr &g, Workspace &ws, hipStream_t s);

// supl low halves to int64 supports.
void supl_to_sup(const uint64_t *supl, int64_t *sup, int64_t m, hipStream_t s);
// The butterfly total two ways (Lemma 1: every butterfly has four edges;
// Lemma 8: a k-bloom holds C(k, 2)): the supports must sum to four times the
// blooms' total, else BT_EDEVICE.
void check_butterfly_total(const uint64_t *supl, int64_t m, const int64_t *butterflies,
                           Workspace &ws, hipStream_t s);

}  // namespace bt
