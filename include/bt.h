/*
 * bt.h - C ABI of the MI355X bitruss library (libbt.so).
 *
 * Bitruss decomposition of a bipartite graph with the BE-Index of
 * Wang, Lin, Qin, Zhang, Zhang, "Efficient Bitruss Decomposition for
 * Large-scale Bipartite Graphs" (ICDE 2020):
 *   - butterfly support of every edge (Section II, Definition 2 and the
 *     counting step of Algorithm 4),
 *   - the BE-Index: maximal priority-obeyed blooms, their edge links and
 *     twin edges (Section IV, Definitions 6-8, Algorithm 3),
 *   - bitruss numbers (Section II, Definitions 4-5) by peeling through
 *     blooms with batch edge and batch bloom processing (Section V-B,
 *     Algorithm 5).
 *
 * Conventions shared by every entry point
 *   Graph: upper-major CSR, all pointers DEVICE pointers.
 *     row_ptr int64[n_upper+1]: row_ptr[0] = 0, non-decreasing,
 *                               row_ptr[n_upper] = m.
 *     col     int32[m]: lower ids in [0, n_lower), strictly increasing
 *                       within a row (the edge set is a set: Section II).
 *   Edge identity: edge e is CSR position e; every per-edge output is
 *     indexed by it.  Vertex priority (Definition 6) orders by degree, ties
 *     by id, with every upper id above every lower id (Section II): lower
 *     vertex j has id j, upper vertex i has id n_lower + i.
 *   Limits: n_upper + n_lower < 2^31 and m < 2^31 (else BT_EOVERFLOW).
 *     A support is then at most m - 1 (Lemma 8's argument), so it fits
 *     32 bits internally; outputs are int64.  The number of
 *     priority-obeyed wedges must be below 2^32 (else BT_EOVERFLOW).
 *   Streams: every call enqueues its work on `stream` (0 = the null
 *     stream) and returns after the results are complete on that stream;
 *     host-side outputs are written before return.
 *   Ownership: the caller owns the graph and every output buffer.  The
 *     library owns its scratch memory (a device workspace cached between
 *     calls, released by bt_release_workspace) and the bt_index handles
 *     until bt_index_free.
 *   Errors: a non-zero bt_status leaves outputs unspecified;
 *     bt_last_error() returns a thread-local message for the last failure.
 *   Threading: calls that use the shared workspace (bt_support,
 *     bt_index_build, bt_decompose, bt_decompose_variant, bt_decompose_pc,
 *     bt_decompose_batch, bt_bitruss_components, bt_tune) serialise on an
 *     internal lock; engines use workspaces of their own.  Cooperative peel
 *     launches (all of the above that peel, and engine batches) run one at
 *     a time in the process.
 */
#ifndef BT_H
#define BT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bt_status {
    BT_OK = 0,
    BT_EINVAL = 1,     /* malformed graph or argument; no output written */
    BT_ENOMEM = 2,     /* device allocation failed; bt_last_error names the size */
    BT_EOVERFLOW = 3,  /* a size limit above was exceeded */
    BT_EDEVICE = 4,    /* a HIP call failed */
    BT_EBUSY = 5       /* engine cannot admit the request now */
} bt_status;

typedef struct bt_csr {
    int32_t n_upper;
    int32_t n_lower;
    int64_t m;
    const int64_t *row_ptr; /* device, int64[n_upper + 1] */
    const int32_t *col;     /* device, int32[m] */
} bt_csr;

/* Counters of one decomposition (all filled by bt_decompose when non-NULL). */
typedef struct bt_stats {
    int64_t butterflies;      /* total butterflies of the graph */
    int64_t wedges_po;        /* priority-obeyed wedges walked (Definition 9) */
    int64_t blooms;           /* maximal priority-obeyed blooms */
    int64_t bloom_wedges;     /* sum of bloom numbers = wedges stored in the index */
    int64_t index_bytes;      /* device bytes of the BE-Index */
    int64_t levels;           /* distinct bitruss levels visited by the peel */
    int64_t rounds;           /* peel rounds (frontiers processed) */
    int64_t max_phi;          /* largest bitruss number */
    int64_t support_updates;  /* support decrements issued by the peel */
    int64_t bloom_visits;     /* touched-bloom visits in batch bloom processing */
    float ms_prepare;         /* validation, priority order, rank-space CSR */
    float ms_count;           /* wedge counting and index emission */
    float ms_link;            /* edge-to-wedge links */
    float ms_peel;            /* peel */
    float ms_peel_kernel;     /* device time of the peel kernels alone (HIP events) */
    int32_t peel_launches;    /* peel kernel (or round-graph) launches */
    int32_t passes;           /* subgraph passes (1, or BiT-PC's thresholds) */
    int64_t support_updates_unbatched; /* the plain peel's decrements had each
                                 survivor taken one unit per removed wedge (no
                                 batch bloom processing, Section V-B); 0 where
                                 not counted */
    int64_t wedge_visits;     /* live wedges of touched blooms visited by batch
                                 bloom processing, summed over rounds: each such
                                 visit lowers the wedge's two edges once */
    int64_t peel_yields;      /* peel launches that ended early to give the
                                 device to a peel of a much smaller batch
                                 waiting in another thread, then resumed */
} bt_stats;

/* Opaque device-resident BE-Index. */
typedef struct bt_index bt_index;

typedef struct bt_index_info {
    int64_t m;
    int64_t blooms;        /* n_B */
    int64_t bloom_wedges;  /* n_W: each wedge is a twin-edge pair */
    int64_t links;         /* 2 n_W edge-to-bloom links */
    int64_t butterflies;
    int64_t wedges_po;
    int64_t bytes;         /* device memory held by the index */
} bt_index_info;

/*
 * Butterfly support of every edge (Definition 2; the counting step of
 * Algorithm 4, done through priority-obeyed wedges as in Algorithm 3's
 * first sweep, with Lemmas 1-3 turning bloom sizes into supports).
 *   g               graph (device CSR), validated on the device.
 *   sup_out         device int64[m]: support of edge e (may be NULL if m == 0).
 *   butterflies_out host int64 (nullable): total butterflies.
 */
bt_status bt_support(const bt_csr *g, int64_t *sup_out, int64_t *butterflies_out,
                     hipStream_t stream);

/*
 * Build the BE-Index (Section IV, Algorithm 3): every maximal
 * priority-obeyed bloom with its bloom number, its wedges (twin-edge
 * pairs, Definition 8) and, per edge, the links to the blooms holding it.
 *   out  receives a handle owning device memory; free with bt_index_free.
 */
bt_status bt_index_build(const bt_csr *g, bt_index **out, hipStream_t stream);

bt_status bt_index_info_get(const bt_index *idx, bt_index_info *info);

/*
 * Copy the index to HOST arrays (for inspection and tests).  Bloom b owns
 * wedges [bloom_woff[b], bloom_woff[b+1]); its bloom number is that length.
 * Wedge w is the twin pair (wedge_ea[w], wedge_eb[w]): wedge_ea is the edge
 * at the bloom's highest-priority vertex, wedge_eb the edge at the other
 * dominant-layer vertex.  edge_link_off/edge_link (nullable) give, for
 * edge e, the wedges holding it: edge_link[edge_link_off[e] ..
 * edge_link_off[e+1]).  Sizes: bloom_woff[blooms+1], wedge_*[bloom_wedges],
 * edge_link_off[m+1], edge_link[2*bloom_wedges], sup[m] (nullable).
 */
bt_status bt_index_export(const bt_index *idx, int64_t *bloom_woff, int32_t *wedge_ea,
                          int32_t *wedge_eb, int64_t *edge_link_off, int64_t *edge_link,
                          int64_t *sup);

void bt_index_free(bt_index *idx);

/*
 * Bitruss number of every edge (Definition 5): support counting, index
 * construction and the bulk-synchronous peel through blooms with batch
 * edge and batch bloom processing (Algorithm 5).
 *   sup_out  device int64[m] (nullable): initial supports.
 *   phi_out  device int64[m]: bitruss numbers.
 *   stats    host (nullable): counters and per-phase device times.
 * Graphs of 2^20 edges or more are peeled with each layer renumbered by
 * decreasing degree (the support atomics then land close together); the
 * outputs are always in the caller's edge order.
 */
bt_status bt_decompose(const bt_csr *g, int64_t *sup_out, int64_t *phi_out,
                       bt_stats *stats, hipStream_t stream);

/*
 * bt_decompose with a round-by-round trace, for inspecting the peel on small
 * graphs (at most 65536 edges, else BT_EOVERFLOW): the rounds of the
 * bulk-synchronous peel of Algorithm 5 (Section V-B) that remove edges,
 * each with
 *   round_level[k]             its level (the minimum support it peels at),
 *   removed[k*m + e]           1 if edge e is removed in round k, else 0,
 *   sup[k*m + e]               the support of e after round k (supports are
 *                              lowered without the clamp at the level, so an
 *                              edge removed earlier may read below it),
 *   wedge_k[k*max_wedges + w]  the bloom number (live wedges) of the bloom
 *                              holding wedge w after round k (its butterflies
 *                              are k(k-1)/2),
 * and the index it peeled through: wedge w is the twin pair
 * (wedge_ea[w], wedge_eb[w]), as in bt_index_export.  All trace buffers are
 * HOST memory of the sizes shown; *n_rounds and *n_wedges receive the counts
 * (BT_EOVERFLOW if they exceed max_rounds or max_wedges).  phi_out is a
 * device int64[m] as for bt_decompose.  The rounds run one at a time from
 * the host, so this is slow; results equal bt_decompose.
 */
bt_status bt_decompose_trace(const bt_csr *g, int64_t *phi_out, int32_t max_rounds,
                             int32_t *n_rounds, int32_t *round_level, int8_t *removed,
                             int64_t *sup, int64_t max_wedges, int64_t *n_wedges,
                             int32_t *wedge_ea, int32_t *wedge_eb, int32_t *wedge_k,
                             hipStream_t stream);

/* Peel variants, for measuring what batch bloom processing saves
 * (Section V-B and the evaluation of the batch optimisations). */
typedef enum bt_peel_variant {
    /* BiT-BU++ (Algorithm 5): batch edge and batch bloom processing; a
     * survivor of a bloom that lost C wedges this round takes one decrement
     * of C.  This is bt_decompose. */
    BT_PEEL_BATCH_BLOOM = 0,
    /* BiT-BU+: batch edge processing only; a survivor takes C decrements of
     * one, as when each removed edge updates its blooms on its own
     * (Algorithm 4's removal step).  The bloom's wedges are still read once
     * per round. */
    BT_PEEL_BATCH_EDGE = 1,
    /* BiT-BU++, or BiT-PC (bt_decompose_pc, tau = 0.05) when the graph has at
     * least 16,384 butterflies per edge: there the peel is bound by support
     * updates, which BiT-PC cuts (20M-edge hub graph, 43k per edge: 40.6 s
     * against 67.4 s), while below it the rounds bound it and BiT-PC's extra
     * passes cost more (5M-edge Chung-Lu graph, 930 per edge; 2M-edge
     * request graph, 5.9k per edge: equal).  Decided after the index build. */
    BT_PEEL_AUTO = 2
} bt_peel_variant;

/*
 * bt_decompose with a chosen peel variant (bt_peel_variant; else
 * BT_EINVAL).  Results are identical for every variant; stats
 * support_updates counts the decrements the variant issued (for
 * BT_PEEL_BATCH_EDGE it equals BT_PEEL_BATCH_BLOOM's
 * support_updates_unbatched).  Arguments as for bt_decompose.
 */
bt_status bt_decompose_variant(const bt_csr *g, int32_t variant, int64_t *sup_out,
                               int64_t *phi_out, bt_stats *stats, hipStream_t stream);

/*
 * Launch parameters.  They decide how the wedge sweeps cut start vertices
 * into tasks and how many workgroups the sweeps and the peel run; no result
 * depends on them.  The library keeps one entry per kind of call (a single
 * graph, or a batch) and size class (bit_length(m) - 10, clamped to
 * [0, 21]); a call uses its class's entry, else the nearest class of its
 * kind that has one, else the defaults shown.  If the environment variable
 * BT_TUNE_CACHE names a file written by bt_tune_save, it is loaded at the
 * first lookup.  Not part of the paper: an implementation aid.
 */
typedef struct bt_tune_params {
    int32_t hash_max_work;   /* start vertices with at most this many priority-obeyed
                                wedges count them in one LDS hash task; [1, 2048], 2048 */
    int32_t dense_chunk;     /* heavier start vertices count in dense ranges of this many
                                end vertices, one workgroup each; [64, 6144], 6144 */
    int32_t wedge_wg_per_cu; /* wedge-sweep workgroups per compute unit; [1, 16], 2 */
    int32_t peel_blocks;     /* workgroups of the cooperative peel (0: three per four
                                compute units; capped at what can be resident);
                                [0, 65536], 0 */
    int32_t active_min;      /* smallest active set the peel rebuilds; >= 1, 16384 */
} bt_tune_params;

enum { BT_TUNE_INDEX = 1, BT_TUNE_PEEL = 2 };

/*
 * Autotuner: times candidate values of each parameter in turn (coordinate
 * search, the others held; a change must gain 2%) on these graphs, and
 * stores the best in the entry of their kind and size class.  n_graphs ==
 * 1 tunes single-graph calls (index parameters timed on the index build,
 * peel parameters on the peel kernel); n_graphs > 1 tunes batches
 * (bt_decompose_batch timed whole; class of the summed edge count).  `what`
 * is a mask of BT_TUNE_INDEX and BT_TUNE_PEEL.  Runs several whole
 * decompositions: seconds for a graph of millions of edges.
 *   gs   host array of n_graphs device graphs.
 *   out  host (nullable): the stored parameters.
 * Errors as for bt_decompose / bt_decompose_batch; on an error the entry
 * is left as it was.
 */
bt_status bt_tune(const bt_csr *gs, int32_t n_graphs, uint32_t what, bt_tune_params *out,
                  hipStream_t stream);

/* The parameters a call of this kind (batch: 0 or 1) and edge count uses. */
bt_status bt_tune_get(int32_t batch, int64_t m, bt_tune_params *out);
/* Sets the entry of this kind and size class (BT_EINVAL if out of range). */
bt_status bt_tune_set(int32_t batch, int64_t m, const bt_tune_params *p);
/* Forgets every entry (calls then use the defaults). */
bt_status bt_tune_reset(void);
/* Writes the entries to a text file: a header "bt-tune 1 <device arch>",
 * then one line per entry "<single|batch> <class> <the five parameters>". */
bt_status bt_tune_save(const char *path);
/* Reads such a file and sets its entries (BT_EINVAL if it is malformed, has
 * a value out of range, or was written for another device architecture;
 * then no entry changes). */
bt_status bt_tune_load(const char *path);

/*
 * Bitruss numbers by progressive compression, BiT-PC (Section V-C,
 * Algorithms 6-7): for thresholds eps = k_max, k_max - alpha, ..., 0 with
 * alpha = ceil(k_max * tau) and k_max the largest k such that k edges have
 * support >= k, build the BE-Index of the subgraph of edges whose support in
 * G is >= eps, with edges fixed by earlier thresholds kept in their blooms
 * but never updated, and peel it, fixing the edges of the eps-bitruss.
 * Results equal bt_decompose; fewer support updates on hub-heavy graphs.
 *   tau      in (0, 1] (else BT_EINVAL); the paper suggests 0.05 - 0.2.
 *   sup_out  device int64[m] (nullable): supports in G.
 *   phi_out  device int64[m]: bitruss numbers.
 *   stats    host (nullable): sums over the passes (passes = thresholds
 *            whose subgraph held an unfixed edge; blooms and bloom_wedges
 *            summed over passes, index_bytes the largest pass).
 */
bt_status bt_decompose_pc(const bt_csr *g, double tau, int64_t *sup_out, int64_t *phi_out,
                          bt_stats *stats, hipStream_t stream);

/*
 * Connected components of the k-bitruss H_k (Definition 4: by Definition 5,
 * the edges with phi_e >= k), the cohesive subgraphs that the applications
 * of Section I look for.
 *   phi              device int64[m]: bitruss numbers (from bt_decompose).
 *   k                any integer; k <= 0 takes every edge.
 *   comp_out         device int32[m]: the component of edge e, numbered
 *                    0, 1, ... in order of each component's smallest edge id;
 *                    -1 where phi_e < k.
 *   n_components_out host int64 (nullable): the number of components.
 * The graph is validated (BT_EINVAL if malformed).
 */
bt_status bt_bitruss_components(const bt_csr *g, const int64_t *phi, int64_t k,
                                int32_t *comp_out, int64_t *n_components_out,
                                hipStream_t stream);

/*
 * Decompose many independent graphs in shared launches.  gs is a HOST
 * array of n_graphs descriptors (device CSRs); sup_out / phi_out are HOST
 * arrays of n_graphs device pointers (sup_out may be NULL, or hold NULLs;
 * phi_out[i] may be NULL only for a graph without edges).  The graphs are
 * decomposed as disjoint unions of at most 2^26 edges (larger ones alone),
 * cut from the graphs in decreasing edge count; within a union every graph
 * peels at its own level when all of them have at most 2^19 edges, else
 * the union peels with one shared level.  Inside a union each graph's
 * vertices are renumbered by decreasing degree (the support atomics then
 * land close together); results are written back in each caller's edge
 * order and equal bt_decompose on each graph.
 * stats (nullable) receives the sums over all graphs; rounds and
 * peel_launches are summed over the unions, levels is the sum over the
 * unions of each union's largest per-graph level count.
 */
bt_status bt_decompose_batch(const bt_csr *gs, int32_t n_graphs, int64_t *const *sup_out,
                             int64_t *const *phi_out, bt_stats *stats, hipStream_t stream);

/*
 * Serving engine with continuous batching (for request streams).
 *
 * bt_engine_create: `slots` worker slots (0: 2), each with its own HIP
 *   stream, cached workspace and worker thread; slots = -1 creates a
 *   caller-driven engine instead (one slot, no threads: see
 *   bt_engine_step); `hbm_budget` bytes of device memory for
 *   the engine (0: half of the free memory); at most `max_batch` requests
 *   per batch (0: 1024).  The peel of a batch holds most of the GPU, so the
 *   peels of different slots take turns; a second slot counts and builds
 *   the index of the next batch while one slot's batch peels, and when that
 *   batch is of a smaller size class, the running peel ends its launch
 *   between two rounds (within 32 rounds), lets the smaller batch peel,
 *   and resumes where it stopped.  With two or more slots one is kept for
 *   the small class: a slot starts a larger class's batch only while fewer
 *   than slots - 1 others run one.
 *   Memory: the budget covers every slot's cached workspace plus what its
 *   running batch may still allocate (the submit-time estimate, replaced by
 *   the exact peel state once the batch's index is built); a slot frees its
 *   cache, or asks idle slots to free theirs, when that is what keeps a
 *   request out.
 * bt_engine_submit: queue one request.  Validates the graph and estimates
 *   its device memory on the device (index and peel state bounded through
 *   the wedge bound of Lemma 6, sum over edges of min(d(u), d(v)), plus
 *   per-edge arrays).  BT_EINVAL for a malformed graph, BT_EBUSY if the
 *   estimate exceeds the whole budget.  Graph and outputs are caller-owned
 *   DEVICE memory that must stay valid until the request completes;
 *   sup_out may be NULL.  Results equal bt_decompose on the same graph.
 * A free slot picks a size class (below) and admits, in arrival order,
 *   queued requests of that class that fit the budget left by the other
 *   slots, and decomposes them as one batch (bt_decompose_batch
 *   semantics).  A batch
 *   holds one size class: below 2^14 edges, below 2^19, or larger (at most
 *   eight of those at a time).  The smallest class queued goes first, unless
 *   the oldest request of a larger class has waited 10 s.  Requests that
 *   arrive meanwhile go to the next free slot, so batches overlap on the
 *   device.
 * bt_engine_step: caller-driven engines only (else BT_EINVAL): admits the
 *   batch a free slot would admit now and decomposes it on the calling
 *   thread, on the engine's own stream; *n_done (nullable) receives the
 *   number of requests it completed (0: nothing was queued).  Their
 *   (id, status) pairs are then ready for bt_engine_poll.  Steps from
 *   several threads take turns.
 * bt_engine_poll: moves up to `cap` completed (id, status) pairs to the
 *   caller's host arrays; *n_done receives how many.
 * bt_engine_drain: blocks until every submitted request has completed (a
 *   caller-driven engine steps on the calling thread until its queue is
 *   empty).
 * bt_engine_memory: the budget, the bytes the slots' workspaces hold now,
 *   the largest such sum so far, and the largest sum of held plus reserved
 *   bytes so far (which admission keeps within the budget).
 * bt_engine_destroy: drains, stops the workers and frees the engine.
 */
typedef struct bt_engine bt_engine;

bt_status bt_engine_create(int64_t hbm_budget, int32_t slots, int32_t max_batch,
                           bt_engine **out);
bt_status bt_engine_submit(bt_engine *engine, const bt_csr *g, int64_t *sup_out,
                           int64_t *phi_out, uint64_t id);
bt_status bt_engine_step(bt_engine *engine, int32_t *n_done);
bt_status bt_engine_poll(bt_engine *engine, uint64_t *ids, int32_t *status, int32_t cap,
                         int32_t *n_done);
bt_status bt_engine_drain(bt_engine *engine);
/* Batches run, requests admitted, requests waiting, and peel launches that
 * gave the device to a much smaller batch of another slot (host pointers,
 * nullable). */
bt_status bt_engine_stats(bt_engine *engine, int64_t *batches, int64_t *admitted,
                          int64_t *queued, int64_t *peel_yields);
/* Host pointers, nullable. */
bt_status bt_engine_memory(bt_engine *engine, int64_t *budget, int64_t *held,
                           int64_t *peak_held, int64_t *peak_committed);
void bt_engine_destroy(bt_engine *engine);

/*
 * Device-memory hook.  Every device buffer the library allocates (the
 * cached workspaces of calls and engine slots, bt_index handles) is taken
 * with alloc(bytes, ctx) and returned with free(ptr, bytes, ctx) on the
 * device current at the call; alloc returns NULL on failure, and the call
 * that needed the memory then fails with BT_ENOMEM, bt_last_error naming
 * the byte count (the library stays usable).  Before a block goes back to
 * free() the library waits for the device to finish its work, so a caching
 * allocator may hand it out again at once.  Blocks are always returned to
 * the hook that made them, even after the hook changes.  Both NULL
 * restores hipMalloc / hipFree; one NULL without the other is BT_EINVAL.
 * Not in the paper: lets a host framework (such as PyTorch's caching
 * allocator) own the library's device memory.
 */
typedef void *(*bt_alloc_fn)(size_t bytes, void *ctx);
typedef void (*bt_free_fn)(void *ptr, size_t bytes, void *ctx);
bt_status bt_set_allocator(bt_alloc_fn alloc, bt_free_fn free, void *ctx);

/*
 * bt_support without allocating: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, results and errors as bt_support.
 * Its scratch memory is a static device array of 64 MiB that every GPU the
 * library runs on holds until the process ends; no hipMalloc, hipFree or
 * allocator hook is called.  Graphs with more than 2^18 edges or more than
 * 2^18 vertices (n_upper + n_lower) fail with BT_EOVERFLOW.  Calls on one
 * device share that array: the library serialises them within a process
 * (each call leaves the array to the next), so work of two calls that
 * overlapped on one GPU, from different processes' copies aside, would
 * race; the call returns only after its work on `stream` is complete.
 */
bt_status bt_support_noalloc(const bt_csr *g, int64_t *sup_out, int64_t *butterflies_out,
                             hipStream_t stream);

/* Free the cached device workspace (it regrows on the next call). */
void bt_release_workspace(void);

/* Thread-local text of the last error. */
const char *bt_last_error(void);

/* Library version string. */
const char *bt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BT_H */
