// pc.hip - device steps of BiT-PC, the progressive compression approach
// (Section V-C, Algorithms 6-7).
//
// Lemma 11: the k-bitruss lies inside G_{>=k}, the subgraph of edges whose
// support in G is at least k.  BiT-PC therefore works down a falling
// threshold eps: it takes G_{>=eps}, builds the BE-Index of that subgraph,
// and peels it, fixing the bitruss numbers of the edges that are removed at
// a level >= eps (the eps-bitruss).  Edges fixed in an earlier pass stay in
// later subgraphs so that their blooms keep their true size, but they get no
// updates: the index marks them, and the peel neither decrements nor
// removes them (Algorithm 6 lines 8-14).  The steps here build each pass's
// subgraph, mark its fixed edges, and fold each pass's results back.
#include <climits>

#include "pipeline.h"

namespace bt {

namespace {

constexpr int kB = 256;
constexpr uint32_t kFixed = 0x80000000u;

__global__ void k_low32(const uint64_t *supl, int64_t m, int32_t *sup0) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        sup0[e] = (int32_t)(supl[e] & 0xffffffffu);
}

// Number of edges with support >= k.
__global__ void k_count_ge(const int32_t *sup0, int64_t m, int32_t k, unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        c += sup0[e] >= k ? 1 : 0;
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

__global__ void k_keep(const int32_t *sup0, int64_t m, int32_t eps, int32_t *keep) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        keep[e] = sup0[e] >= eps ? 1 : 0;
}

// Row i of the subgraph starts at the number of kept edges before row i.
__global__ void k_sub_rows(const int64_t *row_ptr, int32_t nu, const int64_t *pos,
                           int64_t *sub_row_ptr) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= nu;
         i += (int64_t)gridDim.x * blockDim.x)
        sub_row_ptr[i] = pos[row_ptr[i]];
}

// Kept edges keep their order; orig maps subgraph edge ids back.
__global__ void k_sub_edges(const int32_t *col, const int32_t *keep, const int64_t *pos,
                            int64_t m, const int32_t *phi_glob, int32_t *sub_col, int32_t *orig,
                            int32_t *fixed, unsigned long long *n_open) {
    unsigned long long c = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[e]) continue;
        const int64_t p = pos[e];
        sub_col[p] = col[e];
        orig[p] = (int32_t)e;
        const int32_t fx = phi_glob[e] >= 0 ? 1 : 0;
        fixed[p] = fx;
        c += fx ? 0 : 1;
    }
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(n_open, c);
}

__global__ void k_mark_wedges(int32_t *wea, int32_t *web, int64_t nw, const int32_t *fixed) {
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = wea[w], b = web[w];
        if (fixed[a]) wea[w] = (int32_t)((uint32_t)a | kFixed);
        if (fixed[b]) web[w] = (int32_t)((uint32_t)b | kFixed);
    }
}

__global__ void k_mark_links(uint3 *link, int64_t n, const int32_t *fixed) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = link[j].z;
        if (fixed[t]) link[j].z = t | kFixed;
    }
}

// Edges of the eps-bitruss get their numbers (Algorithm 7: only edges
// removed at a level >= eps are assigned in this pass).
__global__ void k_collect(const int64_t *phi_sub, const int32_t *orig, const int32_t *fixed,
                          int64_t m_sub, int32_t eps, int32_t *phi_glob) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m_sub;
         e += (int64_t)gridDim.x * blockDim.x)
        if (!fixed[e] && phi_sub[e] >= eps) phi_glob[orig[e]] = (int32_t)phi_sub[e];
}

__global__ void k_widen(const int32_t *phi_glob, int64_t m, int64_t *phi_out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        phi_out[e] = phi_glob[e];
}

}  // namespace

int32_t pc_kmax(const uint64_t *supl, int64_t m, int32_t *sup0, Workspace &ws, hipStream_t s) {
    if (m == 0) return 0;
    k_low32<<<grid_for(m, kB, 16384), kB, 0, s>>>(supl, m, sup0);
    BT_CHECK_LAUNCH();
    // Largest k with at least k edges of support >= k (Section V-C, Step 1),
    // by bisection on k in [0, m].
    unsigned long long *cnt = ws.get<unsigned long long>("pc_cnt", 1);
    int64_t *h = ws.host(2);
    int64_t lo = 0, hi = std::min<int64_t>(m, INT_MAX);
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        zero_bytes(cnt, sizeof *cnt, s);
        k_count_ge<<<grid_for(m, kB, 4096), kB, 0, s>>>(sup0, m, (int32_t)mid, cnt);
        BT_CHECK_LAUNCH();
        BT_HIP(hipMemcpyAsync(h, cnt, sizeof *cnt, hipMemcpyDeviceToHost, s));
        BT_HIP(hipStreamSynchronize(s));
        if (h[0] >= mid)
            lo = mid;
        else
            hi = mid - 1;
    }
    return (int32_t)lo;
}

int64_t pc_subgraph(const bt_csr &g, const int32_t *sup0, int32_t eps, const int32_t *phi_glob,
                    PcSubgraph &sg, Workspace &ws, hipStream_t s) {
    const int64_t m = g.m;
    int32_t *keep = ws.get<int32_t>("pc_keep", m);
    int64_t *pos = ws.get<int64_t>("pc_pos", m + 1);
    k_keep<<<grid_for(m, kB, 16384), kB, 0, s>>>(sup0, m, eps, keep);
    BT_CHECK_LAUNCH();
    scan_exclusive_i32_to_i64(keep, pos, m, ws, s);
    int64_t *h = ws.host(2);
    BT_HIP(hipMemcpyAsync(h, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    const int64_t ms = h[0];
    sg.row_ptr = ws.get<int64_t>("pc_rowptr", (int64_t)g.n_upper + 1);
    sg.col = ws.get<int32_t>("pc_col", ms);
    sg.orig = ws.get<int32_t>("pc_orig", ms);
    sg.fixed = ws.get<int32_t>("pc_fixed", ms);
    unsigned long long *n_open = ws.get<unsigned long long>("pc_open", 1);
    zero_bytes(n_open, sizeof *n_open, s);
    k_sub_rows<<<grid_for((int64_t)g.n_upper + 1, kB, 16384), kB, 0, s>>>(g.row_ptr, g.n_upper,
                                                                          pos, sg.row_ptr);
    BT_CHECK_LAUNCH();
    k_sub_edges<<<grid_for(m, kB, 16384), kB, 0, s>>>(g.col, keep, pos, m, phi_glob, sg.col,
                                                      sg.orig, sg.fixed, n_open);
    BT_CHECK_LAUNCH();
    BT_HIP(hipMemcpyAsync(h, n_open, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    sg.g = bt_csr{g.n_upper, g.n_lower, ms, sg.row_ptr, sg.col};
    sg.open = h[0];
    return ms;
}

void mark_fixed(IndexArrays &ix, const int32_t *fixed, hipStream_t s) {
    if (ix.n_w == 0) return;
    k_mark_wedges<<<grid_for(ix.n_w, kB, 16384), kB, 0, s>>>(ix.wea, ix.web, ix.n_w, fixed);
    BT_CHECK_LAUNCH();
    k_mark_links<<<grid_for(2 * ix.n_w, kB, 16384), kB, 0, s>>>(ix.link, 2 * ix.n_w, fixed);
    BT_CHECK_LAUNCH();
}

void pc_collect(const int64_t *phi_sub, const PcSubgraph &sg, int32_t eps, int32_t *phi_glob,
                hipStream_t s) {
    if (sg.g.m == 0) return;
    k_collect<<<grid_for(sg.g.m, kB, 16384), kB, 0, s>>>(phi_sub, sg.orig, sg.fixed, sg.g.m, eps,
                                                         phi_glob);
    BT_CHECK_LAUNCH();
}

void pc_widen(const int32_t *phi_glob, int64_t m, int64_t *phi_out, hipStream_t s) {
    if (m == 0) return;
    k_widen<<<grid_for(m, kB, 16384), kB, 0, s>>>(phi_glob, m, phi_out);
    BT_CHECK_LAUNCH();
}

}  // namespace bt
