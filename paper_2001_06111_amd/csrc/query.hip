// query.hip - k-bitruss subgraphs and their connected components.
//
// H_k, the k-bitruss (Definition 4), is the set of edges with phi_e >= k
// (Definition 5); the cohesive groups the paper's applications look for
// (Section I) are its connected components.  Given the bitruss numbers,
// the components come from a lock-free union-find over the vertices that
// H_k's edges join: every root is hooked under a smaller root with one
// compare-and-swap, so parents only decrease and no cycle can form.  Edges
// are then labelled by component, numbered in order of each component's
// smallest edge id, which makes the labelling unique.
#include <climits>

#include "pipeline.h"

namespace bt {

namespace {

constexpr int kB = 256;

template <typename T> __device__ __forceinline__ T ldc(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t x) {
    int32_t p = ldc(&parent[x]);
    while (p != x) {
        x = p;
        p = ldc(&parent[x]);
    }
    return x;
}

__global__ void k_cc_init(int32_t *parent, int32_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        parent[v] = (int32_t)v;
}

// Vertex ids: lower j -> j, upper i -> n_lower + i.
__global__ void k_cc_hook(const int64_t *row_ptr, const int32_t *col, int32_t nu, int32_t nl,
                          const int64_t *phi, int64_t k, int32_t *parent) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < nu;
         i += waves) {
        const int32_t u = nl + (int32_t)i;
        for (int64_t e = row_ptr[i] + lane_id(); e < row_ptr[i + 1]; e += kWave) {
            if (phi[e] < k) continue;
            int32_t a = u, b = col[e];
            while (true) {
                a = find_root(parent, a);
                b = find_root(parent, b);
                if (a == b) break;
                if (a < b) {
                    const int32_t t = a;
                    a = b;
                    b = t;
                }
                // Hook the larger root a under b; retry if a stopped being a root.
                if (atomicCAS(&parent[a], a, b) == a) break;
            }
        }
    }
}

__global__ void k_cc_min_edge(const int64_t *row_ptr, int32_t nu, int32_t nl, const int64_t *phi,
                              int64_t k, int32_t *parent, int32_t *min_edge) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < nu;
         i += waves)
        for (int64_t e = row_ptr[i] + lane_id(); e < row_ptr[i + 1]; e += kWave)
            if (phi[e] >= k) atomicMin(&min_edge[find_root(parent, nl + (int32_t)i)], (int32_t)e);
}

// first[e] = 1 when e is the smallest edge of its component.
__global__ void k_cc_first(const int64_t *row_ptr, int32_t nu, int32_t nl, const int64_t *phi,
                           int64_t k, int32_t *parent, const int32_t *min_edge, int32_t *first) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < nu;
         i += waves)
        for (int64_t e = row_ptr[i] + lane_id(); e < row_ptr[i + 1]; e += kWave)
            first[e] = phi[e] >= k &&
                       min_edge[find_root(parent, nl + (int32_t)i)] == (int32_t)e ? 1 : 0;
}

__global__ void k_cc_label(const int64_t *row_ptr, int32_t nu, int32_t nl, const int64_t *phi,
                           int64_t k, int32_t *parent, const int32_t *min_edge, const int64_t *pos,
                           int32_t *comp) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < nu;
         i += waves)
        for (int64_t e = row_ptr[i] + lane_id(); e < row_ptr[i + 1]; e += kWave)
            comp[e] = phi[e] >= k
                          ? (int32_t)pos[min_edge[find_root(parent, nl + (int32_t)i)]]
                          : -1;
}

}  // namespace

int64_t bitruss_components(const bt_csr &g, const int64_t *phi, int64_t k, int32_t *comp,
                           Workspace &ws, hipStream_t s) {
    const int32_t nu = g.n_upper, nl = g.n_lower;
    const int32_t n = nu + nl;
    const int64_t m = g.m;
    if (m == 0) return 0;
    int32_t *parent = ws.get<int32_t>("q_parent", n);
    int32_t *min_edge = ws.get<int32_t>("q_min_edge", n);
    int32_t *first = ws.get<int32_t>("q_first", m);
    int64_t *pos = ws.get<int64_t>("q_pos", m + 1);
    const int grid_v = grid_for(n, kB, 16384);
    const int grid_r = grid_for((int64_t)nu * kWave, kB, 16384);
    k_cc_init<<<grid_v, kB, 0, s>>>(parent, n);
    BT_CHECK_LAUNCH();
    fill_i32(min_edge, INT_MAX, n, s);
    k_cc_hook<<<grid_r, kB, 0, s>>>(g.row_ptr, g.col, nu, nl, phi, k, parent);
    BT_CHECK_LAUNCH();
    k_cc_min_edge<<<grid_r, kB, 0, s>>>(g.row_ptr, nu, nl, phi, k, parent, min_edge);
    BT_CHECK_LAUNCH();
    k_cc_first<<<grid_r, kB, 0, s>>>(g.row_ptr, nu, nl, phi, k, parent, min_edge, first);
    BT_CHECK_LAUNCH();
    scan_exclusive_i32_to_i64(first, pos, m, ws, s);
    k_cc_label<<<grid_r, kB, 0, s>>>(g.row_ptr, nu, nl, phi, k, parent, min_edge, pos, comp);
    BT_CHECK_LAUNCH();
    int64_t *h = ws.host(2);
    BT_HIP(hipMemcpyAsync(h, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    return h[0];
}

}  // namespace bt
