// graph.hip - input validation, vertex priority order and the rank-space
// adjacency (priority of Definition 6; the "p(v) < p(u)" filters of
// Algorithm 3's sweeps become row prefixes).
#include "pipeline.h"

namespace bt {

namespace {

constexpr int kBlock = 256;

// Validation flags.
enum : int32_t {
    kBadRowPtr = 1,   // row_ptr not a partition of [0, m)
    kBadCol = 2,      // lower id out of range
    kUnsorted = 4,    // lower ids not strictly increasing in a row (or duplicate)
};

// One wave per row.  Reads col only inside a row whose bounds were checked.
__global__ __launch_bounds__(kBlock) void k_validate(const int64_t *row_ptr, const int32_t *col,
                                                     int32_t n_upper, int32_t n_lower,
                                                     int64_t m, int32_t *flags) {
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    int32_t bad = 0;
    for (int64_t i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < n_upper;
         i += waves) {
        const int64_t a = row_ptr[i], b = row_ptr[i + 1];
        if (i == 0 && a != 0) bad |= kBadRowPtr;
        if (i == n_upper - 1 && b != m) bad |= kBadRowPtr;
        if (a < 0 || b < a || b > m) {
            bad |= kBadRowPtr;
            continue;
        }
        for (int64_t k = a + lane_id(); k < b; k += kWave) {
            const int32_t c = col[k];
            if (c < 0 || c >= n_lower) bad |= kBadCol;
            if (k + 1 < b && col[k + 1] <= c) bad |= kUnsorted;
        }
    }
    bad = wave_or(bad);
    if (lane_id() == 0 && bad) atomicOr(flags, bad);
}

// deg[gid]: lower j -> j, upper i -> n_lower + i.
__global__ void k_upper_degree(const int64_t *row_ptr, int32_t n_upper, int32_t n_lower,
                               int32_t *deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_upper;
         i += (int64_t)gridDim.x * blockDim.x)
        deg[n_lower + i] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
}

__global__ void k_lower_degree(const int32_t *col, int64_t m, int32_t *deg) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&deg[col[e]], 1);
}

// Sort key: layer above degree; the stable sort keeps id order on ties.
__global__ void k_rank_keys(const int32_t *deg, int32_t n_lower, int32_t n, uint64_t *keys,
                            uint32_t *vals) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        keys[v] = ((uint64_t)(v >= n_lower) << 31) | (uint64_t)deg[v];
        vals[v] = (uint32_t)v;
    }
}

// Graph of vertex v in a union (offsets of its layer, n + 1 entries).
__device__ __forceinline__ int32_t comp_of(const int64_t *off, int32_t n, int64_t local) {
    int32_t lo = 0, hi = n - 1;  // largest c with off[c] <= local
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= local) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Union: layer above graph above degree; the stable sort keeps id order.
__global__ void k_rank_keys_comp(const int32_t *deg, int32_t n_lower, int32_t n, Components cp,
                                 int cbits, uint64_t *keys, uint32_t *vals) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const bool up = v >= n_lower;
        const int32_t c = up ? comp_of(cp.u_off, cp.n, v - n_lower) : comp_of(cp.l_off, cp.n, v);
        keys[v] = ((uint64_t)up << (31 + cbits)) | ((uint64_t)c << 31) | (uint64_t)deg[v];
        vals[v] = (uint32_t)v;
    }
}

// zbase[p]: the first rank of p's graph in p's layer.
__global__ void k_zbase(const int32_t *new2old, int32_t n_lower, int32_t n, Components cp,
                        int32_t *zbase) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = new2old[p];
        const bool up = v >= n_lower;
        const int32_t c = up ? comp_of(cp.u_off, cp.n, v - n_lower) : comp_of(cp.l_off, cp.n, v);
        zbase[p] = up ? n_lower + (int32_t)cp.u_off[c] : (int32_t)cp.l_off[c];
    }
}

__global__ void k_rank_apply(const uint32_t *order, const int32_t *deg, int32_t n,
                             int32_t *old2new, int32_t *new2old, int32_t *deg_new) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)order[p];
        old2new[v] = (int32_t)p;
        new2old[p] = v;
        deg_new[p] = deg[v];
    }
}

// Two adjacency entries per edge; one wave per upper row.
__global__ __launch_bounds__(kBlock) void k_entries(const int64_t *row_ptr, const int32_t *col,
                                                    int32_t n_upper, int32_t n_lower,
                                                    const int32_t *old2new, int nb,
                                                    uint64_t *keys, uint32_t *vals) {
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < n_upper;
         i += waves) {
        const uint64_t ru = (uint64_t)old2new[n_lower + i];
        for (int64_t e = row_ptr[i] + lane_id(); e < row_ptr[i + 1]; e += kWave) {
            const uint64_t rl = (uint64_t)old2new[col[e]];
            keys[2 * e] = (ru << nb) | rl;
            vals[2 * e] = (uint32_t)e;
            keys[2 * e + 1] = (rl << nb) | ru;
            vals[2 * e + 1] = (uint32_t)e;
        }
    }
}

__global__ void k_entries_apply(const uint64_t *keys, const uint32_t *vals, int64_t n2,
                                uint64_t mask, int32_t *adj, int32_t *eid) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n2;
         j += (int64_t)gridDim.x * blockDim.x) {
        adj[j] = (int32_t)(keys[j] & mask);
        eid[j] = (int32_t)vals[j];
    }
}

__device__ __forceinline__ uint64_t prio(const int32_t *deg_new, const int32_t *new2old,
                                         int32_t v) {
    return ((uint64_t)deg_new[v] << 31) | (uint64_t)new2old[v];
}

// low[x] = number of neighbours of lower priority (a prefix of the row).
__global__ void k_low(const int64_t *off, const int32_t *adj, const int32_t *deg_new,
                      const int32_t *new2old, int32_t n, int32_t *low) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t px = prio(deg_new, new2old, (int32_t)x);
        int64_t lo = off[x], hi = off[x + 1];
        while (lo < hi) {  // first neighbour with priority above x
            const int64_t mid = lo + (hi - lo) / 2;
            if (prio(deg_new, new2old, adj[mid]) < px) lo = mid + 1;
            else hi = mid;
        }
        low[x] = (int32_t)(lo - off[x]);
    }
}

// rev for prefix entries (x -> y): position of x in row y.
__global__ void k_rev(const uint64_t *keys, int64_t n2, int nb, const int64_t *off,
                      const int32_t *adj, const int32_t *low, int32_t *rev) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n2;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = (int32_t)(keys[j] >> nb);
        int32_t r = 0;
        if (j - off[x] < low[x]) {
            const int32_t y = adj[j];
            int64_t lo = off[y], hi = off[y + 1];
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (adj[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            r = (int32_t)(lo - off[y]);
        }
        rev[j] = r;
    }
}

}  // namespace

void validate_graph(const bt_csr &g, Workspace &ws, hipStream_t s) {
    const int32_t nu = g.n_upper, nl = g.n_lower;
    const int64_t m = g.m;
    int64_t *hs = ws.host(4);
    int32_t *flags = ws.get<int32_t>("prep_flags", 4);
    zero_bytes(flags, 4 * sizeof(int32_t), s);
    if (nu > 0) {
        k_validate<<<grid_for((int64_t)nu * kWave, kBlock, 16384), kBlock, 0, s>>>(
            g.row_ptr, g.col, nu, nl, m, flags);
        BT_CHECK_LAUNCH();
    }
    BT_HIP(hipMemcpyAsync(hs, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    const int32_t f = *(int32_t *)hs;
    if (nu == 0 && m != 0) throw Error{BT_EINVAL, "graph has edges but no upper vertices"};
    if (f & kBadRowPtr) throw Error{BT_EINVAL, "row_ptr is not a partition of [0, m)"};
    if (f & kBadCol) throw Error{BT_EINVAL, "a lower id is out of range"};
    if (f & kUnsorted)
        throw Error{BT_EINVAL, "lower ids not strictly increasing within a row (duplicate edge?)"};
}

void prepare(const bt_csr &g, RankCSR &r, Workspace &ws, hipStream_t s,
             const Components *comps) {
    const int32_t nu = g.n_upper, nl = g.n_lower;
    const int64_t m = g.m;
    const int64_t n = (int64_t)nu + nl;
    r.tp = tune_params(false, m);
    r.n_lower = nl;
    r.n = (int32_t)n;
    r.m = m;

    validate_graph(g, ws, s);

    // Degrees and the priority order.
    int32_t *deg = ws.get<int32_t>("prep_deg", n);
    zero_bytes(deg, sizeof(int32_t) * (n > 0 ? n : 1), s);
    if (nu > 0) {
        k_upper_degree<<<grid_for(nu, 256, 8192), 256, 0, s>>>(g.row_ptr, nu, nl, deg);
        BT_CHECK_LAUNCH();
    }
    if (m > 0) {
        k_lower_degree<<<grid_for(m, 256, 16384), 256, 0, s>>>(g.col, m, deg);
        BT_CHECK_LAUNCH();
    }
    uint64_t *vkeys = ws.get<uint64_t>("prep_vkeys", n);
    uint32_t *vorder = ws.get<uint32_t>("prep_vorder", n);
    int32_t *old2new = ws.get<int32_t>("prep_old2new", n);
    int32_t *new2old = ws.get<int32_t>("prep_new2old", n);
    int32_t *deg_new = ws.get<int32_t>("prep_degnew", n);
    const bool uni = comps && comps->n > 1;
    r.zbase = nullptr;
    if (n > 0) {
        if (uni) {
            const int cbits = bits_for((uint64_t)(comps->n - 1));
            k_rank_keys_comp<<<grid_for(n, 256, 8192), 256, 0, s>>>(deg, nl, (int32_t)n, *comps,
                                                                   cbits, vkeys, vorder);
            BT_CHECK_LAUNCH();
            radix_sort_u64_u32(vkeys, vorder, n, 32 + cbits, ws, s);
        } else {
            k_rank_keys<<<grid_for(n, 256, 8192), 256, 0, s>>>(deg, nl, (int32_t)n, vkeys,
                                                              vorder);
            BT_CHECK_LAUNCH();
            radix_sort_u64_u32(vkeys, vorder, n, 32, ws, s);
        }
        k_rank_apply<<<grid_for(n, 256, 8192), 256, 0, s>>>(vorder, deg, (int32_t)n, old2new,
                                                            new2old, deg_new);
        BT_CHECK_LAUNCH();
        if (uni) {
            r.zbase = ws.get<int32_t>("rank_zbase", n);
            k_zbase<<<grid_for(n, 256, 8192), 256, 0, s>>>(new2old, nl, (int32_t)n, *comps,
                                                           r.zbase);
            BT_CHECK_LAUNCH();
        }
    }
    r.off = ws.get<int64_t>("rank_off", n + 1);
    scan_exclusive_i32_to_i64(deg_new, r.off, n, ws, s);

    // Rank-space rows sorted by neighbour priority.
    const int64_t n2 = 2 * m;
    const int nb = bits_for((uint64_t)(n > 0 ? n - 1 : 0)) > 0 ? bits_for((uint64_t)(n - 1)) : 1;
    uint64_t *ekeys = ws.get<uint64_t>("prep_ekeys", n2);
    uint32_t *evals = ws.get<uint32_t>("prep_evals", n2);
    r.adj = ws.get<int32_t>("rank_adj", n2);
    r.eid = ws.get<int32_t>("rank_eid", n2);
    r.rev = ws.get<int32_t>("rank_rev", n2);
    r.low = ws.get<int32_t>("rank_low", n);
    r.wpre = ws.get<int64_t>("rank_wpre", n2 + 1);
    if (m > 0) {
        k_entries<<<grid_for((int64_t)nu * kWave, kBlock, 16384), kBlock, 0, s>>>(
            g.row_ptr, g.col, nu, nl, old2new, nb, ekeys, evals);
        BT_CHECK_LAUNCH();
        radix_sort_u64_u32(ekeys, evals, n2, 2 * nb, ws, s);
        k_entries_apply<<<grid_for(n2, 256, 16384), 256, 0, s>>>(
            ekeys, evals, n2, (uint64_t(1) << nb) - 1, r.adj, r.eid);
        BT_CHECK_LAUNCH();
    }
    if (n > 0) {
        k_low<<<grid_for(n, 256, 8192), 256, 0, s>>>(r.off, r.adj, deg_new, new2old,
                                                     (int32_t)n, r.low);
        BT_CHECK_LAUNCH();
    }
    if (m > 0) {
        k_rev<<<grid_for(n2, 256, 16384), 256, 0, s>>>(ekeys, n2, nb, r.off, r.adj, r.low,
                                                       r.rev);
        BT_CHECK_LAUNCH();
    }
    scan_exclusive_i32_to_i64(r.rev, r.wpre, n2, ws, s);
}

// ------------------------------------------------------------- tasks

namespace {

__device__ __forceinline__ int64_t vertex_work(const int64_t *off, const int32_t *low,
                                               const int64_t *wpre, int32_t x) {
    return wpre[off[x] + low[x]] - wpre[off[x]];
}

// Start vertices with more than hash_max wedges count their end vertices
// in dense ranges of `chunk` counters, one task per range, over the ranks
// below x in x's layer (in a union, x's graph's part of it).
__device__ __forceinline__ int32_t z_base(const int32_t *zbase, int32_t x, int32_t n_lower) {
    return zbase ? zbase[x] : (x >= n_lower ? n_lower : 0);
}
__device__ __forceinline__ int32_t dense_chunks(int32_t x, int32_t base, int32_t chunk) {
    return (x - base + chunk - 1) / chunk;
}

__global__ void k_task_count(const int64_t *off, const int32_t *low, const int64_t *wpre,
                             const int32_t *zbase, int32_t n, int32_t n_lower, int32_t hash_max,
                             int32_t chunk, int64_t *counts) {
    int64_t nh = 0, nd = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = vertex_work(off, low, wpre, (int32_t)x);
        if (w == 0) continue;
        if (w <= hash_max) ++nh;
        else nd += dense_chunks((int32_t)x, z_base(zbase, (int32_t)x, n_lower), chunk);
    }
    nh = wave_sum(nh);
    nd = wave_sum(nd);
    if (lane_id() == 0) {
        if (nh) atomicAdd((unsigned long long *)&counts[0], (unsigned long long)nh);
        if (nd) atomicAdd((unsigned long long *)&counts[1], (unsigned long long)nd);
    }
}

__global__ void k_task_fill(const int64_t *off, const int32_t *low, const int64_t *wpre,
                            const int32_t *zbase, int32_t n, int32_t n_lower, int32_t hash_max,
                            int32_t chunk, WedgeTask *hash, WedgeTask *dense,
                            int32_t *cursors) {
    for (int64_t xi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; xi < n;
         xi += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = (int32_t)xi;
        const int64_t w = vertex_work(off, low, wpre, x);
        if (w == 0) continue;
        if (w <= hash_max) {
            int32_t cap = 128;
            while (cap < 2 * w) cap <<= 1;
            const int32_t p = atomicAdd(&cursors[0], 1);
            hash[p] = WedgeTask{x, 0, 0, cap};
        } else {
            const int32_t base = z_base(zbase, x, n_lower);
            const int32_t nc = dense_chunks(x, base, chunk);
            const int32_t p = atomicAdd(&cursors[1], nc);
            for (int32_t c = 0; c < nc; ++c) {
                const int32_t lo = base + c * chunk;
                const int32_t hi = min(lo + chunk, x);
                dense[p + c] = WedgeTask{x, lo, hi, hi - lo};
            }
        }
    }
}

}  // namespace

void make_tasks(const RankCSR &rc, TaskLists &t, Workspace &ws, hipStream_t s) {
    RankCSR &r = const_cast<RankCSR &>(rc);
    if (!tune_valid(r.tp)) throw Error{BT_EINVAL, "invalid launch parameters"};
    int64_t *counts = ws.get<int64_t>("task_counts", 4);
    zero_bytes(counts, 4 * sizeof(int64_t), s);
    if (r.n > 0) {
        k_task_count<<<grid_for(r.n, 256, 4096), 256, 0, s>>>(
            r.off, r.low, r.wpre, r.zbase, r.n, r.n_lower, r.tp.hash_max_work, r.tp.dense_chunk,
            counts);
        BT_CHECK_LAUNCH();
    }
    int64_t *hs = ws.host(4);
    BT_HIP(hipMemcpyAsync(hs, counts, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipMemcpyAsync(hs + 2, r.wpre + 2 * r.m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    t.n_hash = hs[0];
    t.n_dense = hs[1];
    if (t.n_hash >= INT32_MAX || t.n_dense >= INT32_MAX)
        throw Error{BT_EOVERFLOW, "too many wedge tasks"};
    r.wedges_po = hs[2];
    t.hash = ws.get<WedgeTask>("task_hash", t.n_hash);
    t.dense = ws.get<WedgeTask>("task_dense", t.n_dense);
    int32_t *cur = ws.get<int32_t>("task_cursor", 2);
    zero_bytes(cur, 2 * sizeof(int32_t), s);
    if (r.n > 0 && (t.n_hash + t.n_dense) > 0) {
        k_task_fill<<<grid_for(r.n, 256, 4096), 256, 0, s>>>(
            r.off, r.low, r.wpre, r.zbase, r.n, r.n_lower, r.tp.hash_max_work, r.tp.dense_chunk,
            t.hash, t.dense, cur);
        BT_CHECK_LAUNCH();
    }
}

}  // namespace bt

// ------------------------------------------------------ footprint

namespace bt {

namespace {

// sum over edges of min(d(u), d(v)): one wave per upper row.
__global__ __launch_bounds__(kBlock) void k_min_degree_sum(const int64_t *row_ptr,
                                                           const int32_t *col,
                                                           const int32_t *deg_lower,
                                                           int32_t n_upper,
                                                           unsigned long long *out) {
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    unsigned long long acc = 0;
    for (int64_t i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < n_upper;
         i += waves) {
        const int64_t a = row_ptr[i], b = row_ptr[i + 1];
        const int32_t du = (int32_t)(b - a);
        for (int64_t k = a + lane_id(); k < b; k += kWave) {
            const int32_t dl = deg_lower[col[k]];
            acc += (unsigned long long)(du < dl ? du : dl);
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(out, acc);
}

}  // namespace

int64_t footprint_bytes(const bt_csr &g, Workspace &ws, hipStream_t s) {
    const int32_t nu = g.n_upper, nl = g.n_lower;
    const int64_t m = g.m;
    int32_t *flags = ws.get<int32_t>("fp_flags", 4);
    int32_t *deg = ws.get<int32_t>("fp_deg", nl);
    unsigned long long *sum = ws.get<unsigned long long>("fp_sum", 1);
    zero_bytes(flags, 4 * sizeof(int32_t), s);
    if (nu > 0) {
        k_validate<<<grid_for((int64_t)nu * kWave, kBlock, 16384), kBlock, 0, s>>>(
            g.row_ptr, g.col, nu, nl, m, flags);
        BT_CHECK_LAUNCH();
    }
    int64_t *hs = ws.host(4);
    BT_HIP(hipMemcpyAsync(hs, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    if (*(int32_t *)hs != 0 || (nu == 0 && m != 0)) throw Error{BT_EINVAL, "malformed graph"};
    zero_bytes(deg, sizeof(int32_t) * (nl > 0 ? nl : 1), s);
    zero_bytes(sum, sizeof(unsigned long long), s);
    if (m > 0) {
        k_lower_degree<<<grid_for(m, 256, 16384), 256, 0, s>>>(g.col, m, deg);
        BT_CHECK_LAUNCH();
        k_min_degree_sum<<<grid_for((int64_t)nu * kWave, kBlock, 16384), kBlock, 0, s>>>(
            g.row_ptr, g.col, deg, nu, sum);
        BT_CHECK_LAUNCH();
    }
    BT_HIP(hipMemcpyAsync(hs, sum, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    const int64_t wbound = hs[0];  // priority-obeyed wedges <= this (Lemma 6)
    return 68 * wbound + 250 * m + 40 * ((int64_t)nu + nl) + (int64_t(1) << 20);
}

}  // namespace bt
