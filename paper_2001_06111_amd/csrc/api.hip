// api.hip - the C ABI: argument checks, workspace, stage orchestration.
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
    ix.link = (uint2 *)get("ix_link", sizeof(uint2) * (2 * ix.cap_w + 1));
    ix.cursor = (uint64_t *)get("ix_cursor", sizeof(uint64_t) * 2);
    ix.butterflies = (int64_t *)(ix.cursor + 1);
}

int64_t index_bytes(const IndexArrays &ix, int64_t m) {
    return (int64_t)(sizeof(uint32_t) + 2 * sizeof(int32_t)) * (ix.n_b + 1) +
           (int64_t)(3 * sizeof(int32_t) + 2 * sizeof(uint2)) * ix.n_w +
           (int64_t)(sizeof(uint64_t) + sizeof(int64_t) + sizeof(int32_t) * 2) * m +
           (ix.n_w + 31) / 32 * 4;
}

// prepare -> tasks -> counting + emission + links.  Reads back the sizes.
void build_all(const bt_csr &g, RankCSR &r, IndexArrays &ix, bool owned,
               std::vector<void *> *own, Workspace &ws, hipStream_t s, Events *ev) {
    prepare(g, r, ws, s);
    TaskLists t;
    make_tasks(r, t, ws, s);
    if (ev) ev->mark(1);
    alloc_index(r, ix, owned, ws, own);
    BT_HIP(hipMemsetAsync(ix.supl, 0, sizeof(uint64_t) * (r.m + 1), s));
    BT_HIP(hipMemsetAsync(ix.cursor, 0, sizeof(uint64_t) * 2, s));
    build_index(r, t, ix, ws, s);
    if (ev) ev->mark(2);
    int64_t *hs = host_scalars(4);
    BT_HIP(hipMemcpyAsync(hs, ix.cursor, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BT_HIP(hipStreamSynchronize(s));
    const uint64_t c = (uint64_t)hs[0];
    ix.n_b = (int64_t)(c >> 32);
    ix.n_w = (int64_t)(c & 0xffffffffu);
}

}  // namespace

}  // namespace bt

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
        BT_HIP(hipMemsetAsync(supl, 0, sizeof(uint64_t) * (g->m + 1), stream));
        BT_HIP(hipMemsetAsync(bf, 0, sizeof(int64_t) * 2, stream));
        count_support(r, t, supl, bf, stream);
        supl_to_sup(supl, sup_out, g->m, stream);
        int64_t *hs = host_scalars(2);
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
            int64_t *hs = host_scalars(2);
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
            std::vector<uint2> t(2 * ix.n_w);
            BT_HIP(hipMemcpy(t.data(), ix.link, sizeof(uint2) * t.size(),
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
        Workspace &ws = lib().ws;
        Events ev(stats != nullptr, stream);
        ev.mark(0);
        RankCSR r;
        IndexArrays ix;
        build_all(*g, r, ix, false, nullptr, ws, stream, &ev);
        ev.mark(3);
        PeelCounters pc;
        peel(r, ix, sup_out, phi_out, pc, ws, stream);
        ev.mark(4);
        if (stats) {
            int64_t *hs = host_scalars(2);
            BT_HIP(hipMemcpyAsync(hs, ix.butterflies, sizeof(int64_t), hipMemcpyDeviceToHost,
                                  stream));
            BT_HIP(hipStreamSynchronize(stream));
            std::memset(stats, 0, sizeof *stats);
            stats->butterflies = hs[0];
            stats->wedges_po = r.wedges_po;
            stats->blooms = ix.n_b;
            stats->bloom_wedges = ix.n_w;
            stats->index_bytes = index_bytes(ix, g->m);
            stats->levels = pc.levels;
            stats->rounds = pc.rounds;
            stats->max_phi = pc.max_phi;
            stats->support_updates = pc.updates;
            stats->bloom_visits = pc.bloom_visits;
            stats->ms_prepare = ev.ms(0, 1);
            stats->ms_count = ev.ms(1, 2);
            stats->ms_link = ev.ms(2, 3);
            stats->ms_peel = ev.ms(3, 4);
        } else {
            BT_HIP(hipStreamSynchronize(stream));
        }
    });
}

bt_status bt_decompose_batch(const bt_csr *gs, int32_t n_graphs, int64_t *const *sup_out,
                             int64_t *const *phi_out, bt_stats *stats, hipStream_t stream) {
    if (n_graphs < 0 || (n_graphs > 0 && (!gs || !phi_out))) {
        set_error("invalid batch arguments");
        return BT_EINVAL;
    }
    bt_stats total;
    std::memset(&total, 0, sizeof total);
    for (int32_t i = 0; i < n_graphs; ++i) {
        bt_stats st;
        bt_status rc = bt_decompose(&gs[i], sup_out ? sup_out[i] : nullptr, phi_out[i],
                                    stats ? &st : nullptr, stream);
        if (rc != BT_OK) return rc;
        if (stats) {
            total.butterflies += st.butterflies;
            total.wedges_po += st.wedges_po;
            total.blooms += st.blooms;
            total.bloom_wedges += st.bloom_wedges;
            total.index_bytes += st.index_bytes;
            total.levels = std::max(total.levels, st.levels);
            total.rounds = std::max(total.rounds, st.rounds);
            total.max_phi = std::max(total.max_phi, st.max_phi);
            total.support_updates += st.support_updates;
            total.bloom_visits += st.bloom_visits;
            total.ms_prepare += st.ms_prepare;
            total.ms_count += st.ms_count;
            total.ms_link += st.ms_link;
            total.ms_peel += st.ms_peel;
        }
    }
    if (stats) *stats = total;
    return BT_OK;
}

}  // extern "C"
