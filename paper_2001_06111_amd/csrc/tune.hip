// tune.hip - the autotuner: launch parameters per kind of call and size
// class, measured on the device and kept in a process-wide table that can
// be saved to and loaded from a text file.
//
// The parameters (TuneParams) only change how work is cut into tasks and
// how many workgroups run: every result is the same under all of them.
// A graph of m edges falls in size class bit_length(m) - 10 (clamped to
// [0, kClasses)); a call uses the entry of its own class, else the nearest
// tuned class of the same kind, else the defaults.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "pipeline.h"

namespace bt {

namespace {

constexpr int kClasses = 22;

struct Table {
    std::mutex mu;
    TuneParams p[2][kClasses];
    bool set[2][kClasses] = {};
    bool env_done = false;
};

Table &table() {
    static Table *t = new Table();  // never destroyed: outlives static teardown
    return *t;
}

int size_class(int64_t m) {
    int b = 0;
    while (b < 62 && (int64_t(1) << b) <= m) ++b;
    return std::max(0, std::min(kClasses - 1, b - 10));
}

// Architecture name of the current device, or "unknown" without one.
std::string device_arch() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return "unknown";
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

void load_locked(Table &t, const char *path, bool missing_ok) {
    FILE *f = std::fopen(path, "r");
    if (!f) {
        if (missing_ok) return;
        throw Error{BT_EINVAL, std::string("cannot open tuning file ") + path};
    }
    struct Closer {
        FILE *f;
        ~Closer() { std::fclose(f); }
    } closer{f};
    char arch[64] = {};
    int version = 0;
    if (std::fscanf(f, " bt-tune %d %63s", &version, arch) != 2 || version != 1)
        throw Error{BT_EINVAL, std::string("not a tuning file: ") + path};
    const std::string here = device_arch();
    if (here != "unknown" && std::strcmp(arch, "unknown") != 0 && here != arch)
        throw Error{BT_EINVAL, std::string("tuning file is for ") + arch + ", device is " + here};
    // Entries are checked before any is stored: a bad file changes nothing.
    struct Row {
        int kind, cls;
        TuneParams p;
    };
    std::vector<Row> rows;
    char kind[16];
    int cls;
    TuneParams p;
    int got;
    while ((got = std::fscanf(f, " %15s %d %d %d %d %d %d", kind, &cls, &p.hash_max_work,
                              &p.dense_chunk, &p.wedge_wg_per_cu, &p.peel_blocks,
                              &p.active_min)) == 7) {
        const bool batch = std::strcmp(kind, "batch") == 0;
        if ((!batch && std::strcmp(kind, "single") != 0) || cls < 0 || cls >= kClasses ||
            !tune_valid(p))
            throw Error{BT_EINVAL, std::string("bad entry in tuning file ") + path};
        rows.push_back(Row{batch ? 1 : 0, cls, p});
    }
    if (got != EOF) throw Error{BT_EINVAL, std::string("malformed tuning file ") + path};
    for (const Row &r : rows) {
        t.p[r.kind][r.cls] = r.p;
        t.set[r.kind][r.cls] = true;
    }
}

// BT_TUNE_CACHE names a tuning file read at the first lookup (if present).
void env_once_locked(Table &t) {
    if (t.env_done) return;
    t.env_done = true;
    if (const char *f = std::getenv("BT_TUNE_CACHE")) load_locked(t, f, true);
}

}  // namespace

bool tune_valid(const TuneParams &p) {
    return p.hash_max_work >= 1 && p.hash_max_work <= kHashMaxWorkLimit &&
           p.dense_chunk >= 64 && p.dense_chunk <= kDenseChunkLimit && p.wedge_wg_per_cu >= 1 &&
           p.wedge_wg_per_cu <= 16 && p.peel_blocks >= 0 && p.peel_blocks <= 65536 &&
           p.active_min >= 1;
}

int peel_grid(const TuneParams &p, int cus, int resident) {
    const int want = p.peel_blocks > 0 ? p.peel_blocks : std::max(1, 3 * cus / 4);
    return std::max(1, std::min(want, resident));
}

TuneParams tune_params(bool batch, int64_t m) {
    Table &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    env_once_locked(t);
    const int k = batch ? 1 : 0, c = size_class(m);
    for (int d = 0; d < kClasses; ++d) {
        if (c - d >= 0 && t.set[k][c - d]) return t.p[k][c - d];
        if (c + d < kClasses && t.set[k][c + d]) return t.p[k][c + d];
    }
    return TuneParams{};
}

void tune_store(bool batch, int64_t m, const TuneParams &p) {
    if (!tune_valid(p)) throw Error{BT_EINVAL, "launch parameters out of range"};
    Table &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    env_once_locked(t);
    const int k = batch ? 1 : 0, c = size_class(m);
    t.p[k][c] = p;
    t.set[k][c] = true;
}

void tune_clear() {
    Table &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    env_once_locked(t);
    for (auto &row : t.set)
        for (bool &b : row) b = false;
}

void tune_save(const char *path) {
    Table &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    env_once_locked(t);
    const std::string arch = device_arch();
    FILE *f = std::fopen(path, "w");
    if (!f) throw Error{BT_EINVAL, std::string("cannot write tuning file ") + path};
    std::fprintf(f, "bt-tune 1 %s\n", arch.c_str());
    for (int k = 0; k < 2; ++k)
        for (int c = 0; c < kClasses; ++c)
            if (t.set[k][c]) {
                const TuneParams &p = t.p[k][c];
                std::fprintf(f, "%s %d %d %d %d %d %d\n", k ? "batch" : "single", c,
                             p.hash_max_work, p.dense_chunk, p.wedge_wg_per_cu, p.peel_blocks,
                             p.active_min);
            }
    if (std::fclose(f) != 0) throw Error{BT_EINVAL, std::string("cannot write ") + path};
}

void tune_load(const char *path) {
    Table &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    env_once_locked(t);
    load_locked(t, path, false);
}

// Coordinate search: each parameter in turn takes the candidate value with
// the shortest device time, the others held; a change must gain 2% over the
// current value.  Index parameters are timed on the index build, peel
// parameters on the peel kernel; a batch is timed as a whole.
TuneParams autotune(const bt_csr *gs, int32_t n, uint32_t what, Workspace &ws, hipStream_t s) {
    const bool batch = n > 1;
    int64_t mt = 0;
    for (int32_t i = 0; i < n; ++i) mt += gs[i].m;
    Table &t = table();
    // The class's entry is put back if the search stops on an error.
    bool had;
    TuneParams old;
    {
        std::lock_guard<std::mutex> lk(t.mu);
        env_once_locked(t);
        had = t.set[batch ? 1 : 0][size_class(mt)];
        old = t.p[batch ? 1 : 0][size_class(mt)];
    }
    struct Restore {
        Table &t;
        int k, c;
        bool had, armed = true;
        TuneParams old;
        ~Restore() {
            if (!armed) return;
            std::lock_guard<std::mutex> lk(t.mu);
            t.p[k][c] = old;
            t.set[k][c] = had;
        }
    } restore{t, batch ? 1 : 0, size_class(mt), had, true, old};

    std::vector<int64_t *> phis((size_t)n, nullptr);
    struct Free {
        std::vector<int64_t *> &v;
        ~Free() {
            for (int64_t *p : v)
                if (p) device_free(p);
        }
    } free_phis{phis};
    for (int32_t i = 0; i < n; ++i)
        phis[(size_t)i] = (int64_t *)device_alloc(sizeof(int64_t) * std::max<int64_t>(1, gs[i].m));
    hipEvent_t e0, e1;
    BT_HIP(hipEventCreate(&e0));
    BT_HIP(hipEventCreate(&e1));
    struct EvFree {
        hipEvent_t a, b;
        ~EvFree() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev_free{e0, e1};

    auto run = [&](const TuneParams &p, bool peel) -> float {
        tune_store(batch, mt, p);
        if (batch) {
            BT_HIP(hipEventRecord(e0, s));
            decompose_batch_impl(gs, n, nullptr, phis.data(), nullptr, ws, s);
            BT_HIP(hipEventRecord(e1, s));
            BT_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            BT_HIP(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        }
        if (!peel) return index_build_ms(gs[0], ws, s);
        bt_stats st;
        decompose_impl(gs[0], nullptr, phis[0], &st, ws, s);
        return st.ms_peel_kernel;
    };

    int dev = 0, cus = 0;
    BT_HIP(hipGetDevice(&dev));
    BT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    struct Knob {
        int32_t TuneParams::*f;
        std::vector<int32_t> vals;
        bool peel;
    };
    std::vector<Knob> knobs;
    if (what & BT_TUNE_INDEX) {
        knobs.push_back({&TuneParams::hash_max_work, {512, 1024, 2048}, false});
        knobs.push_back({&TuneParams::dense_chunk, {2048, 4096, 6144}, false});
        knobs.push_back({&TuneParams::wedge_wg_per_cu, {1, 2}, false});
    }
    if (what & BT_TUNE_PEEL) {
        knobs.push_back({&TuneParams::peel_blocks, {cus / 2, 0, cus}, true});
        knobs.push_back({&TuneParams::active_min, {4096, 16384, 65536}, true});
    }
    static const char *const names[] = {"hash_max_work", "dense_chunk", "wedge_wg_per_cu",
                                        "peel_blocks", "active_min"};
    auto name_of = [&](int32_t TuneParams::*f) {
        if (f == &TuneParams::hash_max_work) return names[0];
        if (f == &TuneParams::dense_chunk) return names[1];
        if (f == &TuneParams::wedge_wg_per_cu) return names[2];
        if (f == &TuneParams::peel_blocks) return names[3];
        return names[4];
    };
    const bool verbose = std::getenv("BT_TUNE_VERBOSE") != nullptr;
    TuneParams cur = tune_params(batch, mt);
    if (!knobs.empty()) (void)run(cur, knobs[0].peel);  // warm-up: workspace, code, caches
    for (const Knob &k : knobs) {
        const int reps = (batch || k.peel) ? 1 : 3;
        auto timed = [&](int32_t v) {
            TuneParams p = cur;
            p.*(k.f) = v;
            float best = 1e30f;
            for (int r = 0; r < reps; ++r) best = std::min(best, run(p, k.peel));
            return best;
        };
        const int32_t v0 = cur.*(k.f);
        const float t0 = timed(v0);
        int32_t bv = v0;
        float bt = t0;
        for (int32_t v : k.vals) {
            if (v == v0 || v < 0) continue;
            const float tv = timed(v);
            if (verbose)
                std::fprintf(stderr, "[tune] %s m=%lld %s=%d: %.3f ms (current %d: %.3f ms)\n",
                             batch ? "batch" : "single", (long long)mt, name_of(k.f), v, tv, v0,
                             t0);
            if (tv < bt) {
                bv = v;
                bt = tv;
            }
        }
        if (bv != v0 && bt < 0.98f * t0) cur.*(k.f) = bv;
    }
    tune_store(batch, mt, cur);
    restore.armed = false;
    return cur;
}

}  // namespace bt
