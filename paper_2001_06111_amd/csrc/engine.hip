// engine.hip - serving with continuous batching.
//
// Requests (device CSRs with caller-owned outputs) are queued with a
// device-memory estimate taken at submit time.  Each worker slot owns a HIP
// stream and a workspace; when a slot is free it picks a size class
// (below 2^14 edges, below 2^19, larger) and admits, in arrival order,
// queued requests of that class while the memory they may need fits the
// engine's budget, and decomposes them together as one disjoint union;
// large requests a few at a time.  A batch never mixes classes, so a small
// request never waits inside its batch for a larger graph's peel.  The
// smallest class present goes first unless the oldest request of a larger
// class has waited kLargeWaitS.  Requests that arrive while batches run are
// admitted by the next free slot: with two slots (the default) one slot
// counts and builds the index of its batch on the device while the other
// slot's batch peels, and one slot is kept for the small class.  Each
// result equals the plain single-graph decomposition of the request.
//
// Memory.  A slot's workspace is cached between its batches, so the budget
// covers what every slot holds plus what its running batch may still add:
//   held[i]  bytes slot i's workspace holds (updated by slot i itself),
//   res[i]   bytes its running batch may still allocate: the admission
//            estimate (the wedge bound of Lemma 6) at first, then, once the
//            batch's index is built, the exact peel state it still needs.
// A slot admits a batch of estimate E only if sum over slots of held + res,
// with its own res = E, stays within the budget; if its own cached
// workspace is what stands in the way it frees it first (the bytes count
// until they are freed) and decides again, and idle slots whose cached
// workspaces block an admission are asked to free theirs.
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "pipeline.h"

namespace bt {
namespace {

struct Request {
    bt_csr g;
    int64_t *sup;
    int64_t *phi;
    uint64_t id;
    int64_t bytes;
    std::chrono::steady_clock::time_point t;  // submit time
};

struct Done {
    uint64_t id;
    bt_status st;
};

// Size classes: a batch holds requests of one class.  A batch runs as many
// peel rounds as its slowest graph needs, so small graphs are not held up
// by medium ones in their own batch.
constexpr int64_t kLargeEdges = int64_t(1) << 19;
constexpr int64_t kMediumEdges = int64_t(1) << 14;
constexpr int kClasses = 3;
inline int size_class_of(int64_t m) { return m >= kLargeEdges ? 2 : m >= kMediumEdges ? 1 : 0; }
// Large requests share a batch too (one union, one shared level, so their
// rounds overlap: 2M-edge graphs take 2.18 s alone, 5.00 s four together,
// 8.27 s eight together), but at most this many, to bound each one's
// latency.
constexpr int32_t kLargePerBatch = 8;
// Batches of the smallest class present go first (they take a fraction of
// a larger class's time), unless the oldest request of a larger class has
// waited this long (so a steady stream of small requests cannot starve
// larger ones).
constexpr double kLargeWaitS = 10.0;
constexpr int kDefaultSlots = 2;
// Weights of a batch's turns on the device, by size class (each class's
// bound on its graphs' edges; the large one well above 8x the medium): a
// waiting batch of a smaller class makes a running peel of a larger class
// yield.
constexpr int64_t kClassTurnWeight[kClasses] = {int64_t(1) << 14, int64_t(1) << 19,
                                                int64_t(1) << 23};
// With two or more slots, one is always left for the small class: a slot
// starts a batch of a larger class only while fewer than slots - 1 other
// slots run one, so small requests never queue behind two long batches
// (their peels take the device from a running one of 8x their edges).

struct Slot {
    int64_t held = 0;      // workspace bytes (written by the slot's own thread)
    int64_t res = 0;       // bytes its running batch may still add
    int cls = -1;          // size class of the running batch (-1: idle)
    bool busy = false;
    bool release = false;  // asked to free its cached workspace while idle
};

// An admitted batch: its requests, their estimates, the slot's holdings at
// admission and the batch's size class.
struct Batch {
    std::vector<Request> reqs;
    int64_t bytes = 0;
    int64_t held0 = 0;
    int cls = 0;
};

}  // namespace
}  // namespace bt

using namespace bt;

struct bt_engine {
    int64_t budget = 0;
    int32_t max_batch = 1024;
    std::mutex mu;
    std::condition_variable cv_work, cv_idle;
    std::deque<Request> queue;
    std::vector<Done> done;
    std::vector<Slot> slots;
    int64_t running = 0;  // requests now running
    bool stop = false;
    std::vector<std::thread> workers;
    // submit-time estimates run on their own stream and workspace
    std::mutex est_mu;
    Workspace est_ws;
    hipStream_t est_stream = nullptr;
    int device = 0;
    int64_t batches = 0, admitted = 0;
    int64_t peel_yields = 0;  // peel launches of large batches that gave way
    // BT_ENGINE_VERBOSE=1: one line per batch admitted and done, with times
    // since the engine was created.
    bool verbose = std::getenv("BT_ENGINE_VERBOSE") != nullptr;
    std::chrono::steady_clock::time_point t_created = std::chrono::steady_clock::now();
    double ms_since_created() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                         t_created)
            .count();
    }
    int64_t peak_committed = 0;  // largest sum of held + res seen
    int64_t peak_held = 0;       // largest sum of held seen
    // Caller-driven engine (created with slots = -1): no worker threads;
    // bt_engine_step runs one batch of its single slot on the caller's
    // thread, on this stream and workspace.
    bool manual = false;
    std::mutex step_mu;  // one step at a time
    hipStream_t manual_stream = nullptr;
    Workspace manual_ws;

    void worker_loop(int slot);
    bool take_batch(int slot, std::unique_lock<std::mutex> &lk, bool block, Batch &b,
                    Workspace &ws);
    void run_batch(int slot, const Batch &b, Workspace &ws, hipStream_t s);
    int pick_class(bool larger_ok) const;
    const Request *first_of(int cls) const;
    int64_t committed_except(int s) const;
    void note_peaks();
};

const Request *bt_engine::first_of(int cls) const {
    for (const Request &r : queue)
        if (size_class_of(r.g.m) == cls) return &r;
    return nullptr;
}

// The class of the next batch (call with mu held and the queue non-empty):
// the largest class whose oldest request has waited kLargeWaitS, else the
// smallest class present.
// The class of the next batch, or -1 when no queued request may start now
// (larger_ok false: only the small class may).
int bt_engine::pick_class(bool larger_ok) const {
    if (!larger_ok) return first_of(0) ? 0 : -1;
    const auto now = std::chrono::steady_clock::now();
    for (int c = kClasses - 1; c > 0; --c) {
        const Request *r = first_of(c);
        if (r && std::chrono::duration<double>(now - r->t).count() >= kLargeWaitS) return c;
    }
    for (int c = 0; c < kClasses; ++c)
        if (first_of(c)) return c;
    return -1;
}

int64_t bt_engine::committed_except(int s) const {
    int64_t t = 0;
    for (size_t i = 0; i < slots.size(); ++i)
        if ((int)i != s) t += slots[i].held + slots[i].res;
    return t;
}

void bt_engine::note_peaks() {
    int64_t c = 0, h = 0;
    for (const Slot &sl : slots) {
        c += sl.held + sl.res;
        h += sl.held;
    }
    peak_committed = std::max(peak_committed, c);
    peak_held = std::max(peak_held, h);
}

// Under mu: admits the next batch for `slot` into b.  With block, waits
// until a batch can start (false only when the engine stops); without,
// returns false when none can start now.
bool bt_engine::take_batch(int slot, std::unique_lock<std::mutex> &lk, bool block, Batch &b,
                           Workspace &ws) {
    Slot &me = slots[(size_t)slot];
    while (true) {
        int cls = 0;
        const auto ready = [&] {
            if (stop) return true;
            if (me.release) return true;
            if (queue.empty()) return false;
            int larger = 0;  // other slots running a batch of a larger class
            for (size_t i = 0; i < slots.size(); ++i)
                if ((int)i != slot && slots[i].busy && slots[i].cls > 0) ++larger;
            cls = pick_class(slots.size() < 2 || larger < (int)slots.size() - 1);
            if (cls < 0) return false;
            const int64_t need = first_of(cls)->bytes;
            const int64_t others = committed_except(slot);
            if (others + need <= budget) return true;
            // Idle slots whose cached workspaces stand in the way free them
            // (woken only when a request to free is new, so idle slots do
            // not wake each other in turn).
            bool asked = false;
            for (size_t i = 0; i < slots.size(); ++i)
                if ((int)i != slot && !slots[i].busy && slots[i].held > 0 && !slots[i].release) {
                    slots[i].release = true;
                    asked = true;
                }
            if (asked) cv_work.notify_all();
            return false;
        };
        if (block)
            cv_work.wait(lk, ready);
        else if (!ready())
            return false;
        if (stop) return false;  // destroy drains the queue before it stops workers
        if (me.release) {  // idle and asked to free its cached workspace
            me.release = false;
            if (me.held > 0) {
                lk.unlock();
                ws.release();
                lk.lock();
                me.held = 0;
                note_peaks();
                cv_work.notify_all();
            }
            continue;
        }
        // If this slot's own cached workspace is what keeps the oldest
        // request of the class out, free it first (its bytes stay counted
        // until it is freed), then decide again.
        const int64_t others = committed_except(slot);
        if (me.held > 0 && others + me.held + first_of(cls)->bytes > budget) {
            lk.unlock();
            ws.release();
            lk.lock();
            me.held = 0;
            note_peaks();
            cv_work.notify_all();
            continue;
        }
        // Admit requests of the chosen class in arrival order while the
        // budget, this slot's cache included, allows.
        const int32_t cap = cls == 2 ? std::min(max_batch, kLargePerBatch) : max_batch;
        b = Batch{};
        for (auto it = queue.begin(); it != queue.end() && (int32_t)b.reqs.size() < cap;) {
            if (size_class_of(it->g.m) != cls) {
                ++it;
                continue;
            }
            if (others + me.held + b.bytes + it->bytes > budget) break;
            b.bytes += it->bytes;
            b.reqs.push_back(*it);
            it = queue.erase(it);
        }
        b.held0 = me.held;
        b.cls = cls;
        me.res = b.bytes;
        me.busy = true;
        me.cls = cls;
        running += (int64_t)b.reqs.size();
        batches += 1;
        admitted += (int64_t)b.reqs.size();
        note_peaks();
        if (verbose) {
            int64_t edges = 0;
            for (auto &r : b.reqs) edges += r.g.m;
            std::fprintf(stderr, "[engine] %.1f ms slot %d admits %zu requests of class %d, %lld edges (queue %zu)\n",
                         ms_since_created(), slot, b.reqs.size(), cls, (long long)edges,
                         queue.size());
        }
        return true;
    }
}

// Decomposes an admitted batch on the slot's stream and workspace (without
// mu) and reports its requests as done.
void bt_engine::run_batch(int slot, const Batch &b, Workspace &ws, hipStream_t s) {
    std::vector<bt_csr> gs;
    std::vector<int64_t *> sups, phis;
    for (auto &r : b.reqs) {
        gs.push_back(r.g);
        sups.push_back(r.sup);
        phis.push_back(r.phi);
    }
    // Once the index is built the peel's remaining need replaces what is
    // left of the estimate, so other slots may admit against the
    // difference.  The slot's commitment never grows past its admission
    // (held0 + estimate); its real holdings are re-read at the end.
    const SizedHook on_sized = [&](int64_t held, int64_t peel_bytes) {
        std::lock_guard<std::mutex> lk(mu);
        Slot &me = slots[(size_t)slot];
        me.held = held;
        me.res = std::max<int64_t>(0, std::min(peel_bytes, b.held0 + b.bytes - held));
        note_peaks();
        cv_work.notify_all();
    };
    std::vector<Done> out;
    bt_stats bst{};
    set_turn_weight(kClassTurnWeight[b.cls]);
    try {
        decompose_batch_impl(gs.data(), (int32_t)gs.size(), sups.data(), phis.data(), &bst, ws,
                             s, &on_sized);
        for (auto &r : b.reqs) out.push_back(Done{r.id, BT_OK});
    } catch (const Error &) {
        // Isolate the failure: run the requests of the batch one by one.
        for (auto &r : b.reqs) {
            bt_status st = BT_OK;
            try {
                bt_csr g = r.g;
                int64_t *sp = r.sup, *pp = r.phi;
                decompose_batch_impl(&g, 1, &sp, &pp, nullptr, ws, s);
            } catch (const Error &e) {
                st = e.status;
            } catch (...) {
                st = BT_EDEVICE;
            }
            out.push_back(Done{r.id, st});
        }
    } catch (...) {
        for (auto &r : b.reqs) out.push_back(Done{r.id, BT_EDEVICE});
    }
    set_turn_weight(-1);
    const int64_t held_now = (int64_t)ws.bytes();
    {
        std::lock_guard<std::mutex> lk(mu);
        Slot &me = slots[(size_t)slot];
        me.held = held_now;
        me.res = 0;
        me.busy = false;
        me.cls = -1;
        note_peaks();
        peel_yields += bst.peel_yields;
        if (verbose)
            std::fprintf(stderr, "[engine] %.1f ms slot %d done (%zu requests, %lld peel yields)\n",
                         ms_since_created(), slot, b.reqs.size(), (long long)bst.peel_yields);
        running -= (int64_t)b.reqs.size();
        for (auto &d : out) done.push_back(d);
    }
    cv_work.notify_all();
    cv_idle.notify_all();
}

void bt_engine::worker_loop(int slot) {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    Workspace ws;  // cooperative peels of different slots take turns (see peel.hip)
    ws.bind_stream(s);
    while (true) {
        Batch b;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!take_batch(slot, lk, true, b, ws)) break;
        }
        run_batch(slot, b, ws, s);
    }
    ws.close();
    if (s) (void)hipStreamDestroy(s);
}

extern "C" {

bt_status bt_engine_create(int64_t hbm_budget, int32_t slots, int32_t max_batch,
                           bt_engine **out) {
    if (!out || slots < -1 || max_batch < 0) {
        set_error("invalid engine arguments");
        return BT_EINVAL;
    }
    *out = nullptr;
    bt_engine *E = new bt_engine();
    try {
        BT_HIP(hipGetDevice(&E->device));
        if (hbm_budget <= 0) {
            size_t fr = 0, tot = 0;
            BT_HIP(hipMemGetInfo(&fr, &tot));
            hbm_budget = (int64_t)(fr / 2);
        }
        E->budget = hbm_budget;
        E->max_batch = max_batch > 0 ? max_batch : 1024;
        BT_HIP(hipStreamCreateWithFlags(&E->est_stream, hipStreamNonBlocking));
        E->est_ws.coop = false;
        E->est_ws.bind_stream(E->est_stream);
        if (slots == -1) {
            E->manual = true;
            BT_HIP(hipStreamCreateWithFlags(&E->manual_stream, hipStreamNonBlocking));
            E->manual_ws.bind_stream(E->manual_stream);
            E->slots.resize(1);
        } else {
            const int n = slots > 0 ? slots : kDefaultSlots;
            E->slots.resize((size_t)n);
            for (int i = 0; i < n; ++i) E->workers.emplace_back(&bt_engine::worker_loop, E, i);
        }
    } catch (const Error &e) {
        set_error(e.msg);
        delete E;
        return e.status;
    }
    *out = E;
    return BT_OK;
}

bt_status bt_engine_submit(bt_engine *E, const bt_csr *g, int64_t *sup_out, int64_t *phi_out,
                           uint64_t id) {
    if (!E) {
        set_error("engine is NULL");
        return BT_EINVAL;
    }
    Request r{};
    try {
        check_graph(g);
        if (g->m > 0 && !phi_out) throw Error{BT_EINVAL, "phi_out is NULL"};
        std::lock_guard<std::mutex> lk(E->est_mu);
        r.bytes = footprint_bytes(*g, E->est_ws, E->est_stream);
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    }
    if (r.bytes > E->budget) {
        set_error("request needs about " + std::to_string(r.bytes) +
                  " bytes, more than the engine budget");
        return BT_EBUSY;
    }
    r.g = *g;
    r.sup = sup_out;
    r.phi = phi_out;
    r.id = id;
    r.t = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->queue.push_back(r);
    }
    E->cv_work.notify_all();
    return BT_OK;
}

bt_status bt_engine_poll(bt_engine *E, uint64_t *ids, int32_t *status, int32_t cap,
                         int32_t *n_done) {
    if (!E || !n_done || (cap > 0 && (!ids || !status))) {
        set_error("invalid poll arguments");
        return BT_EINVAL;
    }
    std::lock_guard<std::mutex> lk(E->mu);
    const int32_t n = std::min<int32_t>(cap, (int32_t)E->done.size());
    for (int32_t i = 0; i < n; ++i) {
        ids[i] = E->done[i].id;
        status[i] = E->done[i].st;
    }
    E->done.erase(E->done.begin(), E->done.begin() + n);
    *n_done = n;
    return BT_OK;
}

bt_status bt_engine_step(bt_engine *E, int32_t *n_done) {
    if (!E) {
        set_error("engine is NULL");
        return BT_EINVAL;
    }
    if (!E->manual) {
        set_error("bt_engine_step needs an engine created with slots = -1 (this one runs "
                  "its own worker threads)");
        return BT_EINVAL;
    }
    std::lock_guard<std::mutex> step(E->step_mu);
    Batch b;
    {
        std::unique_lock<std::mutex> lk(E->mu);
        if (!E->take_batch(0, lk, false, b, E->manual_ws)) {
            if (n_done) *n_done = 0;
            return BT_OK;
        }
    }
    // The batch runs on the engine's device; the caller's current device is
    // restored afterwards.
    int prev = E->device;
    (void)hipGetDevice(&prev);
    if (prev != E->device) (void)hipSetDevice(E->device);
    E->run_batch(0, b, E->manual_ws, E->manual_stream);
    if (prev != E->device) (void)hipSetDevice(prev);
    if (n_done) *n_done = (int32_t)b.reqs.size();
    return BT_OK;
}

bt_status bt_engine_drain(bt_engine *E) {
    if (!E) {
        set_error("engine is NULL");
        return BT_EINVAL;
    }
    if (E->manual) {
        // Steps on the caller's thread until nothing is queued.
        while (true) {
            int32_t n = 0;
            const bt_status st = bt_engine_step(E, &n);
            if (st != BT_OK) return st;
            if (n == 0) {
                std::lock_guard<std::mutex> lk(E->mu);
                if (E->queue.empty()) return BT_OK;
                set_error("a queued request cannot be admitted");  // not reached: submit bounds them
                return BT_EDEVICE;
            }
        }
    }
    std::unique_lock<std::mutex> lk(E->mu);
    E->cv_idle.wait(lk, [&] { return E->queue.empty() && E->running == 0; });
    return BT_OK;
}

bt_status bt_engine_stats(bt_engine *E, int64_t *batches, int64_t *admitted, int64_t *queued,
                          int64_t *peel_yields) {
    if (!E) {
        set_error("engine is NULL");
        return BT_EINVAL;
    }
    std::lock_guard<std::mutex> lk(E->mu);
    if (batches) *batches = E->batches;
    if (admitted) *admitted = E->admitted;
    if (queued) *queued = (int64_t)E->queue.size();
    if (peel_yields) *peel_yields = E->peel_yields;
    return BT_OK;
}

bt_status bt_engine_memory(bt_engine *E, int64_t *budget, int64_t *held, int64_t *peak_held,
                           int64_t *peak_committed) {
    if (!E) {
        set_error("engine is NULL");
        return BT_EINVAL;
    }
    std::lock_guard<std::mutex> lk(E->mu);
    int64_t h = 0;
    for (const Slot &sl : E->slots) h += sl.held;
    if (budget) *budget = E->budget;
    if (held) *held = h;
    if (peak_held) *peak_held = E->peak_held;
    if (peak_committed) *peak_committed = E->peak_committed;
    return BT_OK;
}

void bt_engine_destroy(bt_engine *E) {
    if (!E) return;
    bt_engine_drain(E);
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->stop = true;
    }
    E->cv_work.notify_all();
    for (auto &t : E->workers) t.join();
    E->manual_ws.close();
    if (E->manual_stream) (void)hipStreamDestroy(E->manual_stream);
    E->est_ws.close();
    if (E->est_stream) (void)hipStreamDestroy(E->est_stream);
    delete E;
}

}  // extern "C"
