// prims.hip - device-wide scans, stable radix sort, fills, workspace, the
// device-memory allocator hook.

#include <mutex>
#include <unordered_map>

#include "common.h"

namespace bt {

// ------------------------------------------------------------ errors

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace bt

extern "C" const char *bt_last_error(void) { return bt::g_last_error.c_str(); }

namespace bt {

// --------------------------------------------------------- memory
// Every device buffer of the library comes from device_alloc: hipMalloc, or
// the caller's hook (bt_set_allocator).  Each live block remembers the hook
// that made it, so a block is always returned to its own allocator even if
// the hook changes meanwhile.

namespace {
struct Hook {
    bt_alloc_fn alloc = nullptr;
    bt_free_fn free = nullptr;
    void *ctx = nullptr;
};
struct Block {
    Hook hook;
    size_t bytes;
    hipStream_t stream;  // stream-ordered block (nullptr: device-wide)
};
std::mutex &alloc_mu() {
    static std::mutex *m = new std::mutex();  // never destroyed: outlives static teardown
    return *m;
}
Hook g_hook;
std::unordered_map<void *, Block> &live_blocks() {
    static auto *m = new std::unordered_map<void *, Block>();
    return *m;
}
}  // namespace

void set_allocator(bt_alloc_fn a, bt_free_fn f, void *ctx) {
    if ((a == nullptr) != (f == nullptr))
        throw Error{BT_EINVAL, "bt_set_allocator needs both functions or neither"};
    std::lock_guard<std::mutex> lk(alloc_mu());
    g_hook = Hook{a, f, ctx};
}

void *device_alloc(size_t bytes, hipStream_t stream) {
    void *p = nullptr;
    if (bytes == 0) bytes = 256;
    Hook h;
    {
        std::lock_guard<std::mutex> lk(alloc_mu());
        h = g_hook;
    }
    if (h.alloc) {
        p = h.alloc(bytes, h.ctx);
        if (!p)
            throw Error{BT_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                       " bytes failed (allocator hook returned NULL)"};
    } else {
        hipError_t e = stream ? hipMallocAsync(&p, bytes, stream) : hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error{BT_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                       " bytes failed: " + hipGetErrorString(e)};
        }
    }
    std::lock_guard<std::mutex> lk(alloc_mu());
    live_blocks()[p] = Block{h, bytes, stream};
    return p;
}

void device_free(void *p) {
    if (!p) return;
    Block b{};
    {
        std::lock_guard<std::mutex> lk(alloc_mu());
        auto it = live_blocks().find(p);
        if (it != live_blocks().end()) {
            b = it->second;
            live_blocks().erase(it);
        }
    }
    if (b.hook.free) {
        // A hook may hand the block out again at once (a caching allocator),
        // so no kernel of the library may still use it.
        if (b.stream)
            (void)hipStreamSynchronize(b.stream);
        else
            (void)hipDeviceSynchronize();
        b.hook.free(p, b.bytes, b.hook.ctx);
    } else if (b.stream) {
        (void)hipFreeAsync(p, b.stream);
    } else {
        (void)hipFree(p);
    }
}

Workspace::~Workspace() { close(); }

void Workspace::close() {
    release();
    if (!stream_) return;
    (void)hipStreamSynchronize(stream_);
    for (int64_t *h : old_host_) (void)hipHostFree(h);
    old_host_.clear();
    if (host_) (void)hipHostFree(host_);
    host_ = nullptr;
    host_cap_ = 0;
    stream_ = nullptr;
}

void Workspace::use_arena(void *base, size_t cap, int64_t *host, int n_host) {
    release();
    arena_ = static_cast<char *>(base);
    arena_cap_ = cap;
    arena_top_ = 0;
    host_ = host;
    host_cap_ = n_host;
}

void *Workspace::get(const char *name, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (arena_) {
        // Bump allocation; a name asked again for more memory gets a new
        // region (the old one is reclaimed only by release()).
        for (auto &b : bufs_)
            if (b.name == name && b.cap >= bytes) return b.ptr;
        if (arena_top_ + bytes > arena_cap_)
            throw Error{BT_ENOMEM, "the call needs more than the " + std::to_string(arena_cap_) +
                                       "-byte static scratch (" + std::string(name) + ")"};
        Buf nb;
        nb.name = name;
        nb.ptr = arena_ + arena_top_;
        nb.cap = bytes;
        arena_top_ += bytes;
        for (auto &b : bufs_)
            if (b.name == name) {
                b = nb;
                return nb.ptr;
            }
        bufs_.push_back(nb);
        return nb.ptr;
    }
    for (auto &b : bufs_) {
        if (b.name == name) {
            if (b.cap < bytes) {
                device_free(b.ptr);
                b.ptr = nullptr;
                b.cap = 0;
                b.ptr = device_alloc(bytes + bytes / 8, stream_);
                b.cap = bytes + bytes / 8;
            }
            return b.ptr;
        }
    }
    Buf nb;
    nb.name = name;
    nb.ptr = device_alloc(bytes, stream_);
    nb.cap = bytes;
    bufs_.push_back(nb);
    return nb.ptr;
}

void Workspace::release() {
    if (arena_) {
        bufs_.clear();
        arena_top_ = 0;
        return;
    }
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
    for (auto &b : bufs_) device_free(b.ptr);
    bufs_.clear();
    if (stream_) return;  // host scratch stays until the destructor
    if (host_) (void)hipHostFree(host_);
    host_ = nullptr;
    host_cap_ = 0;
}

size_t Workspace::bytes() const {
    if (arena_) return arena_top_;
    size_t t = 0;
    for (auto &b : bufs_) t += b.cap;
    return t;
}

int64_t *Workspace::host(int n) {
    if (arena_) {
        if (n > host_cap_) throw Error{BT_ENOMEM, "host scratch of the arena too small"};
        return host_;
    }
    if (n > host_cap_) {
        if (host_) {
            if (stream_)
                old_host_.push_back(host_);
            else
                (void)hipHostFree(host_);
        }
        host_ = nullptr;
        host_cap_ = 0;
        const int cap = n > 4096 ? n : 4096;
        BT_HIP(hipHostMalloc((void **)&host_, sizeof(int64_t) * cap, hipHostMallocDefault));
        host_cap_ = cap;
    }
    return host_;
}

int grid_for(int64_t n, int block, int max_blocks) {
    int64_t g = ceil_div(n, block);
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

// ------------------------------------------------------------ fills

template <typename T> __global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<int32_t><<<grid_for(n, 256, 8192), 256, 0, s>>>(p, v, n);
    BT_CHECK_LAUNCH();
}
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<int64_t><<<grid_for(n, 256, 8192), 256, 0, s>>>(p, v, n);
    BT_CHECK_LAUNCH();
}
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<uint32_t><<<grid_for(n, 256, 8192), 256, 0, s>>>(p, v, n);
    BT_CHECK_LAUNCH();
}

// Clearing by a kernel rather than hipMemsetAsync: a caller may capture the
// library's work in a HIP graph, where memset nodes are avoided.
void zero_bytes(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(p) % 4 != 0)
        throw Error{BT_EDEVICE, "zero_bytes: size or address not a multiple of 4"};
    fill_u32(static_cast<uint32_t *>(p), 0u, (int64_t)(bytes / 4), s);
}

// ------------------------------------------------------------ scan
// Reduce-then-scan: per-tile sums, a recursive scan of those, then a
// per-tile scan seeded with the tile's offset.  Each thread owns
// kScanItems consecutive elements.

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

template <typename Tin>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const Tin *in, int64_t n,
                                                            int64_t *bsum) {
    __shared__ int64_t part[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        int64_t idx = base + i;
        if (idx < n) s += (int64_t)in[idx];
    }
    s = wave_sum(s);
    if (lane_id() == 0) part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) t += part[w];
        bsum[blockIdx.x] = t;
    }
}

template <typename Tin>
__global__ __launch_bounds__(kScanBlock) void k_scan_tile(const Tin *in, int64_t *out,
                                                          int64_t n, const int64_t *boff) {
    __shared__ int64_t scratch[kScanBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? (int64_t)in[idx] : 0;
        sum += v[i];
    }
    int64_t total;
    int64_t run = block_exclusive_sum(sum, scratch, &total);
    if (boff) run += boff[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
        if (idx == n - 1) out[n] = run;
    }
}

template <typename Tin>
static void scan_impl(const Tin *in, int64_t *out, int64_t n, Workspace &ws, hipStream_t s,
                      int level) {
    if (n <= 0) {
        fill_i64(out, 0, 1, s);
        return;
    }
    int64_t nb = ceil_div(n, kScanTile);
    if (nb == 1) {
        k_scan_tile<Tin><<<1, kScanBlock, 0, s>>>(in, out, n, nullptr);
        BT_CHECK_LAUNCH();
        return;
    }
    char nb_name[32], no_name[32];
    snprintf(nb_name, sizeof nb_name, "scan_bsum%d", level);
    snprintf(no_name, sizeof no_name, "scan_boff%d", level);
    int64_t *bsum = ws.get<int64_t>(nb_name, nb);
    int64_t *boff = ws.get<int64_t>(no_name, nb + 1);
    k_scan_reduce<Tin><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, bsum);
    BT_CHECK_LAUNCH();
    scan_impl<int64_t>(bsum, boff, nb, ws, s, level + 1);
    k_scan_tile<Tin><<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, n, boff);
    BT_CHECK_LAUNCH();
}

void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, Workspace &ws,
                        hipStream_t s) {
    scan_impl<int64_t>(in, out, n, ws, s, 0);
}

void scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, Workspace &ws,
                               hipStream_t s) {
    scan_impl<int32_t>(in, out, n, ws, s, 0);
}

// ------------------------------------------------------- radix sort
// Stable LSD radix sort, 8-bit digits.  Pass: per-tile digit histograms
// (digit-major), one exclusive scan over them, then a stable scatter in
// which each wave ranks equal digits with eight ballots and waves are
// ordered through LDS counters, one row of kRsBlock elements at a time.

constexpr int kRsBlock = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsBlock * kRsItems;
constexpr int kRsWaves = kRsBlock / kWave;

__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const uint64_t *keys, int64_t n,
                                                      int shift, int32_t *hist, int64_t nb) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int i = threadIdx.x; i < kRsTile; i += kRsBlock) {
        int64_t idx = base + i;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const uint64_t *kin,
                                                         const uint32_t *vin, uint64_t *kout,
                                                         uint32_t *vout, int64_t n, int shift,
                                                         const int64_t *offs, int64_t nb) {
    __shared__ int64_t run[256];
    __shared__ int32_t wc[kRsWaves][256];
    const int w = threadIdx.x / kWave;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    for (int i = 0; i < kRsWaves; ++i) wc[i][threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t idx = base + (int64_t)r * kRsBlock + threadIdx.x;
        const bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0;
        uint32_t val = valid ? vin[idx] : 0;
        const int d = (int)((key >> shift) & 255);
        const uint64_t vmask = __ballot(valid);
        uint64_t peers = vmask;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        peers &= vmask;
        const int rank = (int)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wc[w][d] = (int)__popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t pos = run[d] + rank;
            for (int i = 0; i < w; ++i) pos += wc[i][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int64_t add = 0;
        for (int i = 0; i < kRsWaves; ++i) {
            add += wc[i][threadIdx.x];
            wc[i][threadIdx.x] = 0;
        }
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

void radix_sort_u64_u32(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits,
                        Workspace &ws, hipStream_t s) {
    if (n <= 1 || key_bits <= 0) return;
    const int64_t nb = ceil_div(n, kRsTile);
    uint64_t *k2 = ws.get<uint64_t>("rs_keys", n);
    uint32_t *v2 = ws.get<uint32_t>("rs_vals", n);
    int32_t *hist = ws.get<int32_t>("rs_hist", 256 * nb);
    int64_t *offs = ws.get<int64_t>("rs_offs", 256 * nb + 1);
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    const int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_rs_hist<<<(unsigned)nb, kRsBlock, 0, s>>>(ka, n, shift, hist, nb);
        BT_CHECK_LAUNCH();
        scan_exclusive_i32_to_i64(hist, offs, 256 * nb, ws, s);
        k_rs_scatter<<<(unsigned)nb, kRsBlock, 0, s>>>(ka, va, kb, vb, n, shift, offs, nb);
        BT_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        BT_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        BT_HIP(hipMemcpyAsync(vals, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace bt
