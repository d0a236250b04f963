// common.h - shared host/device helpers of the bitruss library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/bt.h"

namespace bt {

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);

struct Error {
    bt_status status;
    std::string msg;
};

#define BT_HIP(call)                                                           \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            throw ::bt::Error{BT_EDEVICE, std::string(#call) + ": " +          \
                                              hipGetErrorString(e_)};          \
    } while (0)

#define BT_CHECK_LAUNCH() BT_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int bits_for(uint64_t v) {  // bits needed to store values in [0, v]
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// ---------------------------------------------------------- device memory

// A named set of device buffers that grow on demand and are kept between
// calls.  Buffers are 256-byte aligned.  Not thread-safe: owners lock.
// Also owns pinned host scratch for small device-to-host reads and the
// peel's captured round graphs, so independent workspaces can serve
// concurrent calls on different streams.
class Workspace {
public:
    ~Workspace();
    // Binds the workspace to the one stream that uses its buffers: they are
    // then allocated and freed in stream order (hipMallocAsync and
    // hipFreeAsync on s), since hipFree and hipHostFree wait for every
    // stream of the device, including a long peel of another caller.  Host
    // scratch is then freed only by the destructor.  Call before any get().
    void bind_stream(hipStream_t s) { stream_ = s; }
    // Frees everything, host scratch included, and unbinds; call before the
    // bound stream is destroyed.
    void close();
    void *get(const char *name, size_t bytes);
    template <typename T> T *get(const char *name, int64_t count) {
        return static_cast<T *>(get(name, (size_t)(count > 0 ? count : 1) * sizeof(T)));
    }
    int64_t *host(int n);  // pinned, at least n int64; valid until a larger request
    void release();
    size_t bytes() const;
    // Arena mode: buffers are carved from [base, base + cap), device memory
    // the caller owns, and host scratch is `host` (n_host int64); nothing is
    // allocated, and a request that does not fit throws BT_ENOMEM.  Every
    // buffer is forgotten by release(), which a call in this mode makes
    // first.
    void use_arena(void *base, size_t cap, int64_t *host, int n_host);

    struct GraphEntry {
        std::vector<unsigned char> key;
        int rounds;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    bool coop = true;  // peel with the cooperative persistent kernel

private:
    struct Buf {
        std::string name;
        void *ptr = nullptr;
        size_t cap = 0;
    };
    std::vector<Buf> bufs_;
    int64_t *host_ = nullptr;
    int host_cap_ = 0;
    hipStream_t stream_ = nullptr;
    std::vector<int64_t *> old_host_;  // outgrown host scratch of a bound workspace
    char *arena_ = nullptr;
    size_t arena_cap_ = 0, arena_top_ = 0;
};

// Throws BT_ENOMEM with the size.  With a stream, the block is allocated
// (and later freed) in that stream's order; a hook's block is then handed
// back after that stream alone has drained, not the whole device.
void *device_alloc(size_t bytes, hipStream_t stream = nullptr);
void device_free(void *p);
void set_allocator(bt_alloc_fn a, bt_free_fn f, void *ctx);


// ------------------------------------------------------ wave primitives

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;
}

template <typename T> __device__ __forceinline__ T wave_inclusive_sum(T v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T t = __shfl_up(v, d, kWave);
        if (lane_id() >= d) v += t;
    }
    return v;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <typename T> __device__ __forceinline__ T wave_or(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v |= __shfl_xor(v, d, kWave);
    return v;
}

template <typename T> __device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, kWave);
        v = o < v ? o : v;
    }
    return v;
}

// Block-wide exclusive sum; `scratch` holds one T per wave.  Returns the
// thread's exclusive prefix and writes the block total to *total.
template <typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T *scratch, T *total) {
    const int nw = blockDim.x / kWave;
    const int w = threadIdx.x / kWave;
    T inc = wave_inclusive_sum(v);
    if (lane_id() == kWave - 1) scratch[w] = inc;
    __syncthreads();
    const int t = (int)threadIdx.x;
    if (t < kWave) {
        T s = t < nw ? scratch[t] : T(0);
        T si = wave_inclusive_sum(s);
        if (t < nw) scratch[t] = si - s;
        if (t == nw - 1) scratch[nw] = si;
    }
    __syncthreads();
    T r = scratch[w] + inc - v;
    *total = scratch[nw];
    __syncthreads();
    return r;
}

// Push `pred`-selected values to a global list with one atomic per wave.
template <typename T>
__device__ __forceinline__ void wave_push(bool pred, T val, T *list, int32_t *count) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(count, (int)__popcll(mask));
    base = __shfl(base, leader, kWave);
    if (pred) list[base + __popcll(mask & lanemask_lt())] = val;
}

// ------------------------------------------------- host-side primitives
// (prims.hip) All enqueue on `s`; sizes are host values.

// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, Workspace &ws,
                        hipStream_t s);
void scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, Workspace &ws,
                               hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `key_bits` bits.
// Sorted data ends in keys/vals (buffers are ping-ponged with ws scratch).
void radix_sort_u64_u32(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits,
                        Workspace &ws, hipStream_t s);

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Sets `bytes` (a multiple of 4, at a 4-byte aligned address) to zero.
void zero_bytes(void *p, size_t bytes, hipStream_t s);

int grid_for(int64_t n, int block, int max_blocks = 1 << 20);

}  // namespace bt
