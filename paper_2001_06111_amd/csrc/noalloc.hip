// noalloc.hip - bt_support_noalloc: butterfly supports with no device
// allocation, for callers that cannot allocate.
//
// All scratch memory of the call lives in `scratch`, a file-scope device
// array of kScratchBytes that each GPU the library runs on holds until the
// process ends.  In host code the array's name is only a host-side stand-in,
// so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and that address is what
// the kernels receive.  Calls on one device take turns on a per-device lock
// and each call starts by forgetting the previous call's buffers; every
// buffer that must start at zero is cleared by a kernel.
#include <mutex>

#include "pipeline.h"

static constexpr size_t kScratchBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace bt {
namespace {

constexpr int64_t kMaxEdges = int64_t(1) << 18;
constexpr int64_t kMaxVertices = int64_t(1) << 18;
constexpr int kMaxDevices = 64;
constexpr int kHostWords = 64;

struct DeviceScratch {
    std::mutex mu;
    void *ptr = nullptr;  // device address of `scratch` on this device
    int64_t host[kHostWords];
    Workspace ws;
};

DeviceScratch &device_scratch(int dev) {
    static DeviceScratch *table = new DeviceScratch[kMaxDevices];  // lives until exit
    return table[dev];
}

}  // namespace
}  // namespace bt

using namespace bt;

extern "C" bt_status bt_support_noalloc(const bt_csr *g, int64_t *sup_out,
                                        int64_t *butterflies_out, hipStream_t stream) {
    try {
        check_graph(g);
        if (g->m > 0 && !sup_out) throw Error{BT_EINVAL, "sup_out is NULL"};
        if (g->m > kMaxEdges || (int64_t)g->n_upper + g->n_lower > kMaxVertices)
            throw Error{BT_EOVERFLOW, "bt_support_noalloc takes at most " +
                                          std::to_string(kMaxEdges) + " edges and " +
                                          std::to_string(kMaxVertices) + " vertices"};
        int dev = 0;
        BT_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices) throw Error{BT_EDEVICE, "device index out of range"};
        DeviceScratch &D = device_scratch(dev);
        std::lock_guard<std::mutex> lk(D.mu);
        if (!D.ptr) {
            void *p = nullptr;
            BT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) throw Error{BT_EDEVICE, "no device address for the static scratch"};
            D.ptr = p;
        }
        Workspace &ws = D.ws;
        ws.use_arena(D.ptr, kScratchBytes, D.host, kHostWords);
        RankCSR r;
        prepare(*g, r, ws, stream);
        TaskLists t;
        make_tasks(r, t, ws, stream);
        uint64_t *supl = ws.get<uint64_t>("sup_supl", g->m + 1);
        int64_t *bf = ws.get<int64_t>("sup_bf", 2);
        zero_bytes(supl, sizeof(uint64_t) * (g->m + 1), stream);
        zero_bytes(bf, sizeof(int64_t) * 2, stream);
        count_support(r, t, supl, bf, stream);
        check_butterfly_total(supl, g->m, bf, ws, stream);
        supl_to_sup(supl, sup_out, g->m, stream);
        int64_t *hs = ws.host(2);
        BT_HIP(hipMemcpyAsync(hs, bf, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        BT_HIP(hipStreamSynchronize(stream));
        if (butterflies_out) *butterflies_out = hs[0];
        return BT_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::exception &e) {
        set_error(e.what());
        return BT_EDEVICE;
    }
}
