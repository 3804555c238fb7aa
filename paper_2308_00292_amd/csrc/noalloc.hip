// dmk_eval_noalloc: dmk_eval with the eval workspace taken from a static
// device array instead of plan-owned memory, for callers that cannot
// allocate device memory at call time.
//
// The array lives for the whole process, one copy per device (each device
// that runs the library holds DMK_NOALLOC_MAX_BYTES).  Host code never uses
// the array's name as an address: its device address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch_dev.  Every call on
// a device shares the array, so calls that overlap in time on one device
// race; the array keeps the previous call's contents, and the eval writes
// every workspace element before reading it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "dmk_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[DMK_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// device address of this device's copy of `scratch` (current device)
void *scratch_base()
{
    int dev = 0;
    DMK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw dmk::Error{DMK_ERR_STATE, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        DMK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw dmk::Error{DMK_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array"};
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}

// Points the plan's workspace fields into the scratch array for one call
// and puts them back afterwards; graph replay and stage timing are off for
// the call (the captured graph holds the plan-owned addresses, and timing
// creates events).
struct ScratchWorkspace {
    dmk::Plan *P;
    std::vector<dmk::WsItem> items;
    std::vector<void *> saved;
    uint64_t flags;
    bool timing;
    ScratchWorkspace(dmk::Plan *p, unsigned char *base) : P(p), flags(p->flags), timing(p->timing)
    {
        dmk::workspace_layout(P, items);
        size_t off = 0;
        for (const dmk::WsItem &it : items) off += (it.bytes + 255) / 256 * 256;
        if (off > (size_t)DMK_NOALLOC_MAX_BYTES)
            throw dmk::Error{DMK_ERR_ARG, "the plan's eval workspace (" + std::to_string(off) +
                                              " bytes) exceeds the static scratch of " +
                                              std::to_string((long long)DMK_NOALLOC_MAX_BYTES) + " bytes"};
        off = 0;
        for (const dmk::WsItem &it : items) {
            saved.push_back(*it.ptr);
            *it.ptr = base + off;
            off += (it.bytes + 255) / 256 * 256;
        }
        P->flags &= ~(uint64_t)DMK_FLAG_BATCHED;
        P->timing = false;
    }
    ~ScratchWorkspace()
    {
        for (size_t i = 0; i < saved.size(); ++i) *items[i].ptr = saved[i];
        P->flags = flags;
        P->timing = timing;
    }
};

}  // namespace

using namespace dmk;

extern "C" dmk_status dmk_eval_noalloc(dmk_plan_t plan, const double *charges, double *pot, void *stream)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (P->is_vol) throw Error{DMK_ERR_ARG, "volume plans are evaluated with dmk_vol_eval"};
        if ((P->nsrc > 0 && !charges) || (P->ntgt > 0 && !pot)) throw Error{DMK_ERR_ARG, "charges or pot is NULL"};
        unsigned char *base = (unsigned char *)scratch_base();
        BusyGuard g(P);
        hipStream_t s = (hipStream_t)stream;
        begin_eval(P, s);
        {
            ScratchWorkspace ws(P, base);
            run_eval(P, charges, pot, nullptr, nullptr, s);
        }
        end_eval(P, s);
    });
}
