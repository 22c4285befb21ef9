// Fixed-point spreading for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops): the workspace of
// ot_spread is a file-scope device array instead of a caller buffer or a
// stream-ordered allocation.
//
// Host code never uses the array's name as an address: the name is a
// host-side stand-in.  The first call on a device, with that device current,
// asks the runtime for the array's device address (each device holds its
// own copy) and keeps it; every later call on that device passes that
// address to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ot_common.h"

extern "C" int ot_spread(const ot_tree *t, const void *force, const void *pos, const int32_t *ids, int32_t dtype,
                         int64_t n, int32_t mode, int32_t accumulate, void *field_out, void *work, void *stream);

namespace {

constexpr int64_t kScratchBytes = ot::kFxHeader + (int64_t)OT_NOALLOC_MAX_LEAVES * 3 * 8;
static_assert(kScratchBytes == 256 + 24 * (int64_t)OT_NOALLOC_MAX_LEAVES, "workspace layout of ot_spread");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices];   // device address of `scratch` on each device (null: not asked yet)

// Address of this device's copy of the array; null with the error recorded.
void *scratch_on(int dev)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            ot::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_addr[dev] = p;
    }
    return g_addr[dev];
}

}  // namespace

extern "C" int ot_spread_noalloc(const ot_tree *t, const void *force, const void *pos, const int32_t *ids,
                                 int32_t dtype, int64_t n, int32_t mode, int32_t accumulate, void *field_out,
                                 void *stream)
{
    if (!t) return ot::fail(OT_ERR_INVALID, "tree is NULL");
    if (mode != OT_SPREAD_FIXED) {
        // ATOMIC spreading needs no workspace: the plain call allocates nothing
        return ot_spread(t, force, pos, ids, dtype, n, mode, accumulate, field_out, nullptr, stream);
    }
    if (t->n_leaves > (int64_t)OT_NOALLOC_MAX_LEAVES)
        return ot::fail(OT_ERR_CAPACITY, "ot_spread_noalloc: the tree has more leaves than the static workspace "
                                         "holds (OT_NOALLOC_MAX_LEAVES)");
    int dev = 0;
    OT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return ot::fail(OT_ERR_INVALID, "ot_spread_noalloc: device index too large");
    if (dev != t->device) return ot::fail(OT_ERR_INVALID, "ot_spread_noalloc: the tree lives on another device");
    void *work = scratch_on(dev);
    if (!work) return OT_ERR_HIP;
    return ot_spread(t, force, pos, ids, dtype, n, mode, accumulate, field_out, work, stream);
}
