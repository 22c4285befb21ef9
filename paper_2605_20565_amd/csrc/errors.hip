// Error codes and the per-thread last-error message of the C ABI.
#include <hip/hip_runtime.h>

#include <string>

#include "ot_common.h"

namespace ot {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return OT_ERR_HIP;
}

}  // namespace ot

extern "C" const char *ot_strerror(int32_t code)
{
    switch (code) {
    case OT_OK: return "success";
    case OT_ERR_INVALID: return "invalid argument";
    case OT_ERR_NOT_PARTITION: return "leaves do not tile the unit cube";
    case OT_ERR_UNSORTED_DUP: return "duplicate Morton key";
    case OT_ERR_LEVEL_RANGE: return "level out of range";
    case OT_ERR_OOM: return "out of device memory";
    case OT_ERR_HIP: return "HIP runtime error";
    case OT_ERR_CAPACITY: return "capacity exceeded";
    default: return "unknown error";
    }
}

extern "C" const char *ot_last_error(void) { return ot::g_last_error.c_str(); }
