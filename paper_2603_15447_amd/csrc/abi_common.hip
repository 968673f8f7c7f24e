// Status codes, thread-local error text and device queries of the C ABI.
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace bzi {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(BZ_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
}

}  // namespace bzi

extern "C" {

int bz_version(void) { return 10000; }

const char *bz_status_string(int code) {
    switch (code) {
        case BZ_OK: return "ok";
        case BZ_ERR_NULL: return "null pointer";
        case BZ_ERR_SHAPE: return "shape out of range";
        case BZ_ERR_DTYPE: return "unknown dtype";
        case BZ_ERR_UNSUPPORTED: return "unsupported combination";
        case BZ_ERR_ALIGN: return "misaligned pointer";
        case BZ_ERR_HIP: return "HIP runtime error";
        case BZ_ERR_NOMEM: return "out of device memory";
        case BZ_ERR_INTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char *bz_last_error(void) { return bzi::g_err; }

int bz_device_cu_count(void) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // extern "C"
