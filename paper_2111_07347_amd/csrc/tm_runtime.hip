// Error reporting, device presence and version for libtm.
#include <cstdio>
#include <mutex>

#include "tm_internal.h"

namespace tmlib {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
}

void clear_error() { g_error.clear(); }

int hip_fail(hipError_t e, const char* what) {
    set_error("%s failed: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
    return TM_EHIP;
}

int require_device() {
    static std::once_flag once;
    static int count = 0;
    std::call_once(once, [] {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
        count = n;
    });
    if (count <= 0) {
        set_error("no HIP device available");
        return TM_ENODEV;
    }
    // Scratch comes from the stream-ordered allocator; keep freed blocks in
    // the device's default pool instead of returning them to the driver at
    // every synchronisation, so repeated calls reuse them (once per device).
    static std::mutex mu;
    static std::vector<char> pool_set;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0) {
        std::lock_guard<std::mutex> lock(mu);
        if (pool_set.size() <= static_cast<size_t>(dev)) pool_set.resize(dev + 1, 0);
        if (!pool_set[dev]) {
            pool_set[dev] = 1;
            hipMemPool_t pool;
            if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t keep = UINT64_MAX;
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            }
        }
    }
    return TM_OK;
}

}  // namespace tmlib

extern "C" const char* tm_last_error(void) { return tmlib::g_error.c_str(); }

extern "C" const char* tm_version(void) { return "tm 0.1.0 gfx950"; }
