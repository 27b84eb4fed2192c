// tm_match_batch_static: tm_match_batch for callers that cannot allocate
// device memory (work captured into HIP graphs, tight serving loops). The
// pre-filter's scratch (kept lists and the score matrix) lives in one
// file-scope device array per GPU instead of the stream-ordered allocator.
//
// The array's name is a host-side stand-in in host code; its device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels.
#include <mutex>
#include <vector>

#include "tm_internal.h"

namespace {

constexpr size_t kStaticScratchBytes = TM_STATIC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
std::vector<void*> g_ptr;   // per device: device address of `scratch`, or null

// Device address of this GPU's scratch array (looked up on first use).
int scratch_for_current_device(void** out) {
    *out = nullptr;
    int dev = 0;
    TM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr.size() <= static_cast<size_t>(dev)) g_ptr.resize(dev + 1, nullptr);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        TM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            tmlib::set_error("hipGetSymbolAddress returned a null address for the static scratch");
            return TM_EHIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TM_OK;
}

}  // namespace

extern "C" int tm_match_batch_static(const tm_library* lib, const float* polar,
                                     const double* norms, const float* profiles, int32_t B,
                                     const tm_match_opts* opts, int32_t N,
                                     int32_t* top_template, int32_t* top_angle, float* top_score,
                                     float* best_score, int16_t* best_angle, void* hip_stream) {
    tmlib::clear_error();
    if (int r = tmlib::require_device()) return r;
    void* p = nullptr;
    if (int r = scratch_for_current_device(&p)) return r;
    return tmlib::match_batch_impl(lib, polar, norms, profiles, B, opts, N, top_template,
                                   top_angle, top_score, best_score, best_angle, hip_stream, p,
                                   kStaticScratchBytes);
}
