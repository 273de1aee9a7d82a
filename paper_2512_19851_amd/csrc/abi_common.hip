// Status strings, HIP error capture and argument validation shared by every
// entry point of libsten.
#include "common.hpp"

namespace sten {

static thread_local int g_last_hip_error = 0;

sten_status hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    return STEN_ERR_HIP;
}

sten_status check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    return STEN_OK;
}

bool is_device_ptr(const void* p) {
    if (p == nullptr) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave a sticky error for the caller
        return false;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return false;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.device == dev;
}

sten_status check_grid_args(const void* u0, const void* out, const void* work, bool need_work,
                            int64_t H, int64_t W, int64_t ld, int32_t T, size_t esize) {
    if (H < 0 || W < 0 || T < 0) return STEN_ERR_ARG;
    if (H > 0 && ld < W) return STEN_ERR_ARG;
    if (H > INT32_MAX - 2 || W > INT32_MAX - 2) return STEN_ERR_ARG;
    if (H == 0 || W == 0) return STEN_OK;
    if (u0 == nullptr || out == nullptr) return STEN_ERR_PTR;
    if (need_work && work == nullptr) return STEN_ERR_PTR;
    size_t n = span_bytes(H, W, ld, esize);
    if (overlaps(u0, n, out, n)) return STEN_ERR_ALIAS;
    if (need_work && (overlaps(u0, n, work, n) || overlaps(out, n, work, n))) return STEN_ERR_ALIAS;
    if (!is_device_ptr(u0) || !is_device_ptr(out)) return STEN_ERR_PTR;
    if (need_work && !is_device_ptr(work)) return STEN_ERR_PTR;
    return STEN_OK;
}

}  // namespace sten

extern "C" {

const char* sten_status_string(sten_status s) {
    switch (s) {
        case STEN_OK: return "STEN_OK";
        case STEN_ERR_ARG: return "STEN_ERR_ARG: invalid size, stride or count";
        case STEN_ERR_ALIAS: return "STEN_ERR_ALIAS: buffers of the call overlap";
        case STEN_ERR_PTR: return "STEN_ERR_PTR: pointer is NULL or not device memory of the current device";
        case STEN_ERR_WORKSPACE: return "STEN_ERR_WORKSPACE: workspace too small";
        case STEN_ERR_HIP: return "STEN_ERR_HIP: a HIP call failed";
        case STEN_ERR_UNSUPPORTED: return "STEN_ERR_UNSUPPORTED: request not handled by this build";
    }
    return "unknown sten_status";
}

int sten_last_hip_error(void) { return sten::g_last_hip_error; }

uint32_t sten_xcd_tile_of_block(uint32_t b, uint32_t nb) { return sten::xcd_tile_of_block(b, nb); }

const char* sten_version(void) { return "libsten 0.1 (gfx950)"; }

}  // extern "C"
