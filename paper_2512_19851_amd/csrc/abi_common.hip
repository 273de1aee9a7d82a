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

size_t sten_workspace_bytes(int op, int64_t H, int64_t W, int32_t T) {
    constexpr int64_t kMaxSide = (int64_t)1 << 30;
    if (H < 0 || W < 0 || T < 0 || H > kMaxSide || W > kMaxSide) return STEN_WORKSPACE_INVALID;
    const bool interior = H >= 3 && W >= 3;
    const size_t points = (size_t)H * (size_t)W;  // below 2^60: no overflow
    switch (op) {
        case STEN_OP_F64: return (interior && T >= 2) ? points * sizeof(double) : 0;
        case STEN_OP_F32:
        case STEN_OP_ADJ: return (interior && T >= 2) ? points * sizeof(float) : 0;
        case STEN_OP_HILO: return (H == 0 || W == 0) ? 0 : sten_jacobi5_f64_hilo_work_bytes(H, W);
        case STEN_OP_BATCH:
            return H > INT32_MAX ? STEN_WORKSPACE_INVALID : sten_batch_workspace_bytes((int32_t)H);
        case STEN_OP_STATES: {
            if (points == 0) return 0;
            const size_t grids = (size_t)T + 1;
            const size_t per = points * sizeof(float);
            if (per > SIZE_MAX / grids) return STEN_WORKSPACE_INVALID;
            return per * grids;
        }
        default: return STEN_WORKSPACE_INVALID;
    }
}

uint32_t sten_xcd_tile_of_block(uint32_t b, uint32_t nb) { return sten::xcd_tile_of_block(b, nb); }

const char* sten_version(void) { return "libsten 0.1 (gfx950)"; }

}  // extern "C"
